"""Triangular 6.6.6 colour code of odd distance d (paper, Sec. II.A).

Construction used here: the honeycomb lattice is the triangular lattice with
one of its three sqrt(3) x sqrt(3) sublattices removed; the removed points are
the hexagon (plaquette) centres and the remaining points are the vertices
(qubits).  Take the triangular-lattice points (i, j) with i, j >= 0 and
i + j <= K, K = 3(d-1)/2.  Points with (i + 2j) mod 3 == 1 are plaquette
centres; every other point is a qubit.  A plaquette holds the qubits among its
six lattice neighbours that lie in the region: six in the bulk, four on the
boundary.  The three region corners have residue 0, so they are qubits.

Counting facts this reproduces (paper Sec. II.A gives the first two):
  n = (3 d^2 + 1) / 4 qubits, (n - 1) / 2 plaquettes, k = 1,
  (3d - 3)/2 weight-4 plaquettes, nnz(H) = 3n - 3d.

The CNOT slot of a qubit inside a plaquette is the index of its lattice offset
from the plaquette centre; the three plaquettes that share a qubit see it in
three distinct slots, so one CNOT layer per slot never touches a qubit twice.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Offsets from a plaquette centre to its six neighbours, in angular order.
SLOT_OFFSETS = ((1, 0), (0, 1), (-1, 1), (-1, 0), (0, -1), (1, -1))


@dataclass(frozen=True)
class ColourCode:
    d: int
    n: int
    # plaquettes[p] = list of (qubit, slot) pairs, qubits ascending
    plaquettes: tuple
    qubit_coords: tuple  # lattice coordinates of each qubit
    plaquette_coords: tuple
    plaquette_colour: tuple  # 0, 1, 2

    @property
    def num_plaquettes(self) -> int:
        return len(self.plaquettes)

    def check_matrix(self) -> np.ndarray:
        """Face-vertex incidence matrix, shape (plaquettes, n), uint8."""
        h = np.zeros((self.num_plaquettes, self.n), dtype=np.uint8)
        for p, members in enumerate(self.plaquettes):
            for q, _slot in members:
                h[p, q] = 1
        return h


def triangular_666(d: int) -> ColourCode:
    if d < 3 or d % 2 == 0:
        raise ValueError("distance must be odd and >= 3")
    K = 3 * (d - 1) // 2
    points = [(i, j) for j in range(K + 1) for i in range(K + 1 - j)]
    inside = set(points)
    qubits = [pt for pt in points if (pt[0] + 2 * pt[1]) % 3 != 1]
    centres = [pt for pt in points if (pt[0] + 2 * pt[1]) % 3 == 1]
    qidx = {pt: k for k, pt in enumerate(qubits)}
    plaquettes = []
    colours = []
    for (ci, cj) in centres:
        members = []
        for slot, (di, dj) in enumerate(SLOT_OFFSETS):
            pt = (ci + di, cj + dj)
            if pt in inside:
                members.append((qidx[pt], slot))
        members.sort()
        plaquettes.append(tuple(members))
        colours.append((ci - cj) % 3)
    return ColourCode(
        d=d,
        n=len(qubits),
        plaquettes=tuple(plaquettes),
        qubit_coords=tuple(qubits),
        plaquette_coords=tuple(centres),
        plaquette_colour=tuple(colours),
    )
