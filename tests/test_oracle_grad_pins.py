"""Pins of the oracle's differentiable-decoder objective (or_bp_loss) and of
its finite-difference gradient (fd_grad), against brute force and closed
forms that do not go through the oracle's code.

The loss is a reading, not the paper's: the paper trains no decoder, and
the unrolled min-sum iteration (Algorithm 1 with one scaling factor per
iteration) is scored by the binary cross-entropy between the syndrome and
the probability that each check is violated when the bits are independent
with the final posteriors as LLRs.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from synth.dem import dem_from_dense


def _graph(H):
    H = np.asarray(H, np.uint8)
    return O.OracleGraph(dem_from_dense(H, np.full(H.shape[1], 0.1), np.ones((1, H.shape[1]), np.uint8)))


def _random_h(rng, m, n):
    """Random parity checks of degree 2..4 with every column used."""
    while True:
        H = np.zeros((m, n), np.uint8)
        for c in range(m):
            H[c, rng.choice(n, int(rng.integers(2, 5)), replace=False)] = 1
        if H.sum(0).min() > 0:
            return H


def _p1(L):
    """P(bit = 1) for LLR L = ln P(0)/P(1)."""
    return 1.0 / (1.0 + np.exp(L))


def _brute_violation(H, L):
    """shat_c = P(odd parity on N(c)) by enumerating every assignment of the
    check's bits, and d shat_c / d L_v for every v (0 off the check)."""
    m, n = H.shape
    p = _p1(L)
    sh = np.zeros(m)
    dsh = np.zeros((m, n))
    for c in range(m):
        nb = np.flatnonzero(H[c])
        for x in itertools.product((0, 1), repeat=len(nb)):
            if sum(x) % 2 == 0:
                continue
            pr = np.array([p[v] if xi else 1 - p[v] for v, xi in zip(nb, x)])
            sh[c] += pr.prod()
            for k, v in enumerate(nb):
                rest = np.prod(np.delete(pr, k))
                dp = -p[v] * (1 - p[v])  # d p_v / d L_v
                dsh[c, v] += rest * (dp if x[k] else -dp)
    return sh, dsh


def _brute_loss(H, s, L):
    sh, dsh = _brute_violation(H, L)
    loss = -np.sum(np.where(s == 1, np.log(sh), np.log(1 - sh)))
    dloss_dsh = np.where(s == 1, -1 / sh, 1 / (1 - sh))
    return loss, dloss_dsh @ dsh  # (loss, d loss / d L_v)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("schedule", ["serial", "parallel"])
def test_loss_with_zero_scaling_is_brute_force(seed, schedule):
    """With every alpha_t = 0 the check messages vanish and the posteriors
    are the channel LLRs, so the loss is the cross-entropy of the syndrome
    against the exact violation probabilities of independent bits.  Breaks
    on a wrong tanh identity (sign, factor 1/2), a swapped BCE orientation or
    a dropped check."""
    rng = np.random.default_rng(seed)
    m, n = 4, 8
    H = _random_h(rng, m, n)
    lam = rng.uniform(-3, 5, n)
    s = rng.integers(0, 2, m).astype(np.uint8)
    g = _graph(H)
    perm = rng.permutation(n).astype(np.uint32) if schedule == "serial" else None
    loss, _, post = O.bp_loss(g, s, lam, np.zeros(3), 3, perm)
    np.testing.assert_array_equal(post, lam)
    want, _ = _brute_loss(H, s, lam)
    assert abs(loss - want) <= 1e-12 * max(1.0, abs(want))


@pytest.mark.parametrize("seed", range(3))
def test_fd_gradient_at_zero_scaling(seed):
    """K = 2, alpha = (0, 0), serial.  Then L_v = lambda_v, so d loss / d
    lambda_v is the brute-force derivative; alpha_1 acts only through the
    iteration-2 messages, which alpha_2 = 0 switches off, so its derivative
    is 0; and d L_v / d alpha_2 = sum over v's checks of the min-sum check
    message computed from messages that all equal lambda.  Breaks on a
    wrong difference quotient (sign, 2h), on swapped iteration indices of
    alpha, or on a check message without the syndrome sign."""
    rng = np.random.default_rng(10 + seed)
    m, n = 4, 8
    H = _random_h(rng, m, n)
    lam = rng.uniform(-3, 5, n)
    s = rng.integers(0, 2, m).astype(np.uint8)
    g = _graph(H)
    perm = rng.permutation(n).astype(np.uint32)
    dl, _, da, _ = O.fd_grad(g, s, lam, np.zeros(2), 2, perm)
    _, dloss_dL = _brute_loss(H, s, lam)
    np.testing.assert_allclose(dl, dloss_dL, rtol=1e-6, atol=1e-8)
    q = np.zeros(n)
    for v in range(n):
        for c in np.flatnonzero(H[:, v]):
            others = [u for u in np.flatnonzero(H[c]) if u != v]
            sign = (-1.0) ** (int(s[c]) + sum(lam[u] < 0 for u in others))
            q[v] += sign * min(abs(lam[u]) for u in others)
    assert abs(da[0]) <= 1e-8
    assert abs(da[1] - dloss_dL @ q) <= 1e-6 * max(1.0, abs(da[1]))


@pytest.mark.parametrize("s", [0, 1])
def test_fd_gradient_two_bit_check(s):
    """One check on two bits, K = 1, serial order (0, 1): bit 0 sees
    (1 - 2s) lambda_1 and bit 1 then sees (1 - 2s) times bit 0's new
    variable message, which is lambda_0 (bit 0 has no other check).  So
    L_0 = lambda_0 + a (1 - 2s) lambda_1 and L_1 = lambda_1 + a (1 - 2s)
    lambda_0, and the chain rule gives the gradient by hand."""
    H = np.array([[1, 1]], np.uint8)
    lam = np.array([1.3, -0.4])
    a = 0.7
    sg = 1 - 2 * s
    L = np.array([lam[0] + a * sg * lam[1], lam[1] + a * sg * lam[0]])
    _, gL = _brute_loss(H, np.array([s], np.uint8), L)
    g = _graph(H)
    loss, _, post = O.bp_loss(g, np.array([s], np.uint8), lam, np.array([a]), 1, np.array([0, 1], np.uint32))
    np.testing.assert_allclose(post, L, rtol=0, atol=1e-15)
    dl, okl, da, oka = O.fd_grad(g, np.array([s], np.uint8), lam, np.array([a]), 1, np.array([0, 1], np.uint32))
    assert okl.all() and oka.all()
    np.testing.assert_allclose(dl, [gL[0] + gL[1] * a * sg, gL[1] + gL[0] * a * sg], rtol=1e-7)
    np.testing.assert_allclose(da, [gL[0] * sg * lam[1] + gL[1] * sg * lam[0]], rtol=1e-7)


def test_fd_smoothness_flags_mark_ties():
    """Three bits on one check with equal LLRs: every check message is a
    minimum over a tie, so moving any lambda_v switches an argmin and the
    flag must be False; with distinct LLRs nothing switches and every flag
    must be True."""
    H = np.array([[1, 1, 1]], np.uint8)
    g = _graph(H)
    perm = np.array([0, 1, 2], np.uint32)
    s = np.array([1], np.uint8)
    _, okl, _, oka = O.fd_grad(g, s, np.full(3, 2.0), np.array([0.6, 0.6]), 2, perm)
    assert not okl.any()
    _, okl, _, oka = O.fd_grad(g, s, np.array([2.0, 2.5, 3.1]), np.array([0.6, 0.6]), 2, perm)
    assert okl.all() and oka.all()
