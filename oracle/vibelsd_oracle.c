/*
 * Plain FP64 reference ("oracle") of the VibeLSD decode path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled and called by the test
 * suite, by the smoke check and by the CPU-baseline leg of the benchmark.
 * The product library never includes, links or calls it, and it shares no
 * code with the HIP path.
 *
 * It is written for readability, not speed: every check-to-variable message
 * is recomputed from its definition by scanning the whole check row.
 *
 * What it follows (paper = arXiv 2508.15743):
 *   - min-sum BP, parallel and serial-V schedules: Appendix A, Algorithm 1,
 *     with the syndrome sign (1 - 2 s_c) of syndrome-based decoding and a
 *     constant or per-iteration scaling factor alpha_t; the layered
 *     (check-serial) schedule that Sec. V names as future work;
 *   - the ensemble, correction limit M, candidate ranking by prior weight
 *     and the normalised LLR average: Sec. III.D.1-2 (offline / online);
 *   - LSD-0 post-processing: Sec. III.C (cluster growth guided by soft
 *     information, merging, per-cluster GF(2) solve), with the growth rule
 *     made precise as the synchronous one-column-per-invalid-cluster rule;
 *     higher LSD orders as the combination sweep of ordered statistics
 *     decoding on every cluster (osd_cs);
 *   - observables L_obs * e mod 2: Sec. II.B.
 * Readings of points the paper leaves open are listed in the design notes.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int m, n;
    const int *rp, *ri; /* CSR: check c -> columns ri[rp[c] .. rp[c+1]) ascending */
    const int *cp, *ci; /* CSC: column v -> checks ci[cp[v] .. cp[v+1]) ascending */
    const int *ce;      /* for CSC entry j, the CSR position of the same edge */
    uint64_t *sig;      /* if non-NULL: hash of every min-sum branch taken (argmin,
                           sign parity, clamps); constant while the loss is smooth */
} ograph;

/* sign convention: a message is "negative" iff it is < 0, so +0 and -0 both
   count as positive. */
static double clampd(double x, double lim) {
    if (x > lim) return lim;
    if (x < -lim) return -lim;
    return x;
}

/* Hard-decision syndrome check: H e == s ? */
static int syndrome_matches(const ograph *g, const uint8_t *e, const uint8_t *s) {
    for (int c = 0; c < g->m; c++) {
        int par = 0;
        for (int k = g->rp[c]; k < g->rp[c + 1]; k++) par ^= e[g->ri[k]];
        if (par != s[c]) return 0;
    }
    return 1;
}

static void sig_mix(uint64_t *h, uint64_t x) { *h = (*h ^ x) * 0x100000001b3ull + 0x9e3779b97f4a7c15ull; }

/* records in the signature that x is about to be clamped */
static double clamp_sig(double x, double lim, uint64_t *sig) {
    if (sig && (x > lim || x < -lim)) sig_mix(sig, 0xc1a3ull);
    return x;
}

/* clampd that also records (in *hit, if non-NULL) that the result reached
   the clamp: |result| >= lim, a message or posterior saturated at +-lim. */
static double clamp_hit(double x, double lim, int *hit) {
    double y = clampd(x, lim);
    if (hit && fabs(y) >= lim) *hit = 1;
    return y;
}

/* Check-to-variable message r_{c->v} from the current variable-to-check
   messages mu (indexed by CSR position), Algorithm 1's check update with the
   syndrome sign: (1 - 2 s_c) * alpha * prod sign * min |mu| over N(c)\v.
   A check with no other neighbour sends the clamp value with sign +. */
static double check_to_var(const ograph *g, const double *mu, const uint8_t *s, int c, int v,
                           double alpha, double lim) {
    double mag = INFINITY;
    int neg = 0, others = 0, am = -1;
    for (int k = g->rp[c]; k < g->rp[c + 1]; k++) {
        if (g->ri[k] == v) continue;
        others++;
        double a = fabs(mu[k]);
        if (a < mag) {
            mag = a;
            am = g->ri[k];
        }
        if (mu[k] < 0) neg ^= 1;
    }
    if (!others) mag = lim;
    if (g->sig) sig_mix(g->sig, ((uint64_t)(uint32_t)am << 1) | (uint64_t)neg);
    double r = alpha * (neg ? -mag : mag);
    return s[c] ? -r : r;
}

/*
 * One BP decoder (Algorithm 1).
 *   perm == NULL : parallel (flooding) schedule.
 *   perm != NULL : serial-V schedule; columns are updated in the order
 *                  perm[0..n-1], each one recomputing its incoming check
 *                  messages from the latest variable messages.
 * alpha[t-1] is the scaling factor of iteration t.  If stop_on_converge, the
 * decoder returns at the first iteration whose hard decision satisfies the
 * syndrome.  Outputs: *t_conv (iteration of convergence, or 0), ehat (the
 * decision of the last iteration run), post (the posteriors L_v of the last
 * iteration run), *iters (iterations run), *min_abs_post (smallest |L_v| of
 * any decision taken), trace (if non-NULL: posteriors of every iteration,
 * [T][n], rows past the last iteration run are left untouched).
 */
static int bp_core(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci, const int *ce,
                   const double *lam, const uint8_t *s, const uint32_t *perm, int T, const double *alpha,
                   double lim, int stop_on_converge, int *t_conv, uint8_t *ehat, double *post, int *iters,
                   double *min_abs_post, double *trace, uint64_t *sig, int *saturated) {
    ograph g = {m, n, rp, ri, cp, ci, ce, sig};
    int E = rp[m];
    double *mu = (double *)malloc(sizeof(double) * (E ? E : 1));
    double *rv = (double *)malloc(sizeof(double) * (E ? E : 1)); /* r by CSC position */
    if (!mu || !rv) {
        free(mu);
        free(rv);
        return -2;
    }
    /* initialisation: every variable-to-check message is the prior LLR */
    for (int c = 0; c < m; c++)
        for (int k = rp[c]; k < rp[c + 1]; k++) mu[k] = clampd(lam[ri[k]], lim);
    memset(ehat, 0, (size_t)n);
    for (int v = 0; v < n; v++) post[v] = clampd(lam[v], lim);
    *t_conv = 0;
    *iters = 0;
    double minabs = INFINITY;

    for (int t = 1; t <= T; t++) {
        double a = alpha[t - 1];
        if (perm) {
            for (int k = 0; k < n; k++) {
                int v = (int)perm[k];
                double lv = clampd(lam[v], lim);
                for (int j = cp[v]; j < cp[v + 1]; j++)
                    rv[j] = check_to_var(&g, mu, s, ci[j], v, a, lim);
                double L = lv;
                for (int j = cp[v]; j < cp[v + 1]; j++) L += rv[j];
                post[v] = clamp_hit(clamp_sig(L, lim, sig), lim, saturated);
                for (int j = cp[v]; j < cp[v + 1]; j++) {
                    double x = lv;
                    for (int j2 = cp[v]; j2 < cp[v + 1]; j2++)
                        if (j2 != j) x += rv[j2];
                    mu[ce[j]] = clamp_hit(clamp_sig(x, lim, sig), lim, saturated);
                }
            }
        } else {
            /* all check messages from the previous iteration's variable messages */
            for (int v = 0; v < n; v++)
                for (int j = cp[v]; j < cp[v + 1]; j++)
                    rv[j] = check_to_var(&g, mu, s, ci[j], v, a, lim);
            for (int v = 0; v < n; v++) {
                double lv = clampd(lam[v], lim);
                double L = lv;
                for (int j = cp[v]; j < cp[v + 1]; j++) L += rv[j];
                post[v] = clamp_hit(clamp_sig(L, lim, sig), lim, saturated);
                for (int j = cp[v]; j < cp[v + 1]; j++) {
                    double x = lv;
                    for (int j2 = cp[v]; j2 < cp[v + 1]; j2++)
                        if (j2 != j) x += rv[j2];
                    mu[ce[j]] = clamp_hit(clamp_sig(x, lim, sig), lim, saturated);
                }
            }
        }
        /* decision: e_v = 1 iff L_v <= 0 */
        for (int v = 0; v < n; v++) {
            ehat[v] = post[v] <= 0.0;
            double aa = fabs(post[v]);
            if (aa < minabs) minabs = aa;
        }
        if (trace) memcpy(trace + (size_t)(t - 1) * n, post, sizeof(double) * n);
        *iters = t;
        if (syndrome_matches(&g, ehat, s)) {
            if (!*t_conv) *t_conv = t;
            if (stop_on_converge) break;
        }
    }
    if (min_abs_post) *min_abs_post = minabs;
    free(mu);
    free(rv);
    return 0;
}

int or_bp(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci, const int *ce,
          const double *lam, const uint8_t *s, const uint32_t *perm, int T, const double *alpha,
          double lim, int stop_on_converge, int *t_conv, uint8_t *ehat, double *post, int *iters,
          double *min_abs_post, double *trace) {
    return bp_core(m, n, rp, ri, cp, ci, ce, lam, s, perm, T, alpha, lim, stop_on_converge, t_conv, ehat,
                   post, iters, min_abs_post, trace, NULL, NULL);
}

/*
 * Min-sum BP with the layered (check-serial) schedule: the checks are visited
 * one at a time in the order cperm (a permutation of the m checks, one per
 * member), and each check works from the latest posteriors.  The paper names
 * layered schedules only as future work (Sec. V); the update is the usual
 * layered form of the same min-sum message passing:
 *   L_v starts at lambda_v (clamped), every check message r_{c->v} at 0;
 *   at check c, for each v in N(c): mu_{v->c} = L_v - r_{c->v} (the variable
 *   message without this check's own contribution), clamped;
 *   r_{c->v} = (1 - 2 s_c) alpha_t prod sign min |mu| over N(c) \ v;
 *   L_v = (L_v - r_old) + r_{c->v}, with the unclamped difference.
 * After all m checks, the posteriors are L_v clamped; the decision, the
 * convergence test and the outputs are those of or_bp.
 */
static int layered_core(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci, const int *ce,
                        const double *lam, const uint8_t *s, const uint32_t *cperm, int T, const double *alpha,
                        double lim, int stop_on_converge, int *t_conv, uint8_t *ehat, double *post, int *iters,
                        double *min_abs_post, double *trace, int *saturated) {
    ograph g = {m, n, rp, ri, cp, ci, ce, NULL};
    int E = rp[m];
    double *r = (double *)calloc((size_t)(E ? E : 1), sizeof(double));    /* by CSR position */
    double *mu = (double *)malloc(sizeof(double) * (E ? E : 1));          /* this check's mu, clamped */
    double *mraw = (double *)malloc(sizeof(double) * (E ? E : 1));        /* unclamped */
    double *rn = (double *)malloc(sizeof(double) * (E ? E : 1));
    double *Lv = (double *)malloc(sizeof(double) * (n ? n : 1));
    if (!r || !mu || !mraw || !rn || !Lv) {
        free(r);
        free(mu);
        free(mraw);
        free(rn);
        free(Lv);
        return -2;
    }
    for (int v = 0; v < n; v++) Lv[v] = clampd(lam[v], lim);
    memset(ehat, 0, (size_t)n);
    for (int v = 0; v < n; v++) post[v] = Lv[v];
    *t_conv = 0;
    *iters = 0;
    double minabs = INFINITY;
    for (int t = 1; t <= T; t++) {
        double a = alpha[t - 1];
        for (int idx = 0; idx < m; idx++) {
            int c = (int)cperm[idx];
            for (int k = rp[c]; k < rp[c + 1]; k++) {
                mraw[k] = Lv[ri[k]] - r[k];
                mu[k] = clamp_hit(mraw[k], lim, saturated);
            }
            /* every message of the row from the same mu (check_to_var reads mu by CSR position) */
            for (int k = rp[c]; k < rp[c + 1]; k++) rn[k] = check_to_var(&g, mu, s, c, ri[k], a, lim);
            for (int k = rp[c]; k < rp[c + 1]; k++) {
                r[k] = rn[k];
                Lv[ri[k]] = mraw[k] + r[k];
            }
        }
        for (int v = 0; v < n; v++) {
            post[v] = clamp_hit(Lv[v], lim, saturated);
            ehat[v] = post[v] <= 0.0;
            double aa = fabs(post[v]);
            if (aa < minabs) minabs = aa;
        }
        if (trace) memcpy(trace + (size_t)(t - 1) * n, post, sizeof(double) * n);
        *iters = t;
        if (syndrome_matches(&g, ehat, s)) {
            if (!*t_conv) *t_conv = t;
            if (stop_on_converge) break;
        }
    }
    if (min_abs_post) *min_abs_post = minabs;
    free(r);
    free(mu);
    free(mraw);
    free(rn);
    free(Lv);
    return 0;
}

int or_bp_layered(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci, const int *ce,
                  const double *lam, const uint8_t *s, const uint32_t *cperm, int T, const double *alpha,
                  double lim, int stop_on_converge, int *t_conv, uint8_t *ehat, double *post, int *iters,
                  double *min_abs_post, double *trace) {
    return layered_core(m, n, rp, ri, cp, ci, ce, lam, s, cperm, T, alpha, lim, stop_on_converge, t_conv, ehat,
                        post, iters, min_abs_post, trace, NULL);
}

/*
 * Soft-syndrome loss of K unrolled iterations (training objective of the
 * differentiable decoder; the paper defines none).  The decoder runs exactly
 * K iterations of Algorithm 1 (serial-V along perm, or parallel if perm is
 * NULL) from the given channel LLRs lam[v] with scaling alpha[t-1] in
 * iteration t.  With the final posteriors L_v, check c is violated with
 * probability shat_c = (1 - prod_{v in N(c)} tanh(L_v / 2)) / 2 when the bits
 * are independent with those LLRs; shat_c is clamped to [eps, 1 - eps] and
 * the loss is the binary cross-entropy summed over the checks,
 *   sum_c -[s_c ln shat_c + (1 - s_c) ln(1 - shat_c)].
 * sig (nullable) receives the hash of every branch taken (argmins, sign
 * parities, clamps); post (nullable, n) the final posteriors.
 */
double or_bp_loss(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci, const int *ce,
                  const double *lam, const uint8_t *s, const uint32_t *perm, int K, const double *alpha,
                  double lim, double eps, uint64_t *sig, double *post) {
    double *L = (double *)malloc(sizeof(double) * (n ? n : 1));
    uint8_t *e = (uint8_t *)malloc(n ? n : 1);
    int tc = 0, it = 0;
    if (sig) *sig = 0;
    bp_core(m, n, rp, ri, cp, ci, ce, lam, s, perm, K, alpha, lim, 0, &tc, e, L, &it, NULL, NULL, sig, NULL);
    double loss = 0.0;
    for (int c = 0; c < m; c++) {
        double prod = 1.0;
        for (int k = rp[c]; k < rp[c + 1]; k++) prod *= tanh(L[ri[k]] / 2.0);
        double sh = 0.5 * (1.0 - prod);
        if (sh < eps || sh > 1.0 - eps) {
            if (sig) sig_mix(sig, 0xe95ull + (uint64_t)c);
            sh = sh < eps ? eps : 1.0 - eps;
        }
        loss -= s[c] ? log(sh) : log(1.0 - sh);
    }
    if (post) memcpy(post, L, sizeof(double) * n);
    free(L);
    free(e);
    return loss;
}

/* ------------------------------------------------------------------------ */
/* GF(2) helpers on dense byte matrices (row-major, rows x cols)              */

/* Gaussian elimination over the columns in the given order.  On return
   piv[j] = 1 iff column j (in that order) is a pivot, i.e. independent of the
   earlier columns.  If b != NULL it is reduced alongside and *consistent is
   set to whether b lies in the column span; x (if non-NULL, length cols)
   receives the unique solution supported on the pivot columns. */
static void gf2_eliminate(uint8_t *A, int rows, int cols, uint8_t *b, uint8_t *piv, int *consistent,
                          uint8_t *x) {
    int *prow = (int *)malloc(sizeof(int) * (cols ? cols : 1));
    int r = 0;
    for (int j = 0; j < cols; j++) {
        piv[j] = 0;
        prow[j] = -1;
        int sel = -1;
        for (int i = r; i < rows; i++)
            if (A[(size_t)i * cols + j]) {
                sel = i;
                break;
            }
        if (sel < 0) continue;
        if (sel != r) {
            for (int k = 0; k < cols; k++) {
                uint8_t tmp = A[(size_t)r * cols + k];
                A[(size_t)r * cols + k] = A[(size_t)sel * cols + k];
                A[(size_t)sel * cols + k] = tmp;
            }
            if (b) {
                uint8_t tmp = b[r];
                b[r] = b[sel];
                b[sel] = tmp;
            }
        }
        for (int i = 0; i < rows; i++) {
            if (i != r && A[(size_t)i * cols + j]) {
                for (int k = 0; k < cols; k++) A[(size_t)i * cols + k] ^= A[(size_t)r * cols + k];
                if (b) b[i] ^= b[r];
            }
        }
        piv[j] = 1;
        prow[j] = r;
        r++;
    }
    if (b && consistent) {
        int ok = 1;
        for (int i = r; i < rows; i++)
            if (b[i]) ok = 0;
        *consistent = ok;
    }
    if (b && x) {
        for (int j = 0; j < cols; j++) x[j] = (piv[j] && b[prow[j]]) ? 1 : 0;
    }
    free(prow);
}

/* ------------------------------------------------------------------------ */
/* LSD-0                                                                      */

typedef struct {
    int alive;     /* 0 once merged into another cluster */
    int valid;     /* s restricted to checks lies in span H[checks, bits] */
    int failed;    /* invalid with an empty boundary */
    uint8_t *chk;  /* membership over checks, length m */
    uint8_t *bit;  /* membership over columns, length n */
} ocluster;

/* does (qa, a) come before (qb, b) in the rank order? */
static int rank_less(double qa, int a, double qb, int b) {
    if (qa < qb) return 1;
    if (qa > qb) return 0;
    return a < b;
}

static int cluster_is_valid(const ograph *g, const uint8_t *s, const ocluster *K) {
    int rows = 0, cols = 0;
    for (int c = 0; c < g->m; c++) rows += K->chk[c];
    for (int v = 0; v < g->n; v++) cols += K->bit[v];
    int *rix = (int *)malloc(sizeof(int) * g->m);
    int *cix = (int *)malloc(sizeof(int) * (cols ? cols : 1));
    int r = 0, cc = 0;
    for (int c = 0; c < g->m; c++) rix[c] = K->chk[c] ? r++ : -1;
    for (int v = 0; v < g->n; v++)
        if (K->bit[v]) cix[cc++] = v;
    uint8_t *A = (uint8_t *)calloc((size_t)rows * (cols ? cols : 1), 1);
    uint8_t *b = (uint8_t *)calloc(rows ? rows : 1, 1);
    uint8_t *piv = (uint8_t *)malloc(cols ? cols : 1);
    for (int j = 0; j < cols; j++) {
        int v = cix[j];
        for (int k = g->cp[v]; k < g->cp[v + 1]; k++)
            if (rix[g->ci[k]] >= 0) A[(size_t)rix[g->ci[k]] * cols + j] = 1;
    }
    for (int c = 0; c < g->m; c++)
        if (rix[c] >= 0) b[rix[c]] = s[c];
    int ok = 0;
    gf2_eliminate(A, rows, cols, b, piv, &ok, NULL);
    free(rix);
    free(cix);
    free(A);
    free(b);
    free(piv);
    return ok;
}

/* Soft values that rank LSD columns: either doubles or int64 fixed-point
   keys (the normalised average, see decode_one).  Rank order is (value,
   index) ascending. */
typedef struct {
    const double *q;
    const int64_t *k;
} osoft;

static int soft_less(const osoft *S, int a, int b) {
    if (S->k) return S->k[a] < S->k[b] || (S->k[a] == S->k[b] && a < b);
    return rank_less(S->q[a], a, S->q[b], b);
}

static double soft_val(const osoft *S, int v) {
    return S->k ? (double)S->k[v] * (1.0 / 72057594037927936.0) : S->q[v];
}

/* LSD-lambda for one valid cluster (its columns ord[0..cols) in rank order,
   H restricted to its checks in A0, s restricted to them in b0, pivots of
   the rank-order elimination in piv): the combination sweep of ordered
   statistics decoding over the non-pivot columns F (in rank order).  The
   candidates, in this order, set to 1 no column of F; each single column
   of F; each pair among the first min(order, |F|) columns of F, pairs in
   lexicographic order.  Every candidate's pivot values are solved afresh
   from s plus the chosen columns.  The candidate of least prior weight
   W(e) = sum_v e_v lam_v (summed in ascending v) replaces x; ties keep the
   earlier candidate.  The paper runs LSD-0, the variant without the
   higher-order search around the first solution (Sec. III.D.1 step 5); the
   sweep is the one of the OSD post-processor it cites (Sec. III.C). */
static void osd_cs(const ograph *g, const uint8_t *bit, const int *ord, int rows, int cols,
                   const uint8_t *A0, const uint8_t *b0, const uint8_t *piv, int order, const double *lam,
                   uint8_t *x) {
    int nf = 0;
    int *F = (int *)malloc(sizeof(int) * (cols ? cols : 1));
    for (int j = 0; j < cols; j++)
        if (!piv[j]) F[nf++] = j;
    if (nf == 0) {
        free(F);
        return;
    }
    const int lo = nf < order ? nf : order;
    const int ncand = 1 + nf + lo * (lo - 1) / 2;
    int *ca = (int *)malloc(sizeof(int) * ncand), *cb = (int *)malloc(sizeof(int) * ncand);
    int t = 0;
    ca[t] = cb[t] = -1;
    t++;
    for (int a = 0; a < nf; a++, t++) {
        ca[t] = F[a];
        cb[t] = -1;
    }
    for (int a = 0; a < lo; a++)
        for (int b = a + 1; b < lo; b++, t++) {
            ca[t] = F[a];
            cb[t] = F[b];
        }
    int *pos = (int *)malloc(sizeof(int) * (g->n ? g->n : 1));
    for (int v = 0; v < g->n; v++) pos[v] = -1;
    for (int j = 0; j < cols; j++) pos[ord[j]] = j;
    uint8_t *A = (uint8_t *)malloc((size_t)rows * cols), *b = (uint8_t *)malloc(rows ? rows : 1);
    uint8_t *pv = (uint8_t *)malloc(cols), *xc = (uint8_t *)malloc(cols), *best = (uint8_t *)malloc(cols);
    double bw = 0.0;
    for (t = 0; t < ncand; t++) {
        memcpy(A, A0, (size_t)rows * cols);
        memcpy(b, b0, (size_t)rows);
        for (int r = 0; r < rows; r++) {
            if (ca[t] >= 0) b[r] ^= A0[(size_t)r * cols + ca[t]];
            if (cb[t] >= 0) b[r] ^= A0[(size_t)r * cols + cb[t]];
        }
        int ok = 0;
        gf2_eliminate(A, rows, cols, b, pv, &ok, xc);
        if (ca[t] >= 0) xc[ca[t]] = 1;
        if (cb[t] >= 0) xc[cb[t]] = 1;
        double w = 0.0;
        for (int v = 0; v < g->n; v++)
            if (bit[v] && xc[pos[v]]) w += lam[v];
        if (t == 0 || w < bw) {
            bw = w;
            memcpy(best, xc, cols);
        }
    }
    memcpy(x, best, cols);
    free(F);
    free(ca);
    free(cb);
    free(pos);
    free(A);
    free(b);
    free(pv);
    free(xc);
    free(best);
}

/* stats layout (int[6]): clusters at the end, largest cluster (columns),
   growth rounds, failed (0/1), columns over all clusters, reserved.
   min_gap (if non-NULL): smallest q gap of any rank decision taken.
   chk_label / bit_label (if non-NULL, lengths m / n): final cluster of every
   check / column, numbered in order of the clusters' first check, or -1. */
static int lsd_impl(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci,
                    const uint8_t *s, const osoft *S, int order, const double *lam, uint8_t *ehat,
                    int *stats, double *min_gap, int *chk_label, int *bit_label) {
    ograph g = {m, n, rp, ri, cp, ci, NULL};
    memset(ehat, 0, (size_t)n);
    double gap = INFINITY;
    int nk = 0;
    for (int c = 0; c < m; c++) nk += s[c];
    ocluster *K = (ocluster *)calloc(nk ? nk : 1, sizeof(ocluster));
    {
        int i = 0;
        for (int c = 0; c < m; c++) {
            if (!s[c]) continue;
            K[i].alive = 1;
            K[i].chk = (uint8_t *)calloc(m, 1);
            K[i].bit = (uint8_t *)calloc(n ? n : 1, 1);
            K[i].chk[c] = 1;
            K[i].valid = 0; /* s restricted to {c} is 1, span of no columns is {0} */
            i++;
        }
    }
    int rounds = 0;
    int *pick = (int *)malloc(sizeof(int) * (nk ? nk : 1));
    for (;;) {
        int any = 0;
        /* 1. every invalid, growing cluster picks its best boundary column,
              all from the state at the start of the round */
        for (int i = 0; i < nk; i++) {
            pick[i] = -1;
            if (!K[i].alive || K[i].valid || K[i].failed) continue;
            int best = -1;
            double bq = 0, second = INFINITY;
            for (int v = 0; v < n; v++) {
                if (K[i].bit[v]) continue;
                int adj = 0;
                for (int k = cp[v]; k < cp[v + 1]; k++)
                    if (K[i].chk[ci[k]]) adj = 1;
                if (!adj) continue;
                if (best < 0 || soft_less(S, v, best)) {
                    if (best >= 0) second = fmin(second, bq);
                    best = v;
                    bq = soft_val(S, v);
                } else {
                    second = fmin(second, soft_val(S, v));
                }
            }
            if (best < 0) {
                K[i].failed = 1;
                continue;
            }
            if (second < INFINITY && second - bq < gap) gap = second - bq;
            pick[i] = best;
            any = 1;
        }
        if (!any) break;
        rounds++;
        /* 2. apply every addition */
        for (int i = 0; i < nk; i++) {
            if (pick[i] < 0) continue;
            int v = pick[i];
            K[i].bit[v] = 1;
            for (int k = cp[v]; k < cp[v + 1]; k++) K[i].chk[ci[k]] = 1;
        }
        /* 3. merge clusters whose check sets intersect, until none do */
        int merged = 1;
        while (merged) {
            merged = 0;
            for (int a = 0; a < nk; a++) {
                if (!K[a].alive) continue;
                for (int b = a + 1; b < nk; b++) {
                    if (!K[b].alive) continue;
                    int meet = 0;
                    for (int c = 0; c < m && !meet; c++) meet = K[a].chk[c] && K[b].chk[c];
                    if (!meet) continue;
                    for (int c = 0; c < m; c++) K[a].chk[c] |= K[b].chk[c];
                    for (int v = 0; v < n; v++) K[a].bit[v] |= K[b].bit[v];
                    K[a].failed |= K[b].failed;
                    K[b].alive = 0;
                    merged = 1;
                }
            }
        }
        /* 4. validity of every live cluster */
        for (int i = 0; i < nk; i++)
            if (K[i].alive) K[i].valid = cluster_is_valid(&g, s, &K[i]);
    }

    /* per-cluster OSD-0: columns in rank order; a column is a pivot iff it is
       independent of the earlier ones; solve on the pivots */
    int nclusters = 0, largest = 0, failed = 0, total = 0;
    for (int i = 0; i < nk; i++) {
        if (!K[i].alive) continue;
        nclusters++;
        int cols = 0, rows = 0;
        for (int v = 0; v < n; v++) cols += K[i].bit[v];
        for (int c = 0; c < m; c++) rows += K[i].chk[c];
        if (cols > largest) largest = cols;
        total += cols;
        if (!K[i].valid) {
            failed = 1;
            continue;
        }
        int *ord = (int *)malloc(sizeof(int) * (cols ? cols : 1));
        int cc = 0;
        for (int v = 0; v < n; v++)
            if (K[i].bit[v]) ord[cc++] = v;
        /* insertion sort by (q, index): plain and stable */
        for (int a = 1; a < cols; a++) {
            int x = ord[a], b = a - 1;
            while (b >= 0 && soft_less(S, x, ord[b])) {
                ord[b + 1] = ord[b];
                b--;
            }
            ord[b + 1] = x;
        }
        for (int a = 0; a + 1 < cols; a++) {
            double d = soft_val(S, ord[a + 1]) - soft_val(S, ord[a]);
            if (d < gap) gap = d;
        }
        int *rix = (int *)malloc(sizeof(int) * m);
        int r = 0;
        for (int c = 0; c < m; c++) rix[c] = K[i].chk[c] ? r++ : -1;
        uint8_t *A = (uint8_t *)calloc((size_t)rows * (cols ? cols : 1), 1);
        uint8_t *b = (uint8_t *)calloc(rows ? rows : 1, 1);
        uint8_t *piv = (uint8_t *)malloc(cols ? cols : 1);
        uint8_t *x = (uint8_t *)malloc(cols ? cols : 1);
        for (int j = 0; j < cols; j++) {
            int v = ord[j];
            for (int k = cp[v]; k < cp[v + 1]; k++) A[(size_t)rix[ci[k]] * cols + j] = 1;
        }
        for (int c = 0; c < m; c++)
            if (rix[c] >= 0) b[rix[c]] = s[c];
        uint8_t *A0 = (uint8_t *)malloc((size_t)rows * (cols ? cols : 1));
        uint8_t *b0 = (uint8_t *)malloc(rows ? rows : 1);
        memcpy(A0, A, (size_t)rows * cols);
        memcpy(b0, b, (size_t)rows);
        int ok = 0;
        gf2_eliminate(A, rows, cols, b, piv, &ok, x);
        if (order > 0) osd_cs(&g, K[i].bit, ord, rows, cols, A0, b0, piv, order, lam, x);
        for (int j = 0; j < cols; j++)
            if (x[j]) ehat[ord[j]] = 1;
        free(A0);
        free(b0);
        free(ord);
        free(rix);
        free(A);
        free(b);
        free(piv);
        free(x);
    }
    if (stats) {
        stats[0] = nclusters;
        stats[1] = largest;
        stats[2] = rounds;
        stats[3] = failed;
        stats[4] = total;
        stats[5] = 0;
    }
    if (min_gap) *min_gap = gap;
    if (chk_label) for (int c = 0; c < m; c++) chk_label[c] = -1;
    if (bit_label) for (int v = 0; v < n; v++) bit_label[v] = -1;
    {
        int lab = 0;
        for (int i = 0; i < nk; i++) {
            if (!K[i].alive) continue;
            for (int c = 0; c < m; c++)
                if (K[i].chk[c] && chk_label) chk_label[c] = lab;
            for (int v = 0; v < n; v++)
                if (K[i].bit[v] && bit_label) bit_label[v] = lab;
            lab++;
        }
    }
    for (int i = 0; i < nk; i++) {
        free(K[i].chk);
        free(K[i].bit);
    }
    free(K);
    free(pick);
    return failed ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* The full decoder for one shot.                                             */

/* LSD on double soft values (rank by (q, index) ascending); order 0 is
   LSD-0, order > 0 adds the combination sweep (osd_cs) with weights lam. */
int or_lsd(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci,
           const uint8_t *s, const double *q, int order, const double *lam, uint8_t *ehat, int *stats,
           double *min_gap, int *chk_label, int *bit_label) {
    osoft S = {q, NULL};
    return lsd_impl(m, n, rp, ri, cp, ci, s, &S, order, lam, ehat, stats, min_gap, chk_label, bit_label);
}

/* The same on int64 fixed-point soft values. */
int or_lsd_key(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci,
               const uint8_t *s, const int64_t *qk, int order, const double *lam, uint8_t *ehat,
               int *stats, double *min_gap, int *chk_label, int *bit_label) {
    osoft S = {NULL, qk};
    return lsd_impl(m, n, rp, ri, cp, ci, s, &S, order, lam, ehat, stats, min_gap, chk_label, bit_label);
}

/* per-shot record written by or_decode_batch, 16 doubles:
   [0] flags: bit0 BP converged, bit1 LSD used, bit2 LSD failed, bit3 saturated
       (a message or posterior reached the clamp: in the winner's run, or
       in any member's if LSD ran)
   [1] winning member (or -1)   [2] its convergence iteration
   [3] number of converged members
   [4] LSD clusters  [5] LSD largest cluster  [6] LSD growth rounds
   [7] smallest |L_v| of any decision by any member (tie witness)
   [8] smallest q gap of any LSD rank decision (tie witness)
   [9] chosen candidate's weight W   [10] weight gap to the runner-up
   [11..15] reserved */
#define OR_REC 16

typedef struct {
    int m, n, k;
    const int *rp, *ri, *cp, *ci, *ce, *lp, *li;
    const double *lam;
    const uint32_t *perms; /* L x n (serial-V) or L x m (layered) */
    int L, M, T;
    const double *alpha; /* T */
    double lim;
    int schedule; /* 0 serial-V, 1 parallel (members ignore perms), 2 layered */
    int lsd_order; /* 0 = LSD-0; > 0 adds the combination sweep */
} odec;

static void decode_one(const odec *D, const uint8_t *s, uint8_t *ehat, uint8_t *obs, double *rec,
                       int *t_members, double *q_out) {
    int n = D->n, L = D->L;
    uint8_t *e = (uint8_t *)malloc((size_t)L * (n ? n : 1));
    double *post = (double *)malloc(sizeof(double) * (size_t)L * (n ? n : 1));
    int *tc = (int *)malloc(sizeof(int) * L);
    double minabs_all = INFINITY;
    for (int i = 0; i < 16; i++) rec[i] = 0;
    rec[1] = -1;
    rec[8] = INFINITY;
    rec[10] = INFINITY;
    int *sat = (int *)calloc(L, sizeof(int));
    for (int i = 0; i < L; i++) {
        int iters = 0;
        double mn = INFINITY;
        if (D->schedule == 2)
            layered_core(D->m, n, D->rp, D->ri, D->cp, D->ci, D->ce, D->lam, s, D->perms + (size_t)i * D->m,
                         D->T, D->alpha, D->lim, 1, &tc[i], e + (size_t)i * n, post + (size_t)i * n, &iters, &mn,
                         NULL, &sat[i]);
        else
            bp_core(D->m, n, D->rp, D->ri, D->cp, D->ci, D->ce, D->lam, s,
                    D->schedule == 0 ? D->perms + (size_t)i * n : NULL, D->T, D->alpha, D->lim, 1,
                    &tc[i], e + (size_t)i * n, post + (size_t)i * n, &iters, &mn, NULL, NULL, &sat[i]);
        if (mn < minabs_all) minabs_all = mn;
        if (t_members) t_members[i] = tc[i];
    }
    rec[7] = minabs_all;
    int nconv = 0;
    for (int i = 0; i < L; i++) nconv += tc[i] > 0;
    rec[3] = nconv;
    memset(ehat, 0, (size_t)n);
    if (nconv) {
        /* first M converged members in (iteration, index) order */
        int *S = (int *)malloc(sizeof(int) * L);
        int ns = 0;
        for (int t = 1; t <= D->T && ns < D->M; t++)
            for (int i = 0; i < L && ns < D->M; i++)
                if (tc[i] == t) S[ns++] = i;
        int best = -1;
        double bw = 0, second = INFINITY;
        for (int a = 0; a < ns; a++) {
            int i = S[a];
            double w = 0;
            for (int v = 0; v < n; v++)
                if (e[(size_t)i * n + v]) w += D->lam[v];
            if (best < 0 || w < bw) {
                if (best >= 0) second = fmin(second, bw);
                best = i;
                bw = w;
            } else {
                second = fmin(second, w);
            }
        }
        memcpy(ehat, e + (size_t)best * n, (size_t)n);
        rec[0] = 1 | (sat[best] ? 8 : 0);
        rec[1] = best;
        rec[2] = tc[best];
        rec[9] = bw;
        rec[10] = second - bw;
        free(S);
    } else {
        /* normalised average of the members' final posteriors,
           q = (1/L) sum_i LLR^i / ||LLR^i||.  ||LLR^i||^2 is summed in
           ascending v; each term LLR^i_v / ||LLR^i|| is rounded to a
           multiple of 2^-56 (as LLR^i_v * (2^56 / ||LLR^i||), to nearest)
           and the terms are added exactly in int64, so q does not depend on
           the order of the members.  The factor 1/L does not change the
           ranking and is applied only to the reported q. */
        int64_t *qk = (int64_t *)calloc(n ? n : 1, sizeof(int64_t));
        for (int i = 0; i < L; i++) {
            double ss = 0;
            for (int v = 0; v < n; v++) ss += post[(size_t)i * n + v] * post[(size_t)i * n + v];
            double nrm = sqrt(ss);
            if (nrm == 0) continue;
            double scale = 72057594037927936.0 / nrm;
            for (int v = 0; v < n; v++) qk[v] += llrint(post[(size_t)i * n + v] * scale);
        }
        if (q_out)
            for (int v = 0; v < n; v++) q_out[v] = (double)qk[v] * (1.0 / 72057594037927936.0) / L;
        int st[6];
        double gap = INFINITY;
        int f = or_lsd_key(D->m, n, D->rp, D->ri, D->cp, D->ci, s, qk, D->lsd_order, D->lam, ehat, st, &gap,
                           NULL, NULL);
        int any_sat = 0;
        for (int i = 0; i < L; i++) any_sat |= sat[i];
        rec[0] = 2 | (f ? 4 : 0) | (any_sat ? 8 : 0);
        rec[4] = st[0];
        rec[5] = st[1];
        rec[6] = st[2];
        rec[8] = gap;
        free(qk);
    }
    for (int r = 0; r < D->k; r++) {
        int par = 0;
        for (int a = D->lp[r]; a < D->lp[r + 1]; a++) par ^= ehat[D->li[a]];
        obs[r] = (uint8_t)par;
    }
    /* a zero syndrome with every LLR positive is decided without running BP
       (the decision e = 0 at the first iteration is certain): no saturation
       is reported for it */
    {
        int zero = 1, pos = 1;
        for (int c = 0; c < D->m; c++) zero &= s[c] == 0;
        for (int v = 0; v < n; v++) pos &= D->lam[v] > 0.0;
        if (zero && pos) rec[0] = (double)((int)rec[0] & ~8);
    }
    free(sat);
    free(e);
    free(post);
    free(tc);
}

typedef struct {
    const odec *D;
    const uint8_t *synd;
    uint8_t *ehat, *obs;
    double *rec;
    int *t_members;
    double *q_out;
    int64_t next, end;
    pthread_mutex_t *lock;
} oworker;

static void *worker_main(void *arg) {
    oworker *w = (oworker *)arg;
    const odec *D = w->D;
    for (;;) {
        pthread_mutex_lock(w->lock);
        int64_t b = w->next < w->end ? w->next++ : -1;
        pthread_mutex_unlock(w->lock);
        if (b < 0) break;
        decode_one(D, w->synd + (size_t)b * D->m, w->ehat + (size_t)b * D->n, w->obs + (size_t)b * D->k,
                   w->rec + (size_t)b * OR_REC, w->t_members ? w->t_members + (size_t)b * D->L : NULL,
                   w->q_out ? w->q_out + (size_t)b * D->n : NULL);
    }
    return NULL;
}

/* Decode B shots with `threads` host threads.  lam[v] must already be the
   clamped prior LLR.  t_members (B x L, nullable) receives every member's
   convergence iteration (0 = none); q_out (B x n, nullable) receives the
   normalised average for shots that reach LSD. */
int or_decode_batch(int m, int n, int k, const int *rp, const int *ri, const int *cp, const int *ci,
                    const int *ce, const int *lp, const int *li, const double *lam,
                    const uint32_t *perms, int L, int M, int T, const double *alpha, double lim,
                    int schedule, int lsd_order, const uint8_t *synd, int64_t B, int threads,
                    uint8_t *ehat, uint8_t *obs, double *rec, int *t_members, double *q_out) {
    odec D = {m, n, k, rp, ri, cp, ci, ce, lp, li, lam, perms, L, M, T, alpha, lim, schedule, lsd_order};
    pthread_mutex_t lock;
    pthread_mutex_init(&lock, NULL);
    oworker w = {&D, synd, ehat, obs, rec, t_members, q_out, 0, B, &lock};
    if (threads < 1) threads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    for (int i = 0; i < threads; i++) pthread_create(&th[i], NULL, worker_main, &w);
    for (int i = 0; i < threads; i++) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&lock);
    return 0;
}
