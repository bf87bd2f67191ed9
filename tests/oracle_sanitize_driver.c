/*
 * Drives every entry point of the CPU oracle (oracle/vibelsd_oracle.c) on
 * small graphs, for a build under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_oracle_sanitizers.py compiles and runs it; no GPU).
 * Graphs: a repetition chain, a triangle of checks with pendant columns, and
 * a random sparse matrix from a fixed linear congruential generator with a
 * column in no check, a check with no column and a degree-1 check.  Every
 * call checks its result for validity where one is defined (H e = s on
 * every shot LSD did not flag).  Exit status 0 means every call returned
 * sane results; the sanitizers abort on any memory or UB error.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int or_bp(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci, const int *ce,
          const double *lam, const uint8_t *s, const uint32_t *perm, int T, const double *alpha, double lim,
          int stop_on_converge, int *t_conv, uint8_t *ehat, double *post, int *iters, double *min_abs_post,
          double *trace);
int or_bp_layered(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci, const int *ce,
                  const double *lam, const uint8_t *s, const uint32_t *cperm, int T, const double *alpha,
                  double lim, int stop_on_converge, int *t_conv, uint8_t *ehat, double *post, int *iters,
                  double *min_abs_post, double *trace);
double or_bp_loss(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci, const int *ce,
                  const double *lam, const uint8_t *s, const uint32_t *perm, int K, const double *alpha,
                  double lim, double eps, uint64_t *sig, double *post);
int or_lsd(int m, int n, const int *rp, const int *ri, const int *cp, const int *ci, const uint8_t *s,
           const double *q, int order, const double *lam, uint8_t *ehat, int *stats, double *min_gap,
           int *chk_label, int *bit_label);
int or_decode_batch(int m, int n, int k, const int *rp, const int *ri, const int *cp, const int *ci,
                    const int *ce, const int *lp, const int *li, const double *lam, const uint32_t *perms, int L,
                    int M, int T, const double *alpha, double lim, int schedule, int lsd_order,
                    const uint8_t *synd, int64_t B, int threads, uint8_t *ehat, uint8_t *obs, double *rec,
                    int *t_members, double *q_out);

static uint64_t lcg = 88172645463325252ull;
static uint32_t rnd(uint32_t mod) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(lcg >> 33) % mod;
}

typedef struct {
    int m, n;
    int *rp, *ri, *cp, *ci, *ce;
    double *lam;
} graph;

/* CSR/CSC/edge map of a dense 0/1 matrix (rows x cols). */
static graph from_dense(const uint8_t *H, int m, int n, double p) {
    graph g;
    g.m = m;
    g.n = n;
    int E = 0;
    for (int i = 0; i < m * n; i++) E += H[i];
    g.rp = malloc(sizeof(int) * (m + 1));
    g.ri = malloc(sizeof(int) * (E ? E : 1));
    g.cp = malloc(sizeof(int) * (n + 1));
    g.ci = malloc(sizeof(int) * (E ? E : 1));
    g.ce = malloc(sizeof(int) * (E ? E : 1));
    g.lam = malloc(sizeof(double) * n);
    int k = 0;
    for (int c = 0; c < m; c++) {
        g.rp[c] = k;
        for (int v = 0; v < n; v++)
            if (H[c * n + v]) g.ri[k++] = v;
    }
    g.rp[m] = k;
    k = 0;
    for (int v = 0; v < n; v++) {
        g.cp[v] = k;
        for (int c = 0; c < m; c++)
            if (H[c * n + v]) {
                g.ci[k] = c;
                for (int a = g.rp[c]; a < g.rp[c + 1]; a++)
                    if (g.ri[a] == v) g.ce[k] = a;
                k++;
            }
        g.lam[v] = log((1.0 - p) / p) + 0.01 * (double)(v % 7);
    }
    g.cp[n] = k;
    return g;
}

static void free_graph(graph *g) {
    free(g->rp);
    free(g->ri);
    free(g->cp);
    free(g->ci);
    free(g->ce);
    free(g->lam);
}

static int check_syndrome(const graph *g, const uint8_t *e, const uint8_t *s) {
    for (int c = 0; c < g->m; c++) {
        int par = 0;
        for (int a = g->rp[c]; a < g->rp[c + 1]; a++) par ^= e[g->ri[a]];
        if (par != s[c]) return 0;
    }
    return 1;
}

static void perm_of(uint32_t *p, int n) {
    for (int i = 0; i < n; i++) p[i] = (uint32_t)i;
    for (int i = n - 1; i > 0; i--) {
        int j = (int)rnd((uint32_t)i + 1);
        uint32_t t = p[i];
        p[i] = p[j];
        p[j] = t;
    }
}

static int exercise(const graph *g, int B, int L, int T, int order) {
    const int m = g->m, n = g->n;
    double alpha[64];
    for (int t = 0; t < 64; t++) alpha[t] = 0.625 + 0.01 * (t % 3);
    uint32_t *perms = malloc(sizeof(uint32_t) * L * (n > m ? n : m));
    uint8_t *synd = calloc((size_t)B * (m ? m : 1), 1);
    uint8_t *e = malloc(n ? n : 1);
    for (int b = 0; b < B; b++) {
        memset(e, 0, n);
        for (int v = 0; v < n; v++) e[v] = rnd(100) < 8;
        for (int c = 0; c < m; c++)
            for (int a = g->rp[c]; a < g->rp[c + 1]; a++) synd[(size_t)b * m + c] ^= e[g->ri[a]];
    }
    int lp[2] = {0, n < 5 ? n : 5}, li[5] = {0, 1, 2, 3, 4};
    int bad = 0;
    /* members, all three schedules, with traces */
    double *post = malloc(sizeof(double) * n), *trace = malloc(sizeof(double) * T * n);
    int tc, it;
    double mn;
    for (int b = 0; b < B && b < 4; b++) {
        const uint8_t *s = synd + (size_t)b * m;
        perm_of(perms, n);
        or_bp(m, n, g->rp, g->ri, g->cp, g->ci, g->ce, g->lam, s, perms, T, alpha, 1e6, 1, &tc, e, post, &it, &mn,
              trace);
        or_bp(m, n, g->rp, g->ri, g->cp, g->ci, g->ce, g->lam, s, NULL, T, alpha, 1e6, 0, &tc, e, post, &it, &mn,
              trace);
        perm_of(perms, m);
        or_bp_layered(m, n, g->rp, g->ri, g->cp, g->ci, g->ce, g->lam, s, perms, T, alpha, 1e6, 1, &tc, e, post, &it,
                      &mn, trace);
        uint64_t sig = 0;
        perm_of(perms, n);
        double loss = or_bp_loss(m, n, g->rp, g->ri, g->cp, g->ci, g->ce, g->lam, s, perms, 6, alpha, 1e6, 1e-7,
                                 &sig, post);
        if (!(loss >= 0.0) || !isfinite(loss)) bad++;
        /* LSD on noisy soft values, orders 0 and `order` */
        double *q = malloc(sizeof(double) * n);
        for (int v = 0; v < n; v++) q[v] = g->lam[v] + 0.1 * (double)rnd(50) - 2.5;
        int st[6], *cl = malloc(sizeof(int) * (m ? m : 1)), *bl = malloc(sizeof(int) * n);
        double gap;
        for (int o = 0; o <= order; o += order ? order : 1) {
            int f = or_lsd(m, n, g->rp, g->ri, g->cp, g->ci, s, q, o, g->lam, e, st, &gap, cl, bl);
            if (!f && !check_syndrome(g, e, s)) bad++;
            if (!order) break;
        }
        free(q);
        free(cl);
        free(bl);
    }
    /* whole decoder, every schedule, threaded, with member records and q */
    for (int sched = 0; sched < 3; sched++) {
        for (int i = 0; i < L; i++) perm_of(perms + (size_t)i * (sched == 2 ? m : n), sched == 2 ? m : n);
        uint8_t *E = malloc((size_t)B * n), *obs = malloc((size_t)B);
        double *rec = malloc(sizeof(double) * 16 * B), *qo = malloc(sizeof(double) * (size_t)B * n);
        int *tm = malloc(sizeof(int) * (size_t)B * L);
        or_decode_batch(m, n, 1, g->rp, g->ri, g->cp, g->ci, g->ce, lp, li, g->lam, perms, L, L > 2 ? 3 : 1, T,
                        alpha, 1e6, sched, order, synd, B, 3, E, obs, rec, tm, qo);
        for (int b = 0; b < B; b++) {
            const int fl = (int)rec[16 * b];
            if (!(fl & 4) && !check_syndrome(g, E + (size_t)b * n, synd + (size_t)b * m)) bad++;
        }
        free(E);
        free(obs);
        free(rec);
        free(qo);
        free(tm);
    }
    free(post);
    free(trace);
    free(perms);
    free(synd);
    free(e);
    return bad;
}

int main(void) {
    int bad = 0;
    /* repetition chain, 5 checks x 6 columns */
    uint8_t chain[30] = {0};
    for (int c = 0; c < 5; c++) chain[c * 6 + c] = chain[c * 6 + c + 1] = 1;
    graph g1 = from_dense(chain, 5, 6, 0.1);
    bad += exercise(&g1, 40, 4, 12, 2);
    free_graph(&g1);
    /* triangle of checks with pendant columns */
    uint8_t tri[18] = {1, 0, 1, 1, 0, 0, 1, 1, 0, 0, 1, 0, 0, 1, 1, 0, 0, 1};
    graph g2 = from_dense(tri, 3, 6, 0.15);
    bad += exercise(&g2, 40, 3, 10, 10);
    free_graph(&g2);
    /* random sparse matrix: 30 checks x 80 columns, weights 0..4; column 0
       in no check, check 0 with no column, check 1 of degree 1 */
    const int m = 30, n = 80;
    uint8_t *H = calloc(m * n, 1);
    for (int v = 1; v < n; v++) {
        int w = 1 + (int)rnd(4);
        for (int j = 0; j < w; j++) H[(2 + rnd(m - 2)) * n + v] = 1;
    }
    H[1 * n + 5] = 1;
    graph g3 = from_dense(H, m, n, 0.05);
    bad += exercise(&g3, 120, 8, 20, 10);
    free_graph(&g3);
    free(H);
    printf("oracle sanitizer driver: %d invalid results\n", bad);
    return bad ? 1 : 0;
}
