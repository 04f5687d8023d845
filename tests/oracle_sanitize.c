/* Drives every entry point of the oracle (oracle/oracle.c) on small seeded inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py compiles and runs it on
 * the host).  Exit status 0 when every call succeeds and every result is finite; a sanitizer report
 * aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct or_tree or_tree;
int or_allpairs_field(int64_t n, const double *pos, const double *mom, double *H);
int or_allpairs_field_subset(int64_t n, const double *pos, const double *mom, int64_t nt, const int64_t *t,
                             double *H);
double or_energy(int64_t n, const double *mom, const double *H, const double *hext);
int or_allpairs_grad_r(int64_t n, const double *pos, const double *mom, double *dEdr);
int or_allpairs_grad_r_subset(int64_t n, const double *pos, const double *mom, int64_t nt, const int64_t *t,
                              double *g);
or_tree *or_tree_build(int64_t n, const double *pos, const double *mom, int leaf);
void or_tree_free(or_tree *t);
int64_t or_tree_num_nodes(const or_tree *t);
void or_tree_export(const or_tree *t, double *bbox, uint64_t *code, int64_t *perm, int32_t *level, int64_t *first,
                    int64_t *count, int32_t *nchild, int64_t *child8, int64_t *parent, double *S, double *M, double *c,
                    double *s2);
void or_tree_export_D(const or_tree *t, double *D);
int or_bh_field(const or_tree *t, double theta, double *H, int64_t *n_far, int64_t *n_near);
int or_bh_field_order(const or_tree *t, double theta, int order, double *H, int64_t *n_far, int64_t *n_near);
int or_bh_field_subset(const or_tree *t, double theta, int64_t nt, const int64_t *targets, double *H, int64_t *nf,
                       int64_t *nr);
int or_bh_lists(const or_tree *t, double theta, int64_t *far_ptr, int64_t *far_node, int64_t *near_ptr,
                int64_t *near_idx);
int or_bh_vjp(const or_tree *t, double theta, const double *hbar, double *dLdr, double *dLdm);
int or_bh_vjp_order(const or_tree *t, double theta, int order, const double *hbar, double *dLdr, double *dLdm);
double or_energy_frozen_order(int64_t n, const double *pos, const double *mom, const double *hext, int64_t nn,
                              const int64_t *first, const int64_t *count, const int64_t *perm,
                              const int64_t *far_ptr, const int64_t *far_node, const int64_t *near_ptr,
                              const int64_t *near_idx, int order, double *scratch);
int or_fd_grad_frozen_order(int64_t n, const double *pos, const double *mom, const double *hext, int64_t nn,
                            const int64_t *first, const int64_t *count, const int64_t *perm,
                            const int64_t *far_ptr, const int64_t *far_node, const int64_t *near_ptr,
                            const int64_t *near_idx, double h, int order, double *dEdr, double *dEdm);

static uint64_t rng = 88172645463325252ull;
static double uni(void)
{
    rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;  /* xorshift64 */
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int finite_all(const double *a, int64_t k)
{
    for (int64_t i = 0; i < k; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);  \
            return 1;                                                       \
        }                                                                   \
    } while (0)

static int run(int64_t n, int leaf, double theta)
{
    double *pos = malloc(3 * n * sizeof(double)), *mom = malloc(3 * n * sizeof(double));
    /* jittered grid points (distinct, at least 0.3 apart) and unit moments */
    int64_t side = 1;
    while (side * side * side < n) ++side;
    for (int64_t i = 0; i < n; ++i) {
        pos[i] = (double)(i % side) + 0.35 * uni();
        pos[n + i] = (double)((i / side) % side) + 0.35 * uni();
        pos[2 * n + i] = (double)(i / (side * side)) + 0.35 * uni();
        double m[3] = {uni() - 0.5, uni() - 0.5, uni() - 0.5};
        double r = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) + 1e-12;
        for (int a = 0; a < 3; ++a) mom[a * n + i] = m[a] / r;
    }
    const double hext[3] = {0.1, 0.0, 0.4};
    double *H = malloc(3 * n * sizeof(double)), *G = malloc(3 * n * sizeof(double));
    double *dr = malloc(3 * n * sizeof(double)), *dm = malloc(3 * n * sizeof(double));
    int64_t *nf = malloc(n * sizeof(int64_t)), *nr = malloc(n * sizeof(int64_t));
    int64_t nt = n < 7 ? n : 7, tg[7];
    for (int64_t k = 0; k < nt; ++k) tg[k] = (k * 5) % n;
    double Hs[21], gs[21];
    CHECK(or_allpairs_field(n, pos, mom, H) == 0 && finite_all(H, 3 * n));
    CHECK(or_allpairs_field_subset(n, pos, mom, nt, tg, Hs) == 0 && finite_all(Hs, 3 * nt));
    CHECK(isfinite(or_energy(n, mom, H, hext)));
    CHECK(or_allpairs_grad_r(n, pos, mom, G) == 0 && finite_all(G, 3 * n));
    CHECK(or_allpairs_grad_r_subset(n, pos, mom, nt, tg, gs) == 0 && finite_all(gs, 3 * nt));
    or_tree *t = or_tree_build(n, pos, mom, leaf);
    CHECK(t != NULL);
    const int64_t nn = or_tree_num_nodes(t);
    CHECK(nn >= 1);
    double bbox[5];
    uint64_t *code = malloc(n * sizeof(uint64_t));
    int64_t *perm = malloc(n * sizeof(int64_t)), *first = malloc(nn * sizeof(int64_t));
    int64_t *count = malloc(nn * sizeof(int64_t)), *child8 = malloc(8 * nn * sizeof(int64_t));
    int64_t *parent = malloc(nn * sizeof(int64_t));
    int32_t *level = malloc(nn * sizeof(int32_t)), *nchild = malloc(nn * sizeof(int32_t));
    double *S = malloc(3 * nn * sizeof(double)), *M = malloc(3 * nn * sizeof(double));
    double *c = malloc(3 * nn * sizeof(double)), *s2 = malloc(nn * sizeof(double));
    double *D = malloc(9 * nn * sizeof(double));
    or_tree_export(t, bbox, code, perm, level, first, count, nchild, child8, parent, S, M, c, s2);
    or_tree_export_D(t, D);
    CHECK(finite_all(c, 3 * nn) && finite_all(D, 9 * nn));
    for (int order = 1; order <= 2; ++order) {
        CHECK(or_bh_field_order(t, theta, order, H, nf, nr) == 0 && finite_all(H, 3 * n));
        for (int64_t i = 0; i < n; ++i) {
            G[i] = -0.5 * mom[i]; G[n + i] = -0.5 * mom[n + i]; G[2 * n + i] = -0.5 * mom[2 * n + i];
        }
        CHECK(or_bh_vjp_order(t, theta, order, G, dr, dm) == 0 && finite_all(dr, 3 * n) && finite_all(dm, 3 * n));
    }
    CHECK(or_bh_field(t, theta, H, nf, nr) == 0);
    CHECK(or_bh_vjp(t, theta, G, dr, dm) == 0);
    CHECK(or_bh_field_subset(t, theta, nt, tg, Hs, nf, nr) == 0 && finite_all(Hs, 3 * nt));
    int64_t *fp = calloc(n + 1, sizeof(int64_t)), *np = calloc(n + 1, sizeof(int64_t));
    CHECK(or_bh_lists(t, theta, fp, NULL, np, NULL) == 0);
    int64_t *fn = malloc((fp[n] > 0 ? fp[n] : 1) * sizeof(int64_t));
    int64_t *ni = malloc((np[n] > 0 ? np[n] : 1) * sizeof(int64_t));
    CHECK(or_bh_lists(t, theta, fp, fn, np, ni) == 0);
    double *scr = malloc(15 * nn * sizeof(double));
    for (int order = 1; order <= 2; ++order) {
        CHECK(isfinite(or_energy_frozen_order(n, pos, mom, hext, nn, first, count, perm, fp, fn, np, ni, order,
                                              scr)));
        CHECK(or_fd_grad_frozen_order(n, pos, mom, hext, nn, first, count, perm, fp, fn, np, ni, 1e-6, order, dr,
                                      dm) == 0 && finite_all(dr, 3 * n) && finite_all(dm, 3 * n));
    }
    or_tree_free(t);
    free(pos); free(mom); free(H); free(G); free(dr); free(dm); free(nf); free(nr); free(code); free(perm);
    free(first); free(count); free(child8); free(parent); free(level); free(nchild); free(S); free(M); free(c);
    free(s2); free(D); free(fp); free(np); free(fn); free(ni); free(scr);
    return 0;
}

int main(void)
{
    /* a single particle, a root that is a leaf, leaves of one particle, and a few hundred particles */
    const int64_t ns[] = {1, 2, 17, 64, 300};
    const int leaves[] = {16, 1, 16, 1, 16};
    for (int k = 0; k < 5; ++k)
        for (int q = 0; q < 2; ++q) {
            const double theta = q ? 0.7 : 0.0;
            if (run(ns[k], leaves[k], theta) != 0) {
                fprintf(stderr, "failed: n %lld leaf %d theta %g\n", (long long)ns[k], leaves[k], theta);
                return 1;
            }
        }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
