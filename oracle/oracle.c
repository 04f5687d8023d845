/*
 * oracle.c -- plain FP64 CPU reference for the Barnes-Hut dipolar field (TEST INFRASTRUCTURE ONLY).
 *
 * This is the checker for the GPU library, not part of it.  Only the test suite, the package smoke check
 * and the CPU-baseline leg of the benchmark load it; the GPU library never links, loads or calls it, and
 * the two share no code.  Everything here is written from the paper
 *   A.Yu. Polyakov et al., "Large-scale ferrofluid simulations on graphics processing units",
 *   arXiv:1212.2934,
 * and from the readings of it recorded with each function.  It is deliberately slow and literal:
 * FP64 throughout, one target at a time, no blocking and no reordering beyond what the definition says.
 * OpenMP only splits independent targets (or independent finite-difference coordinates) over threads.
 *
 * Array convention: a vector field over n particles is FP64 structure-of-arrays of shape (3, n):
 * x components at [0, n), y at [n, 2n), z at [2n, 3n).
 *
 * Reduced units as in Sec. 2 (reduced equations): positions in units of the diameter d = 1, unit
 * moments, no mu0/4pi prefactor, so the pair field is Eq. (H_dip) verbatim.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_BITS 21                    /* bits of the quantised coordinate per axis */
#define OR_QMAX ((1u << OR_BITS) - 1u)
#define OR_MAXLEVEL 21                /* deepest cell level (side / 2^21)          */

/* ------------------------------------------------------------------------------------------------ */
/* Pair kernels                                                                                       */
/* ------------------------------------------------------------------------------------------------ */

/* Field at offset x = r_target - r_source of a dipole m, Eq. (H_dip) of Sec. 2:
 *   h = [3 x (m . x) - m |x|^2] / |x|^5                                                              */
static void dip_field(const double x[3], const double m[3], double h[3])
{
    double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    double r = sqrt(r2);
    double r5 = r2 * r2 * r;
    double mx = m[0] * x[0] + m[1] * x[1] + m[2] * x[2];
    for (int a = 0; a < 3; ++a) h[a] = (3.0 * x[a] * mx - m[a] * r2) / r5;
}

/* Gradient kernel: the x-gradient of a . T(x) b, where T(x) b is the field of dipole b at offset x.
 * This is the summand of the reduced dipolar force f_dip of Sec. 2 with a = u_k, b = u_j, x = rho_kj:
 *   g = 3 [x (a.b) + a (b.x) + b (a.x)] / |x|^5 - 15 x (a.x)(b.x) / |x|^7                            */
static void grad_kernel(const double x[3], const double a[3], const double b[3], double g[3])
{
    double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    double r = sqrt(r2);
    double r5 = r2 * r2 * r;
    double r7 = r5 * r2;
    double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double ax = a[0] * x[0] + a[1] * x[1] + a[2] * x[2];
    double bx = b[0] * x[0] + b[1] * x[1] + b[2] * x[2];
    for (int c = 0; c < 3; ++c)
        g[c] = 3.0 * (x[c] * ab + a[c] * bx + b[c] * ax) / r5 - 15.0 * x[c] * ax * bx / r7;
}

static inline void load3(const double *v, int64_t n, int64_t i, double out[3])
{
    out[0] = v[i];
    out[1] = v[n + i];
    out[2] = v[2 * n + i];
}

/* ------------------------------------------------------------------------------------------------ */
/* All-pairs (the exact sum that Barnes-Hut approximates)                                             */
/* ------------------------------------------------------------------------------------------------ */

/* H_i = sum_{j != i} h_ij over ascending j (Eq. H of Sec. 2, dipolar part only). */
int or_allpairs_field(int64_t n, const double *pos, const double *mom, double *H)
{
    if (n < 0 || (n > 0 && (!pos || !mom || !H))) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double ri[3], rj[3], mj[3], x[3], h[3], acc[3] = {0.0, 0.0, 0.0};
        load3(pos, n, i, ri);
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            load3(pos, n, j, rj);
            load3(mom, n, j, mj);
            for (int a = 0; a < 3; ++a) x[a] = ri[a] - rj[a];
            dip_field(x, mj, h);
            for (int a = 0; a < 3; ++a) acc[a] += h[a];
        }
        for (int a = 0; a < 3; ++a) H[a * n + i] = acc[a];
    }
    return 0;
}

/* All-pairs field for a subset of targets (rows of H_out follow the order of `targets`). */
int or_allpairs_field_subset(int64_t n, const double *pos, const double *mom, int64_t nt,
                             const int64_t *targets, double *H_out)
{
    if (n < 0 || nt < 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets[t];
        double ri[3], rj[3], mj[3], x[3], h[3], acc[3] = {0.0, 0.0, 0.0};
        load3(pos, n, i, ri);
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            load3(pos, n, j, rj);
            load3(mom, n, j, mj);
            for (int a = 0; a < 3; ++a) x[a] = ri[a] - rj[a];
            dip_field(x, mj, h);
            for (int a = 0; a < 3; ++a) acc[a] += h[a];
        }
        for (int a = 0; a < 3; ++a) H_out[a * nt + t] = acc[a];
    }
    return 0;
}

/* Total energy E = -1/2 sum_i m_i . H_i - sum_i m_i . H_ext, H_i the dipolar field. */
double or_energy(int64_t n, const double *mom, const double *H, const double *hext)
{
    double e_dip = 0.0, e_ext = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            e_dip += mom[a * n + i] * H[a * n + i];
            e_ext += mom[a * n + i] * (hext ? hext[a] : 0.0);
        }
    }
    return -0.5 * e_dip - e_ext;
}

/* dE/dr_k of the all-pairs energy: -sum_{j != k} g(r_k - r_j; m_k, m_j), i.e. minus the reduced
 * dipolar force f_dip of Sec. 2.  (The Zeeman term does not depend on r.)                           */
int or_allpairs_grad_r(int64_t n, const double *pos, const double *mom, double *dEdr)
{
    if (n < 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double rk[3], mk[3], rj[3], mj[3], x[3], g[3], acc[3] = {0.0, 0.0, 0.0};
        load3(pos, n, k, rk);
        load3(mom, n, k, mk);
        for (int64_t j = 0; j < n; ++j) {
            if (j == k) continue;
            load3(pos, n, j, rj);
            load3(mom, n, j, mj);
            for (int a = 0; a < 3; ++a) x[a] = rk[a] - rj[a];
            grad_kernel(x, mk, mj, g);
            for (int a = 0; a < 3; ++a) acc[a] += g[a];
        }
        for (int a = 0; a < 3; ++a) dEdr[a * n + k] = -acc[a];
    }
    return 0;
}

/* Same, for a subset of targets. */
int or_allpairs_grad_r_subset(int64_t n, const double *pos, const double *mom, int64_t nt,
                              const int64_t *targets, double *out)
{
    if (n < 0 || nt < 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t k = targets[t];
        double rk[3], mk[3], rj[3], mj[3], x[3], g[3], acc[3] = {0.0, 0.0, 0.0};
        load3(pos, n, k, rk);
        load3(mom, n, k, mk);
        for (int64_t j = 0; j < n; ++j) {
            if (j == k) continue;
            load3(pos, n, j, rj);
            load3(mom, n, j, mj);
            for (int a = 0; a < 3; ++a) x[a] = rk[a] - rj[a];
            grad_kernel(x, mk, mj, g);
            for (int a = 0; a < 3; ++a) acc[a] += g[a];
        }
        for (int a = 0; a < 3; ++a) out[a * nt + t] = -acc[a];
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------------ */
/* Octree (Sec. 3.2): the "main cell" is a cube, recursively split into 8 sub-cells.                  */
/*                                                                                                    */
/* Readings where the paper is silent:                                                                */
/*  - The cube is anchored at the componentwise minimum of the positions, side = largest extent.      */
/*  - A position is mapped to the integer cell grid of level 21: q = min(2^21-1, floor((r-lo)*scale)),*/
/*    scale = 2^21/side (0 if side == 0).  Cell membership at level l is the top l bits of q.         */
/*  - Splitting stops when a cell holds at most `leaf` particles (the paper's leaves hold one; the    */
/*    leaf size is a parameter here) or at level 21.                                                  */
/*  - Sub-cells are kept in octant order o = 4*xbit + 2*ybit + zbit; particles in (code, index) order. */
/* Unary cells (one non-empty child) are kept as they are: this tree is the uncollapsed definition.   */
/* ------------------------------------------------------------------------------------------------ */

typedef struct or_tree {
    int64_t n;
    int leaf;
    double lo[3], side, scale;
    double *pos, *mom;   /* private copies, (3, n), original order */
    uint64_t *code;      /* per original particle */
    int64_t *perm;       /* sorted position -> original index */
    int64_t *rank;       /* original index -> sorted position */
    int64_t nn, cap;
    int32_t *level, *nchild;
    int64_t *first, *count, *parent;
    int64_t *child;      /* 8 per node, first nchild used, octant order */
    double *S, *M, *c;   /* per node, 3 each: position sum, moment sum, centroid */
    double *s2;          /* per node: squared side of the cell */
    double *D;           /* per node, 9: first moment D[3k+b] = sum_j (r_j - c)_k m_j,b (order-2 cells) */
} or_tree;

static uint64_t interleave(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint64_t code = 0;
    for (int k = 0; k < OR_BITS; ++k) {
        code |= (uint64_t)((qx >> k) & 1u) << (3 * k + 2);
        code |= (uint64_t)((qy >> k) & 1u) << (3 * k + 1);
        code |= (uint64_t)((qz >> k) & 1u) << (3 * k);
    }
    return code;
}

static uint32_t quantise(double r, double lo, double scale)
{
    double t = (r - lo) * scale;
    double f = floor(t);
    if (f >= (double)OR_QMAX) return OR_QMAX;
    if (f <= 0.0) return 0u;
    return (uint32_t)f;
}

static const uint64_t *g_sort_code;
static int cmp_code_index(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    uint64_t ca = g_sort_code[a], cb = g_sort_code[b];
    if (ca != cb) return ca < cb ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static int64_t new_node(or_tree *t)
{
    if (t->nn == t->cap) {
        int64_t cap = t->cap ? 2 * t->cap : 1024;
        t->level = realloc(t->level, cap * sizeof(int32_t));
        t->nchild = realloc(t->nchild, cap * sizeof(int32_t));
        t->first = realloc(t->first, cap * sizeof(int64_t));
        t->count = realloc(t->count, cap * sizeof(int64_t));
        t->parent = realloc(t->parent, cap * sizeof(int64_t));
        t->child = realloc(t->child, 8 * cap * sizeof(int64_t));
        t->cap = cap;
    }
    return t->nn++;
}

static int64_t build_rec(or_tree *t, int level, int64_t a, int64_t b, int64_t parent)
{
    int64_t id = new_node(t);
    t->level[id] = level;
    t->first[id] = a;
    t->count[id] = b - a;
    t->parent[id] = parent;
    t->nchild[id] = 0;
    if (b - a <= t->leaf || level == OR_MAXLEVEL) return id;
    int shift = 3 * (OR_MAXLEVEL - 1 - level); /* the octant digit of level+1 */
    int64_t s = a;
    for (int o = 0; o < 8; ++o) {
        int64_t e = s;
        while (e < b && (int)((t->code[t->perm[e]] >> shift) & 7u) == o) ++e;
        if (e > s) {
            int64_t ch = build_rec(t, level + 1, s, e, id);
            t->child[8 * id + t->nchild[id]] = ch;
            t->nchild[id] += 1;
        }
        s = e;
    }
    return id;
}

/* Pseudo-particle of every cell, Eq. (magCenter) of Sec. 3.2: moment = vector sum of the members'
 * moments, position = geometric centre of the members.  Sums are formed bottom-up: a leaf sums its
 * members in sorted order starting from +0.0, a parent sums its children in octant order.            */
static void upward_rec(or_tree *t, int64_t id)
{
    int64_t n = t->n;
    double S[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0};
    if (t->nchild[id] == 0) {
        for (int64_t k = t->first[id]; k < t->first[id] + t->count[id]; ++k) {
            int64_t j = t->perm[k];
            for (int a = 0; a < 3; ++a) {
                S[a] = S[a] + t->pos[a * n + j];
                M[a] = M[a] + t->mom[a * n + j];
            }
        }
    } else {
        for (int q = 0; q < t->nchild[id]; ++q) {
            int64_t ch = t->child[8 * id + q];
            upward_rec(t, ch);
            for (int a = 0; a < 3; ++a) {
                S[a] = S[a] + t->S[3 * ch + a];
                M[a] = M[a] + t->M[3 * ch + a];
            }
        }
    }
    for (int a = 0; a < 3; ++a) {
        t->S[3 * id + a] = S[a];
        t->M[3 * id + a] = M[a];
        t->c[3 * id + a] = S[a] / (double)t->count[id];
    }
    double s = ldexp(t->side, -t->level[id]);
    t->s2[id] = s * s;
}

/* First moment of every cell about its pseudo-particle position (beyond the paper: the next term of the
 * cell's expansion, used by the order-2 field).  Taylor-expanding Eq. (H_dip) of a member j at offset
 * x - delta_j (x = r_i - c, delta_j = r_j - c) gives
 *     sum_j T(x - delta_j) m_j = T(x) M - sum_{k,b} d_k T_ab(x) D_kb + O(|delta|^2),
 *     D_kb = sum_j delta_j,k m_j,b ,
 * the first term being the paper's pseudo-particle.  D is formed here straight from that definition,
 * member by member in sorted order, for every cell.                                                    */
static void first_moments(or_tree *t)
{
    int64_t n = t->n;
    t->D = malloc(9 * t->nn * sizeof(double));
    for (int64_t id = 0; id < t->nn; ++id) {
        double D[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t k = t->first[id]; k < t->first[id] + t->count[id]; ++k) {
            int64_t j = t->perm[k];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    D[3 * a + b] += (t->pos[a * n + j] - t->c[3 * id + a]) * t->mom[b * n + j];
        }
        memcpy(&t->D[9 * id], D, sizeof(D));
    }
}

void or_tree_free(or_tree *t)
{
    if (!t) return;
    free(t->pos); free(t->mom); free(t->code); free(t->perm); free(t->rank);
    free(t->level); free(t->nchild); free(t->first); free(t->count); free(t->parent); free(t->child);
    free(t->S); free(t->M); free(t->c); free(t->s2); free(t->D);
    free(t);
}

or_tree *or_tree_build(int64_t n, const double *pos, const double *mom, int leaf)
{
    if (n < 1 || leaf < 1 || !pos || !mom) return NULL;
    or_tree *t = calloc(1, sizeof(or_tree));
    t->n = n;
    t->leaf = leaf;
    t->pos = malloc(3 * n * sizeof(double));
    t->mom = malloc(3 * n * sizeof(double));
    memcpy(t->pos, pos, 3 * n * sizeof(double));
    memcpy(t->mom, mom, 3 * n * sizeof(double));

    /* bounding cube (Sec. 3.2, kernel 1): minimum corner and the largest extent */
    double hi[3];
    for (int a = 0; a < 3; ++a) {
        t->lo[a] = pos[a * n];
        hi[a] = pos[a * n];
        for (int64_t i = 1; i < n; ++i) {
            double v = pos[a * n + i];
            if (v < t->lo[a]) t->lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    }
    t->side = 0.0;
    for (int a = 0; a < 3; ++a) {
        double e = hi[a] - t->lo[a];
        if (e > t->side) t->side = e;
    }
    t->scale = t->side > 0.0 ? 2097152.0 / t->side : 0.0;

    t->code = malloc(n * sizeof(uint64_t));
    for (int64_t i = 0; i < n; ++i) {
        uint32_t qx = quantise(pos[i], t->lo[0], t->scale);
        uint32_t qy = quantise(pos[n + i], t->lo[1], t->scale);
        uint32_t qz = quantise(pos[2 * n + i], t->lo[2], t->scale);
        t->code[i] = interleave(qx, qy, qz);
    }
    t->perm = malloc(n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) t->perm[i] = i;
    g_sort_code = t->code;
    qsort(t->perm, (size_t)n, sizeof(int64_t), cmp_code_index);
    t->rank = malloc(n * sizeof(int64_t));
    for (int64_t k = 0; k < n; ++k) t->rank[t->perm[k]] = k;

    build_rec(t, 0, 0, n, -1);
    t->S = malloc(3 * t->nn * sizeof(double));
    t->M = malloc(3 * t->nn * sizeof(double));
    t->c = malloc(3 * t->nn * sizeof(double));
    t->s2 = malloc(t->nn * sizeof(double));
    upward_rec(t, 0);
    first_moments(t);
    return t;
}

int64_t or_tree_num_nodes(const or_tree *t) { return t ? t->nn : -1; }

/* Export the tree.  Any pointer may be NULL.  bbox = (lo_x, lo_y, lo_z, side, scale). */
void or_tree_export(const or_tree *t, double *bbox, uint64_t *code, int64_t *perm, int32_t *level,
                    int64_t *first, int64_t *count, int32_t *nchild, int64_t *child8, int64_t *parent,
                    double *S, double *M, double *c, double *s2)
{
    int64_t n = t->n, nn = t->nn;
    if (bbox) { bbox[0] = t->lo[0]; bbox[1] = t->lo[1]; bbox[2] = t->lo[2]; bbox[3] = t->side;
                bbox[4] = t->scale; }
    if (code) memcpy(code, t->code, n * sizeof(uint64_t));
    if (perm) memcpy(perm, t->perm, n * sizeof(int64_t));
    if (level) memcpy(level, t->level, nn * sizeof(int32_t));
    if (first) memcpy(first, t->first, nn * sizeof(int64_t));
    if (count) memcpy(count, t->count, nn * sizeof(int64_t));
    if (nchild) memcpy(nchild, t->nchild, nn * sizeof(int32_t));
    if (child8) {
        for (int64_t i = 0; i < nn; ++i)
            for (int q = 0; q < 8; ++q) child8[8 * i + q] = q < t->nchild[i] ? t->child[8 * i + q] : -1;
    }
    if (parent) memcpy(parent, t->parent, nn * sizeof(int64_t));
    if (S) memcpy(S, t->S, 3 * nn * sizeof(double));
    if (M) memcpy(M, t->M, 3 * nn * sizeof(double));
    if (c) memcpy(c, t->c, 3 * nn * sizeof(double));
    if (s2) memcpy(s2, t->s2, nn * sizeof(double));
}

/* First moments of every cell, (nn, 9) row-major D[3k+b]. */
void or_tree_export_D(const or_tree *t, double *D)
{
    memcpy(D, t->D, 9 * t->nn * sizeof(double));
}

/* ------------------------------------------------------------------------------------------------ */
/* Traversal (Sec. 3.2): starting at the root, a cell that is far enough from the target is replaced  */
/* by its pseudo-particle; otherwise its sub-cells are examined, down to the leaves, whose particles  */
/* interact directly.  The paper gives no criterion; the reading used here, per target i:            */
/*   - a cell containing i is always opened (a leaf containing i: direct sum over its other members); */
/*   - otherwise the cell is accepted iff s^2 < (theta*theta) * d^2, with s the cell side and          */
/*     d^2 = fma(dz,dz, fma(dy,dy, dx*dx)), dx = x_i - cx (the pseudo-particle position);            */
/*   - an unaccepted leaf contributes all its members directly; an unaccepted parent is opened.        */
/* Sub-cells are visited in octant order, members in sorted order, contributions summed in visit order.*/
/* ------------------------------------------------------------------------------------------------ */

typedef struct {
    const or_tree *t;
    double theta2;
    int order;       /* 1: the paper's pseudo-particle; 2: plus the first-moment term (forward only) */
    int64_t si;      /* target's sorted position */
    double ri[3];
    /* forward */
    double H[3];
    int64_t n_far, n_near;
    /* adjoint (NULL when not used) */
    const double *hbar;  /* the target's upstream gradient (3) */
    double gr[3];        /* gathered d/dr_i */
    double *A, *B;       /* per-node accumulators (3 * nn) */
    double *E;           /* order 2: per-node first-moment adjoint accumulators (9 * nn) */
    double *sr, *sm;     /* per-particle scatters (3, n), original order */
    /* list recording (NULL when not used) */
    int64_t *far_out, *near_out;
} visit_ctx;

/* Field of a cell's first moment D at offset x from its pseudo-particle: h_a = -sum_{k,b} d_k T_ab(x) D_kb
 * with T_ab(x) = 3 x_a x_b / |x|^5 - delta_ab / |x|^3 (the tensor of Eq. H_dip), whose derivative is
 *     d_k T_ab = 3 (delta_ak x_b + delta_bk x_a + delta_ab x_k) / |x|^5 - 15 x_a x_b x_k / |x|^7 ,
 * so that, with u = D x (u_a = sum_b D_ab x_b), w = D^T x, tr D and q = x.D x,
 *     h = -3 (u + w + x tr D) / |x|^5 + 15 q x / |x|^7 .                                              */
static void first_moment_field(const double x[3], const double D[9], double h[3])
{
    double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    double r = sqrt(r2);
    double r5 = r2 * r2 * r;
    double r7 = r5 * r2;
    double u[3], w[3], tr = D[0] + D[4] + D[8], q = 0.0;
    for (int a = 0; a < 3; ++a) {
        u[a] = D[3 * a] * x[0] + D[3 * a + 1] * x[1] + D[3 * a + 2] * x[2];
        w[a] = D[a] * x[0] + D[3 + a] * x[1] + D[6 + a] * x[2];
    }
    for (int a = 0; a < 3; ++a) q += x[a] * u[a];
    for (int a = 0; a < 3; ++a) h[a] = -3.0 * (u[a] + w[a] + x[a] * tr) / r5 + 15.0 * q * x[a] / r7;
}

/* Third and fourth derivatives of phi = 1/|x| (T_ab = d_a d_b phi is the tensor of Eq. H_dip):
 *   P_abk  = d_a d_b d_k phi = 3 (delta_ab x_k + delta_ak x_b + delta_bk x_a) / r^5 - 15 x_a x_b x_k / r^7,
 *   Q_abkl = d_l P_abk = 105 x_a x_b x_k x_l / r^9
 *            - 15 (delta_ab x_k x_l + delta_ak x_b x_l + delta_bk x_a x_l
 *                  + delta_al x_b x_k + delta_bl x_a x_k + delta_kl x_a x_b) / r^7
 *            + 3 (delta_ab delta_kl + delta_ak delta_bl + delta_bk delta_al) / r^5 .                      */
static void phi3(const double x[3], double P[27])
{
    double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    double r = sqrt(r2);
    double r5 = r2 * r2 * r, r7 = r5 * r2;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int k = 0; k < 3; ++k)
                P[(3 * a + b) * 3 + k] = 3.0 * ((a == b) * x[k] + (a == k) * x[b] + (b == k) * x[a]) / r5 -
                                         15.0 * x[a] * x[b] * x[k] / r7;
}

static void phi4(const double x[3], double Q[81])
{
    double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    double r = sqrt(r2);
    double r5 = r2 * r2 * r, r7 = r5 * r2, r9 = r7 * r2;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double t4 = 105.0 * x[a] * x[b] * x[k] * x[l] / r9;
                    double t2 = ((a == b) * x[k] * x[l] + (a == k) * x[b] * x[l] + (b == k) * x[a] * x[l] +
                                 (a == l) * x[b] * x[k] + (b == l) * x[a] * x[k] + (k == l) * x[a] * x[b]) / r7;
                    double t0 = ((a == b) * (k == l) + (a == k) * (b == l) + (b == k) * (a == l)) / r5;
                    Q[((3 * a + b) * 3 + k) * 3 + l] = t4 - 15.0 * t2 + 3.0 * t0;
                }
}

/* Adjoint of one order-2 cell term Lambda = u . h_D(x), h_D,a = -sum_{k,b} P_abk D_kb, for u = the
 * target's upstream gradient: d Lambda / d x_l = -sum_{a,b,k} u_a D_kb Q_abkl (to the target, and with
 * the opposite sign to the cell's centre) and d Lambda / d D_kb = -sum_a u_a P_abk.                     */
static void first_moment_adjoint(const double x[3], const double D[9], const double u[3], double G[3],
                                 double E[9])
{
    double P[27], Q[81];
    phi3(x, P);
    phi4(x, Q);
    for (int l = 0; l < 3; ++l) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int k = 0; k < 3; ++k) s += u[a] * D[3 * k + b] * Q[((3 * a + b) * 3 + k) * 3 + l];
        G[l] = -s;
    }
    for (int k = 0; k < 3; ++k)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a) s += u[a] * P[(3 * a + b) * 3 + k];
            E[3 * k + b] = -s;
        }
}

static void do_far(visit_ctx *v, int64_t id)
{
    const or_tree *t = v->t;
    double x[3], h[3];
    for (int a = 0; a < 3; ++a) x[a] = v->ri[a] - t->c[3 * id + a];
    if (v->far_out) v->far_out[v->n_far] = id;
    v->n_far += 1;
    if (!v->hbar) {
        dip_field(x, &t->M[3 * id], h);
        for (int a = 0; a < 3; ++a) v->H[a] += h[a];
        if (v->order == 2) {
            first_moment_field(x, &t->D[9 * id], h);
            for (int a = 0; a < 3; ++a) v->H[a] += h[a];
        }
    } else {
        double g[3];
        grad_kernel(x, v->hbar, &t->M[3 * id], g);
        dip_field(x, v->hbar, h); /* T(x) hbar: T is symmetric */
        for (int a = 0; a < 3; ++a) {
            v->gr[a] += g[a];
            v->B[3 * id + a] -= g[a];
            v->A[3 * id + a] += h[a];
        }
        if (v->order == 2) {
            double G[3], E[9];
            first_moment_adjoint(x, &t->D[9 * id], v->hbar, G, E);
            for (int a = 0; a < 3; ++a) {
                v->gr[a] += G[a];
                v->B[3 * id + a] -= G[a];
            }
            for (int q = 0; q < 9; ++q) v->E[9 * id + q] += E[q];
        }
    }
}

static void do_near(visit_ctx *v, int64_t id)
{
    const or_tree *t = v->t;
    int64_t n = t->n;
    for (int64_t k = t->first[id]; k < t->first[id] + t->count[id]; ++k) {
        if (k == v->si) continue;
        int64_t j = t->perm[k];
        double x[3], mj[3], h[3];
        for (int a = 0; a < 3; ++a) {
            x[a] = v->ri[a] - t->pos[a * n + j];
            mj[a] = t->mom[a * n + j];
        }
        if (v->near_out) v->near_out[v->n_near] = j;
        v->n_near += 1;
        if (!v->hbar) {
            dip_field(x, mj, h);
            for (int a = 0; a < 3; ++a) v->H[a] += h[a];
        } else {
            double g[3];
            grad_kernel(x, v->hbar, mj, g);
            dip_field(x, v->hbar, h);
            for (int a = 0; a < 3; ++a) {
                v->gr[a] += g[a];
                v->sr[a * n + j] -= g[a];
                v->sm[a * n + j] += h[a];
            }
        }
    }
}

static int mac_accept(const visit_ctx *v, int64_t id)
{
    const or_tree *t = v->t;
    double dx = v->ri[0] - t->c[3 * id + 0];
    double dy = v->ri[1] - t->c[3 * id + 1];
    double dz = v->ri[2] - t->c[3 * id + 2];
    double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
    return t->s2[id] < v->theta2 * d2;
}

static void visit(visit_ctx *v, int64_t id)
{
    const or_tree *t = v->t;
    int contains = t->first[id] <= v->si && v->si < t->first[id] + t->count[id];
    if (!contains && mac_accept(v, id)) {
        do_far(v, id);
        return;
    }
    if (t->nchild[id] == 0) {
        do_near(v, id);
        return;
    }
    for (int q = 0; q < t->nchild[id]; ++q) visit(v, t->child[8 * id + q]);
}

static void ctx_init(visit_ctx *v, const or_tree *t, double theta, int64_t i)
{
    memset(v, 0, sizeof(*v));
    v->t = t;
    v->order = 1;
    v->theta2 = theta * theta;
    v->si = t->rank[i];
    load3(t->pos, t->n, i, v->ri);
}

/* Barnes-Hut field on all particles (original order) plus per-target interaction counts. */
int or_bh_field(const or_tree *t, double theta, double *H, int64_t *n_far, int64_t *n_near)
{
    if (!t || !(theta >= 0.0)) return -1;
    int64_t n = t->n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        visit_ctx v;
        ctx_init(&v, t, theta, i);
        visit(&v, 0);
        for (int a = 0; a < 3; ++a) H[a * n + i] = v.H[a];
        if (n_far) n_far[i] = v.n_far;
        if (n_near) n_near[i] = v.n_near;
    }
    return 0;
}

/* Barnes-Hut field with cells of the given order (1: Eq. magCenter pseudo-particles, the paper's
 * scheme; 2: plus each accepted cell's first-moment term), all particles, original order. */
int or_bh_field_order(const or_tree *t, double theta, int order, double *H, int64_t *n_far, int64_t *n_near)
{
    if (!t || !(theta >= 0.0) || (order != 1 && order != 2)) return -1;
    int64_t n = t->n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        visit_ctx v;
        ctx_init(&v, t, theta, i);
        v.order = order;
        visit(&v, 0);
        for (int a = 0; a < 3; ++a) H[a * n + i] = v.H[a];
        if (n_far) n_far[i] = v.n_far;
        if (n_near) n_near[i] = v.n_near;
    }
    return 0;
}

/* Barnes-Hut field for a subset of targets (original indices); rows follow `targets`. */
int or_bh_field_subset(const or_tree *t, double theta, int64_t nt, const int64_t *targets,
                       double *H_out, int64_t *n_far, int64_t *n_near)
{
    if (!t || !(theta >= 0.0)) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nt; ++q) {
        visit_ctx v;
        ctx_init(&v, t, theta, targets[q]);
        visit(&v, 0);
        for (int a = 0; a < 3; ++a) H_out[a * nt + q] = v.H[a];
        if (n_far) n_far[q] = v.n_far;
        if (n_near) n_near[q] = v.n_near;
    }
    return 0;
}

/* Interaction lists (frozen structure).  Call once with far_node = near_idx = NULL to get the per-
 * target counts in far_ptr[1..n], near_ptr[1..n] (far_ptr[0] = near_ptr[0] = 0, prefix sums), then
 * again with the arrays sized far_ptr[n], near_ptr[n].  far_node holds node ids, near_idx original
 * particle indices.                                                                                  */
int or_bh_lists(const or_tree *t, double theta, int64_t *far_ptr, int64_t *far_node,
                int64_t *near_ptr, int64_t *near_idx)
{
    int64_t n = t->n;
    if (!far_node || !near_idx) {
        far_ptr[0] = near_ptr[0] = 0;
        for (int64_t i = 0; i < n; ++i) {
            visit_ctx v;
            ctx_init(&v, t, theta, i);
            visit(&v, 0);
            far_ptr[i + 1] = far_ptr[i] + v.n_far;
            near_ptr[i + 1] = near_ptr[i] + v.n_near;
        }
        return 0;
    }
    for (int64_t i = 0; i < n; ++i) {
        visit_ctx v;
        ctx_init(&v, t, theta, i);
        v.far_out = far_node + far_ptr[i];
        v.near_out = near_idx + near_ptr[i];
        visit(&v, 0);
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------------ */
/* Adjoint.  With the tree, the membership of every cell and every acceptance decision held fixed,   */
/* H_i = sum_{C in F_i} T(r_i - c_C) M_C + sum_{k in N_i} T(r_i - r_k) m_k, c_C = mean of the members'*/
/* positions, M_C = sum of their moments (Eq. magCenter).  For L = sum_i Hbar_i . H_i the exact       */
/* reverse-mode derivative is                                                                          */
/*   far (i, C):  dL/dr_i += g(x; Hbar_i, M_C),  dL/dr_k -= g / n_C and dL/dm_k += T(x) Hbar_i for   */
/*                every member k of C  (x = r_i - c_C);                                               */
/*   near (i, k): dL/dr_i += g(x; Hbar_i, m_k),  dL/dr_k -= g,  dL/dm_k += T(x) Hbar_i.               */
/* g is the gradient kernel (the f_dip summand of Sec. 2); T is symmetric, so T(x)^T Hbar = T(x) Hbar.*/
/* ------------------------------------------------------------------------------------------------ */

int or_bh_vjp(const or_tree *t, double theta, const double *hbar, double *dLdr, double *dLdm)
{
    if (!t || !(theta >= 0.0) || !hbar || !dLdr || !dLdm) return -1;
    int64_t n = t->n, nn = t->nn;
    int nth = omp_get_max_threads();
    double *A = calloc((size_t)nth * 3 * nn, sizeof(double));
    double *B = calloc((size_t)nth * 3 * nn, sizeof(double));
    double *sr = calloc((size_t)nth * 3 * n, sizeof(double));
    double *sm = calloc((size_t)nth * 3 * n, sizeof(double));
    double *gather = calloc((size_t)3 * n, sizeof(double));
    if (!A || !B || !sr || !sm || !gather) {
        free(A); free(B); free(sr); free(sm); free(gather);
        return -2;
    }
#pragma omp parallel num_threads(nth)
    {
        int tid = omp_get_thread_num();
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            visit_ctx v;
            double hb[3];
            ctx_init(&v, t, theta, i);
            load3(hbar, n, i, hb);
            v.hbar = hb;
            v.A = A + (size_t)tid * 3 * nn;
            v.B = B + (size_t)tid * 3 * nn;
            v.sr = sr + (size_t)tid * 3 * n;
            v.sm = sm + (size_t)tid * 3 * n;
            visit(&v, 0);
            for (int a = 0; a < 3; ++a) gather[a * n + i] = v.gr[a];
        }
    }
    /* reduce thread-private accumulators in thread order */
    for (int q = 1; q < nth; ++q) {
        for (int64_t x = 0; x < 3 * nn; ++x) {
            A[x] += A[(size_t)q * 3 * nn + x];
            B[x] += B[(size_t)q * 3 * nn + x];
        }
        for (int64_t x = 0; x < 3 * n; ++x) {
            sr[x] += sr[(size_t)q * 3 * n + x];
            sm[x] += sm[(size_t)q * 3 * n + x];
        }
    }
    /* distribute cell adjoints to members: every member of C receives A_C and B_C / n_C */
    for (int64_t i = 0; i < 3 * n; ++i) {
        dLdr[i] = gather[i] + sr[i];
        dLdm[i] = sm[i];
    }
    for (int64_t id = 0; id < nn; ++id) {
        double inv = 1.0 / (double)t->count[id];
        for (int64_t k = t->first[id]; k < t->first[id] + t->count[id]; ++k) {
            int64_t j = t->perm[k];
            for (int a = 0; a < 3; ++a) {
                dLdm[a * n + j] += A[3 * id + a];
                dLdr[a * n + j] += B[3 * id + a] * inv;
            }
        }
    }
    free(A); free(B); free(sr); free(sm); free(gather);
    return 0;
}

/* Adjoint with cells of the given order (see or_bh_field_order).  Order 2 adds, per accepted cell, the
 * first-moment term's gradient to the target and the cell centre, and accumulates dL/dD_C (E_C); since
 * D_C = sum_j (r_j - c_C) m_j^T with c_C the members' mean, every member j of C then receives
 *     dL/dr_j += E_C m_j - E_C M_C / n_C ,   dL/dm_j += E_C^T (r_j - c_C) .                              */
int or_bh_vjp_order(const or_tree *t, double theta, int order, const double *hbar, double *dLdr, double *dLdm)
{
    if (!t || !(theta >= 0.0) || !hbar || !dLdr || !dLdm || (order != 1 && order != 2)) return -1;
    int64_t n = t->n, nn = t->nn;
    int nth = omp_get_max_threads();
    double *A = calloc((size_t)nth * 3 * nn, sizeof(double));
    double *B = calloc((size_t)nth * 3 * nn, sizeof(double));
    double *E = calloc((size_t)nth * 9 * nn, sizeof(double));
    double *sr = calloc((size_t)nth * 3 * n, sizeof(double));
    double *sm = calloc((size_t)nth * 3 * n, sizeof(double));
    double *gather = calloc((size_t)3 * n, sizeof(double));
    if (!A || !B || !E || !sr || !sm || !gather) {
        free(A); free(B); free(E); free(sr); free(sm); free(gather);
        return -2;
    }
#pragma omp parallel num_threads(nth)
    {
        int tid = omp_get_thread_num();
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            visit_ctx v;
            double hb[3];
            ctx_init(&v, t, theta, i);
            v.order = order;
            load3(hbar, n, i, hb);
            v.hbar = hb;
            v.A = A + (size_t)tid * 3 * nn;
            v.B = B + (size_t)tid * 3 * nn;
            v.E = E + (size_t)tid * 9 * nn;
            v.sr = sr + (size_t)tid * 3 * n;
            v.sm = sm + (size_t)tid * 3 * n;
            visit(&v, 0);
            for (int a = 0; a < 3; ++a) gather[a * n + i] = v.gr[a];
        }
    }
    for (int q = 1; q < nth; ++q) {
        for (int64_t x = 0; x < 3 * nn; ++x) {
            A[x] += A[(size_t)q * 3 * nn + x];
            B[x] += B[(size_t)q * 3 * nn + x];
        }
        for (int64_t x = 0; x < 9 * nn; ++x) E[x] += E[(size_t)q * 9 * nn + x];
        for (int64_t x = 0; x < 3 * n; ++x) {
            sr[x] += sr[(size_t)q * 3 * n + x];
            sm[x] += sm[(size_t)q * 3 * n + x];
        }
    }
    for (int64_t i = 0; i < 3 * n; ++i) {
        dLdr[i] = gather[i] + sr[i];
        dLdm[i] = sm[i];
    }
    for (int64_t id = 0; id < nn; ++id) {
        double inv = 1.0 / (double)t->count[id];
        const double *Ec = &E[9 * id], *Mc = &t->M[3 * id], *cc = &t->c[3 * id];
        double EM[3];
        for (int k = 0; k < 3; ++k) EM[k] = Ec[3 * k] * Mc[0] + Ec[3 * k + 1] * Mc[1] + Ec[3 * k + 2] * Mc[2];
        for (int64_t q = t->first[id]; q < t->first[id] + t->count[id]; ++q) {
            int64_t j = t->perm[q];
            for (int a = 0; a < 3; ++a) {
                dLdm[a * n + j] += A[3 * id + a];
                dLdr[a * n + j] += B[3 * id + a] * inv;
            }
            if (order == 2) {
                double mj[3], dj[3];
                load3(t->mom, n, j, mj);
                for (int a = 0; a < 3; ++a) dj[a] = t->pos[a * n + j] - cc[a];
                for (int k = 0; k < 3; ++k)
                    dLdr[k * n + j] += Ec[3 * k] * mj[0] + Ec[3 * k + 1] * mj[1] + Ec[3 * k + 2] * mj[2] - EM[k] * inv;
                for (int b = 0; b < 3; ++b)
                    dLdm[b * n + j] += Ec[b] * dj[0] + Ec[3 + b] * dj[1] + Ec[6 + b] * dj[2];
            }
        }
    }
    free(A); free(B); free(E); free(sr); free(sm); free(gather);
    return 0;
}

/* ------------------------------------------------------------------------------------------------ */
/* Frozen-structure energy and its finite-difference gradient.                                        */
/* The structure is: node membership (first/count over the sorted order `perm`) and the lists of      */
/* accepted cells and direct partners of every target.  Pseudo-particles are recomputed from the      */
/* given (pos, mom), so this is the function whose exact gradient the adjoint returns.                */
/* ------------------------------------------------------------------------------------------------ */

static double energy_frozen_order(int64_t n, const double *pos, const double *mom, const double *hext,
                                  int64_t nn, const int64_t *first, const int64_t *count, const int64_t *perm,
                                  const int64_t *far_ptr, const int64_t *far_node, const int64_t *near_ptr,
                                  const int64_t *near_idx, int order, double *scratch /* 15 * nn */);

double or_energy_frozen(int64_t n, const double *pos, const double *mom, const double *hext,
                        int64_t nn, const int64_t *first, const int64_t *count, const int64_t *perm,
                        const int64_t *far_ptr, const int64_t *far_node, const int64_t *near_ptr,
                        const int64_t *near_idx, double *scratch /* 6 * nn */)
{
    return energy_frozen_order(n, pos, mom, hext, nn, first, count, perm, far_ptr, far_node, near_ptr, near_idx,
                               1, scratch);
}

/* Frozen-structure energy with cells of the given order (order 2: each far cell also contributes its
 * first moment, recomputed from (pos, mom) about the recomputed centre). */
double or_energy_frozen_order(int64_t n, const double *pos, const double *mom, const double *hext,
                              int64_t nn, const int64_t *first, const int64_t *count, const int64_t *perm,
                              const int64_t *far_ptr, const int64_t *far_node, const int64_t *near_ptr,
                              const int64_t *near_idx, int order, double *scratch /* 15 * nn */)
{
    return energy_frozen_order(n, pos, mom, hext, nn, first, count, perm, far_ptr, far_node, near_ptr, near_idx,
                               order, scratch);
}

static double energy_frozen_order(int64_t n, const double *pos, const double *mom, const double *hext,
                                  int64_t nn, const int64_t *first, const int64_t *count, const int64_t *perm,
                                  const int64_t *far_ptr, const int64_t *far_node, const int64_t *near_ptr,
                                  const int64_t *near_idx, int order, double *scratch)
{
    double *c = scratch, *M = scratch + 3 * nn, *D = scratch + 6 * nn;
    for (int64_t id = 0; id < nn; ++id) {
        double S[3] = {0.0, 0.0, 0.0}, Ms[3] = {0.0, 0.0, 0.0};
        for (int64_t k = first[id]; k < first[id] + count[id]; ++k) {
            int64_t j = perm[k];
            for (int a = 0; a < 3; ++a) {
                S[a] += pos[a * n + j];
                Ms[a] += mom[a * n + j];
            }
        }
        for (int a = 0; a < 3; ++a) {
            c[3 * id + a] = S[a] / (double)count[id];
            M[3 * id + a] = Ms[a];
        }
        if (order == 2) {
            double Dc[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int64_t k = first[id]; k < first[id] + count[id]; ++k) {
                int64_t j = perm[k];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) Dc[3 * a + b] += (pos[a * n + j] - c[3 * id + a]) * mom[b * n + j];
            }
            memcpy(&D[9 * id], Dc, sizeof(Dc));
        }
    }
    double e_dip = 0.0, e_ext = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double ri[3], mi[3], H[3] = {0.0, 0.0, 0.0}, x[3], h[3], mj[3];
        load3(pos, n, i, ri);
        load3(mom, n, i, mi);
        for (int64_t q = far_ptr[i]; q < far_ptr[i + 1]; ++q) {
            int64_t id = far_node[q];
            for (int a = 0; a < 3; ++a) x[a] = ri[a] - c[3 * id + a];
            dip_field(x, &M[3 * id], h);
            for (int a = 0; a < 3; ++a) H[a] += h[a];
            if (order == 2) {
                first_moment_field(x, &D[9 * id], h);
                for (int a = 0; a < 3; ++a) H[a] += h[a];
            }
        }
        for (int64_t q = near_ptr[i]; q < near_ptr[i + 1]; ++q) {
            int64_t j = near_idx[q];
            for (int a = 0; a < 3; ++a) x[a] = ri[a] - pos[a * n + j];
            load3(mom, n, j, mj);
            dip_field(x, mj, h);
            for (int a = 0; a < 3; ++a) H[a] += h[a];
        }
        for (int a = 0; a < 3; ++a) {
            e_dip += mi[a] * H[a];
            e_ext += mi[a] * (hext ? hext[a] : 0.0);
        }
    }
    return -0.5 * e_dip - e_ext;
}

/* Central differences of the frozen-structure energy (cells of the given order) in every coordinate of
 * pos and mom (step h). */
int or_fd_grad_frozen_order(int64_t n, const double *pos, const double *mom, const double *hext,
                            int64_t nn, const int64_t *first, const int64_t *count, const int64_t *perm,
                            const int64_t *far_ptr, const int64_t *far_node, const int64_t *near_ptr,
                            const int64_t *near_idx, double h, int order, double *dEdr, double *dEdm);

int or_fd_grad_frozen(int64_t n, const double *pos, const double *mom, const double *hext,
                      int64_t nn, const int64_t *first, const int64_t *count, const int64_t *perm,
                      const int64_t *far_ptr, const int64_t *far_node, const int64_t *near_ptr,
                      const int64_t *near_idx, double h, double *dEdr, double *dEdm)
{
    return or_fd_grad_frozen_order(n, pos, mom, hext, nn, first, count, perm, far_ptr, far_node, near_ptr,
                                   near_idx, h, 1, dEdr, dEdm);
}

int or_fd_grad_frozen_order(int64_t n, const double *pos, const double *mom, const double *hext,
                            int64_t nn, const int64_t *first, const int64_t *count, const int64_t *perm,
                            const int64_t *far_ptr, const int64_t *far_node, const int64_t *near_ptr,
                            const int64_t *near_idx, double h, int order, double *dEdr, double *dEdm)
{
#pragma omp parallel
    {
        double *p = malloc(3 * n * sizeof(double));
        double *m = malloc(3 * n * sizeof(double));
        double *scr = malloc(15 * nn * sizeof(double));
        memcpy(p, pos, 3 * n * sizeof(double));
        memcpy(m, mom, 3 * n * sizeof(double));
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < 6 * n; ++q) {
            double *arr = q < 3 * n ? p : m;
            int64_t x = q < 3 * n ? q : q - 3 * n;
            double keep = arr[x];
            arr[x] = keep + h;
            double ep = energy_frozen_order(n, p, m, hext, nn, first, count, perm, far_ptr, far_node,
                                            near_ptr, near_idx, order, scr);
            arr[x] = keep - h;
            double em = energy_frozen_order(n, p, m, hext, nn, first, count, perm, far_ptr, far_node,
                                            near_ptr, near_idx, order, scr);
            arr[x] = keep;
            double d = (ep - em) / (2.0 * h);
            if (q < 3 * n) dEdr[x] = d; else dEdm[x] = d;
        }
        free(p); free(m); free(scr);
    }
    return 0;
}

int or_num_threads(void) { return omp_get_max_threads(); }
