/*
 * stokes_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the Stokeslet/stresslet treecode of
 * Wang, Tlupova & Krasny, "A Treecode Algorithm for 3D Stokeslets and Stresslets"
 * (arXiv 1811.12498).  It exists to check the HIP library; it shares no code,
 * header, table or helper with it.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  The product path never does.
 *
 * Build:  gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared  (no FMA contraction,
 * so every geometric quantity below is the correctly rounded IEEE result of the
 * expression as written).
 *
 * Conventions (readings of the paper, each one also listed in the design notes):
 *   - kernels exactly as printed in the introduction (eqs. Stokeslet, stresslet),
 *     no 1/(8 pi) prefactor, T positive;
 *   - d = x - y: target minus source (or minus cluster centre);
 *   - a pair is skipped iff |d|^2 == 0 (the n != m exclusion of eq. StoStre);
 *   - flattened moment order is graded-lex: n = 0..p, k1 = n..0, k2 = n-k1..0;
 *   - octree on the root cube [lo, lo+L]^3 (lo = componentwise min, L = largest
 *     extent) via 21-bit integer coordinates q = floor((y-lo) * (2^21/L));
 *     a node is split iff it holds more than N0 particles and its level < 21;
 *     children in Morton order (x bit most significant); empty children dropped;
 *   - cluster centre y_c = centre of the tight bounding box of the node's
 *     particles; radius r = max |y - y_c| over those particles (Sec. 2, Fig. 1
 *     caption; box shrinking of Sec. 6 test case 1);
 *   - MAC: R > 0 and r <= theta * R (eq. MAC, evaluated without division).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_LEVEL 21

/* ------------------------------------------------------------------------- */
/* Multi-index bookkeeping (Sec. 2 multi-index conventions; Sec. 6 flattening) */
/* ------------------------------------------------------------------------- */

int orc_nm(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

/* Graded-lex table of all k with ||k|| <= p, the "fixed order" of the
 * flattened moment arrays (Sec. 6, memory discussion). */
void orc_kindex(int p, int32_t *k)
{
    int a = 0;
    for (int n = 0; n <= p; n++)
        for (int k1 = n; k1 >= 0; k1--)
            for (int k2 = n - k1; k2 >= 0; k2--) {
                k[3 * a + 0] = k1;
                k[3 * a + 1] = k2;
                k[3 * a + 2] = n - k1 - k2;
                a++;
            }
}

static double ipow(double x, int k)
{
    double r = 1.0;
    for (int i = 0; i < k; i++) r *= x;
    return r;
}

/* (y - y_c)^k with the multi-index power convention of Sec. 2. */
static double monomial(const double dy[3], int k1, int k2, int k3)
{
    return ipow(dy[0], k1) * ipow(dy[1], k2) * ipow(dy[2], k3);
}

/* ------------------------------------------------------------------------- */
/* Coulomb Taylor coefficients b^k (Sec. 3, eqs. GreenFunc and recurrence_1) */
/* ------------------------------------------------------------------------- */

/* Dense storage: b[(k1*(P+1)+k2)*(P+1)+k3] for ||k|| <= P. */
static double bget(const double *b, int P, int k1, int k2, int k3)
{
    if (k1 < 0 || k2 < 0 || k3 < 0 || k1 + k2 + k3 > P) return 0.0;
    return b[(k1 * (P + 1) + k2) * (P + 1) + k3];
}

/* b^k(x, y) = (1/k!) D_y^k 1/|x - y| for all ||k|| <= P, with d = x - y.
 * b^0 = G; b^k = 0 for any negative index; for ||k|| = n >= 1 the recurrence
 *   n |d|^2 b^k = (2n-1) sum_i d_i b^{k-e_i} - (n-1) sum_i b^{k-2e_i}. */
void orc_coulomb_taylor(const double d[3], int P, double *b)
{
    const int S = P + 1;
    memset(b, 0, sizeof(double) * (size_t)S * S * S);
    const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    b[0] = 1.0 / sqrt(R2);
    for (int n = 1; n <= P; n++)
        for (int k1 = n; k1 >= 0; k1--)
            for (int k2 = n - k1; k2 >= 0; k2--) {
                const int k3 = n - k1 - k2;
                const double s1 = d[0] * bget(b, P, k1 - 1, k2, k3) +
                                  d[1] * bget(b, P, k1, k2 - 1, k3) +
                                  d[2] * bget(b, P, k1, k2, k3 - 1);
                const double s2 = bget(b, P, k1 - 2, k2, k3) + bget(b, P, k1, k2 - 2, k3) +
                                  bget(b, P, k1, k2, k3 - 2);
                b[(k1 * S + k2) * S + k3] = ((2.0 * n - 1.0) * s1 - (n - 1.0) * s2) / (n * R2);
            }
}

/* b at k + (shift vector) */
static double bsh(const double *b, int P, const int k[3], int s0, int s1, int s2)
{
    return bget(b, P, k[0] + s0, k[1] + s1, k[2] + s2);
}

static int delta(int i, int j) { return i == j ? 1 : 0; }

/* unit vector components */
static void ev(int i, int e[3]) { e[0] = (i == 0); e[1] = (i == 1); e[2] = (i == 2); }

/* Stokeslet Taylor coefficients a^k_ij for ||k|| <= p from the b's
 * (Sec. 3, eq. recurrence_2):
 *   a^k_ij = delta_ij b^k + d_j (k_i+1) b^{k+e_i} - (k_i+1-delta_ij) b^{k+e_i-e_j}.
 * Output layout a[(a_index*3 + i)*3 + j]. */
static void stokeslet_coeffs_from_b(const double d[3], int p, const double *b, int P, double *out)
{
    const int nm = orc_nm(p);
    int32_t *kk = malloc(sizeof(int32_t) * 3 * nm);
    orc_kindex(p, kk);
    for (int a = 0; a < nm; a++) {
        const int k[3] = {kk[3 * a], kk[3 * a + 1], kk[3 * a + 2]};
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                int ei[3], ej[3];
                ev(i, ei);
                ev(j, ej);
                double v = delta(i, j) * bsh(b, P, k, 0, 0, 0) +
                           d[j] * (k[i] + 1) * bsh(b, P, k, ei[0], ei[1], ei[2]) -
                           (k[i] + 1 - delta(i, j)) *
                               bsh(b, P, k, ei[0] - ej[0], ei[1] - ej[1], ei[2] - ej[2]);
                out[(a * 3 + i) * 3 + j] = v;
            }
    }
    free(kk);
}

/* Stresslet Taylor coefficients (Sec. 3, eq. recurrence_3):
 *   3 at^k_ijl = d_l (k_i+1)(k_j+1+delta_ij) b^{k+e_i+e_j}
 *              - (k_i+1-delta_il)(k_j+1+delta_ij-delta_jl) b^{k+e_i+e_j-e_l}
 *              + delta_ij (k_l+1) b^{k+e_l}.
 * Output layout at[((a*3 + i)*3 + j)*3 + l]. */
static void stresslet_coeffs_from_b(const double d[3], int p, const double *b, int P, double *out)
{
    const int nm = orc_nm(p);
    int32_t *kk = malloc(sizeof(int32_t) * 3 * nm);
    orc_kindex(p, kk);
    for (int a = 0; a < nm; a++) {
        const int k[3] = {kk[3 * a], kk[3 * a + 1], kk[3 * a + 2]};
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                for (int l = 0; l < 3; l++) {
                    int ei[3], ej[3], el[3];
                    ev(i, ei);
                    ev(j, ej);
                    ev(l, el);
                    double v = d[l] * (k[i] + 1) * (k[j] + 1 + delta(i, j)) *
                                   bsh(b, P, k, ei[0] + ej[0], ei[1] + ej[1], ei[2] + ej[2]) -
                               (k[i] + 1 - delta(i, l)) * (k[j] + 1 + delta(i, j) - delta(j, l)) *
                                   bsh(b, P, k, ei[0] + ej[0] - el[0], ei[1] + ej[1] - el[1],
                                       ei[2] + ej[2] - el[2]) +
                               delta(i, j) * (k[l] + 1) * bsh(b, P, k, el[0], el[1], el[2]);
                    out[((a * 3 + i) * 3 + j) * 3 + l] = v / 3.0;
                }
    }
    free(kk);
}

/* Public: explicit a^k_ij and at^k_ijl at d = x - y_c (for pins only). */
void orc_stokeslet_coeffs(const double d[3], int p, double *a)
{
    const int P = p + 1, S = P + 1;
    double *b = malloc(sizeof(double) * S * S * S);
    orc_coulomb_taylor(d, P, b);
    stokeslet_coeffs_from_b(d, p, b, P, a);
    free(b);
}

void orc_stresslet_coeffs(const double d[3], int p, double *at)
{
    const int P = p + 2, S = P + 1;
    double *b = malloc(sizeof(double) * S * S * S);
    orc_coulomb_taylor(d, P, b);
    stresslet_coeffs_from_b(d, p, b, P, at);
    free(b);
}

/* ------------------------------------------------------------------------- */
/* Far-field particle-cluster approximation                                   */
/* ------------------------------------------------------------------------- */

/* Contracted form of Sec. 4: eq. S_final for the Stokeslet part and
 * eq. T_final for the stresslet part, with sigma^k, tau_j, m^k, m_ij^k.
 * d = x - y_c; M is (nm,3) and Mt is (nm,9) (index j*3+l) for one cluster.
 * Adds the cluster's contribution into u. */
static void far_contracted_b(const double d[3], int p, const double *b, int P, const int32_t *kk,
                             const double *M, const double *Mt, double u[3])
{
    const int nm = orc_nm(p);
    for (int a = 0; a < nm; a++) {
        const int k[3] = {kk[3 * a], kk[3 * a + 1], kk[3 * a + 2]};
        const double *Ma = M + 3 * a;
        const double *Ta = Mt + 9 * a;
        const double sigma = d[0] * Ma[0] + d[1] * Ma[1] + d[2] * Ma[2];
        double tau[3];
        for (int j = 0; j < 3; j++) tau[j] = d[0] * Ta[3 * j + 0] + d[1] * Ta[3 * j + 1] + d[2] * Ta[3 * j + 2];
        const double mk = Ta[0] + Ta[4] + Ta[8];
        for (int i = 0; i < 3; i++) {
            int ei[3];
            ev(i, ei);
            const double ki1 = k[i] + 1;
            /* S_final */
            double sm = 0.0;
            for (int j = 0; j < 3; j++) {
                int ej[3];
                ev(j, ej);
                sm += bsh(b, P, k, ei[0] - ej[0], ei[1] - ej[1], ei[2] - ej[2]) * Ma[j];
            }
            const double sto = 2.0 * bsh(b, P, k, 0, 0, 0) * Ma[i] +
                               ki1 * (bsh(b, P, k, ei[0], ei[1], ei[2]) * sigma - sm);
            /* T_final */
            double t1 = 0.0, t2 = 0.0, t4 = 0.0;
            for (int j = 0; j < 3; j++) {
                int ej[3];
                ev(j, ej);
                const double cj = k[j] + 1 + delta(i, j);
                t1 += cj * bsh(b, P, k, ei[0] + ej[0], ei[1] + ej[1], ei[2] + ej[2]) * tau[j];
                for (int l = 0; l < 3; l++) {
                    int el[3];
                    ev(l, el);
                    t2 += cj *
                          bsh(b, P, k, ei[0] + ej[0] - el[0], ei[1] + ej[1] - el[1],
                              ei[2] + ej[2] - el[2]) *
                          Ta[3 * j + l];
                }
                const double mij = Ta[3 * i + j] + Ta[3 * j + i];
                t4 += (k[j] + 1) * bsh(b, P, k, ej[0], ej[1], ej[2]) * mij;
            }
            const double t3 = ki1 * bsh(b, P, k, ei[0], ei[1], ei[2]) * mk;
            const double str = (ki1 * t1 - ki1 * t2 + t3 + t4) / 3.0;
            u[i] += sto + str;
        }
    }
}

void orc_far_contracted(const double d[3], int p, const double *M, const double *Mt, double u[3])
{
    const int P = p + 2, S = P + 1;
    const int nm = orc_nm(p);
    double *b = malloc(sizeof(double) * S * S * S);
    int32_t *kk = malloc(sizeof(int32_t) * 3 * nm);
    orc_kindex(p, kk);
    orc_coulomb_taylor(d, P, b);
    u[0] = u[1] = u[2] = 0.0;
    far_contracted_b(d, p, b, P, kk, M, Mt, u);
    free(kk);
    free(b);
}

/* Un-contracted form, eq. pc_interaction: sum_k a^k_ij M_j^k + at^k_ijl Mt_jl^k,
 * with the coefficients formed explicitly from recurrence_2 and recurrence_3. */
void orc_far_explicit(const double d[3], int p, const double *M, const double *Mt, double u[3])
{
    const int nm = orc_nm(p);
    double *a = malloc(sizeof(double) * nm * 9);
    double *at = malloc(sizeof(double) * nm * 27);
    orc_stokeslet_coeffs(d, p, a);
    orc_stresslet_coeffs(d, p, at);
    u[0] = u[1] = u[2] = 0.0;
    for (int q = 0; q < nm; q++)
        for (int i = 0; i < 3; i++) {
            for (int j = 0; j < 3; j++) u[i] += a[(q * 3 + i) * 3 + j] * M[3 * q + j];
            for (int j = 0; j < 3; j++)
                for (int l = 0; l < 3; l++) u[i] += at[((q * 3 + i) * 3 + j) * 3 + l] * Mt[9 * q + 3 * j + l];
        }
    free(at);
    free(a);
}

/* ------------------------------------------------------------------------- */
/* Direct sums (Sec. 1 eq. StoStre; Sec. 4.1 contracted form)                 */
/* ------------------------------------------------------------------------- */

/* One source's contribution to one target, contracted form of Sec. 4.1:
 *   u_i += f_i/r + d_i s + d_i t,  s = (d.f)/r^3,  t = (d.h)(d.nu)/r^5. */
static void pair_contracted(const double x[3], const double y[3], const double f[3], const double h[3],
                            const double nu[3], double u[3])
{
    const double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (r2 == 0.0) return;
    const double r = sqrt(r2);
    const double r3 = r2 * r;
    const double r5 = r3 * r2;
    const double s = (d0 * f[0] + d1 * f[1] + d2 * f[2]) / r3;
    const double t = (d0 * h[0] + d1 * h[1] + d2 * h[2]) * (d0 * nu[0] + d1 * nu[1] + d2 * nu[2]) / r5;
    u[0] += f[0] / r + d0 * s + d0 * t;
    u[1] += f[1] / r + d1 * s + d1 * t;
    u[2] += f[2] / r + d2 * s + d2 * t;
}

/* Direct sum in contracted form over all sources, for each target. */
void orc_direct(const double *tgt, int64_t m, const double *src, int64_t n, const double *f,
                const double *h, const double *nu, double *u)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; t++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t s = 0; s < n; s++)
            pair_contracted(tgt + 3 * t, src + 3 * s, f + 3 * s, h + 3 * s, nu + 3 * s, acc);
        u[3 * t + 0] = acc[0];
        u[3 * t + 1] = acc[1];
        u[3 * t + 2] = acc[2];
    }
}

/* Direct sum with the kernel tensors formed explicitly (eqs. Stokeslet,
 * stresslet, StoStre): u_i = sum_n S_ij f_j + T_ijl h_j nu_l. */
void orc_direct_tensor(const double *tgt, int64_t m, const double *src, int64_t n, const double *f,
                       const double *h, const double *nu, double *u)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; t++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t s = 0; s < n; s++) {
            double d[3];
            for (int i = 0; i < 3; i++) d[i] = tgt[3 * t + i] - src[3 * s + i];
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 == 0.0) continue;
            const double r = sqrt(r2);
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    const double S = delta(i, j) / r + d[i] * d[j] / (r * r * r);
                    acc[i] += S * f[3 * s + j];
                    for (int l = 0; l < 3; l++) {
                        const double T = d[i] * d[j] * d[l] / (r * r * r * r * r);
                        acc[i] += T * h[3 * s + j] * nu[3 * s + l];
                    }
                }
        }
        for (int i = 0; i < 3; i++) u[3 * t + i] = acc[i];
    }
}

/* ------------------------------------------------------------------------- */
/* Tree (Sec. 5: root cube, bisection into 8 children, leaves hold <= N0)     */
/* ------------------------------------------------------------------------- */

typedef struct orc_tree {
    int64_t n;
    int32_t n0;
    int64_t *perm;   /* sorted position -> input index */
    double *ys;      /* positions in sorted order (n,3) */
    uint64_t *keys;  /* sorted Morton keys */
    double root[4];  /* lo[3], L */
    int64_t nnodes, cap;
    int32_t *level, *parent, *child0, *nchild;
    int64_t *start, *count;
    double *bmin, *bmax, *center, *radius;
} orc_tree;

typedef struct {
    uint64_t key;
    int64_t idx;
} keyidx;

static int cmp_keyidx(const void *a, const void *b)
{
    const keyidx *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

/* 21-bit integer coordinate of one axis inside the root cube. */
static uint64_t quantize(double y, double lo, double scale)
{
    const double v = floor((y - lo) * scale);
    if (!(v > 0.0)) return 0;
    if (v > 2097151.0) return 2097151;
    return (uint64_t)v;
}

/* Interleave three 21-bit coordinates, x bit most significant per level. */
static uint64_t morton(uint64_t qx, uint64_t qy, uint64_t qz)
{
    uint64_t key = 0;
    for (int bit = 20; bit >= 0; bit--) {
        key = (key << 3) | (((qx >> bit) & 1) << 2) | (((qy >> bit) & 1) << 1) | ((qz >> bit) & 1);
    }
    return key;
}

static void tree_grow(orc_tree *t)
{
    if (t->nnodes < t->cap) return;
    t->cap = t->cap ? 2 * t->cap : 64;
    t->level = realloc(t->level, sizeof(int32_t) * t->cap);
    t->parent = realloc(t->parent, sizeof(int32_t) * t->cap);
    t->child0 = realloc(t->child0, sizeof(int32_t) * t->cap);
    t->nchild = realloc(t->nchild, sizeof(int32_t) * t->cap);
    t->start = realloc(t->start, sizeof(int64_t) * t->cap);
    t->count = realloc(t->count, sizeof(int64_t) * t->cap);
}

static int64_t tree_add(orc_tree *t, int32_t level, int32_t parent, int64_t start, int64_t count)
{
    tree_grow(t);
    const int64_t i = t->nnodes++;
    t->level[i] = level;
    t->parent[i] = parent;
    t->child0[i] = -1;
    t->nchild[i] = 0;
    t->start[i] = start;
    t->count[i] = count;
    return i;
}

orc_tree *orc_tree_build(const double *src, int64_t n, int32_t n0)
{
    orc_tree *t = calloc(1, sizeof(orc_tree));
    t->n = n;
    t->n0 = n0;
    /* root cube: componentwise minimum and the largest extent */
    double lo[3], hi[3];
    for (int a = 0; a < 3; a++) lo[a] = hi[a] = src[a];
    for (int64_t s = 1; s < n; s++)
        for (int a = 0; a < 3; a++) {
            if (src[3 * s + a] < lo[a]) lo[a] = src[3 * s + a];
            if (src[3 * s + a] > hi[a]) hi[a] = src[3 * s + a];
        }
    double L = 0.0;
    for (int a = 0; a < 3; a++)
        if (hi[a] - lo[a] > L) L = hi[a] - lo[a];
    for (int a = 0; a < 3; a++) t->root[a] = lo[a];
    t->root[3] = L;
    const int degenerate = !(L > 0.0);
    const double scale = degenerate ? 0.0 : 2097152.0 / L;

    keyidx *ki = malloc(sizeof(keyidx) * n);
    for (int64_t s = 0; s < n; s++) {
        uint64_t q[3] = {0, 0, 0};
        if (!degenerate)
            for (int a = 0; a < 3; a++) q[a] = quantize(src[3 * s + a], lo[a], scale);
        ki[s].key = morton(q[0], q[1], q[2]);
        ki[s].idx = s;
    }
    qsort(ki, n, sizeof(keyidx), cmp_keyidx);
    t->perm = malloc(sizeof(int64_t) * n);
    t->keys = malloc(sizeof(uint64_t) * n);
    t->ys = malloc(sizeof(double) * 3 * n);
    for (int64_t s = 0; s < n; s++) {
        t->perm[s] = ki[s].idx;
        t->keys[s] = ki[s].key;
        for (int a = 0; a < 3; a++) t->ys[3 * s + a] = src[3 * ki[s].idx + a];
    }
    free(ki);

    /* breadth-first subdivision; the queue order is the node numbering */
    tree_add(t, 0, -1, 0, n);
    for (int64_t i = 0; i < t->nnodes; i++) {
        const int32_t lev = t->level[i];
        const int64_t s0 = t->start[i], c = t->count[i];
        if (degenerate || c <= n0 || lev >= ORC_MAX_LEVEL) continue;
        const int shift = 3 * (ORC_MAX_LEVEL - 1 - lev);
        int64_t s = s0;
        for (int oct = 0; oct < 8; oct++) {
            int64_t e = s;
            while (e < s0 + c && (int)((t->keys[e] >> shift) & 7) == oct) e++;
            if (e > s) {
                const int64_t ch = tree_add(t, lev + 1, (int32_t)i, s, e - s);
                if (t->child0[i] < 0) t->child0[i] = (int32_t)ch;
                t->nchild[i]++;
            }
            s = e;
        }
    }

    /* tight boxes, centres and radii */
    const int64_t nn = t->nnodes;
    t->bmin = malloc(sizeof(double) * 3 * nn);
    t->bmax = malloc(sizeof(double) * 3 * nn);
    t->center = malloc(sizeof(double) * 3 * nn);
    t->radius = malloc(sizeof(double) * nn);
    for (int64_t i = 0; i < nn; i++) {
        const int64_t s0 = t->start[i], c = t->count[i];
        for (int a = 0; a < 3; a++) t->bmin[3 * i + a] = t->bmax[3 * i + a] = t->ys[3 * s0 + a];
        for (int64_t s = s0; s < s0 + c; s++)
            for (int a = 0; a < 3; a++) {
                if (t->ys[3 * s + a] < t->bmin[3 * i + a]) t->bmin[3 * i + a] = t->ys[3 * s + a];
                if (t->ys[3 * s + a] > t->bmax[3 * i + a]) t->bmax[3 * i + a] = t->ys[3 * s + a];
            }
        for (int a = 0; a < 3; a++) t->center[3 * i + a] = 0.5 * (t->bmin[3 * i + a] + t->bmax[3 * i + a]);
        double r2max = 0.0;
        for (int64_t s = s0; s < s0 + c; s++) {
            const double dx = t->ys[3 * s] - t->center[3 * i];
            const double dy = t->ys[3 * s + 1] - t->center[3 * i + 1];
            const double dz = t->ys[3 * s + 2] - t->center[3 * i + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 > r2max) r2max = r2;
        }
        t->radius[i] = sqrt(r2max);
    }
    return t;
}

int64_t orc_tree_nnodes(const orc_tree *t) { return t->nnodes; }

void orc_tree_export(const orc_tree *t, int64_t *perm, int32_t *level, int32_t *parent, int32_t *child0,
                     int32_t *nchild, int64_t *start, int64_t *count, double *bmin, double *bmax,
                     double *center, double *radius, double *root)
{
    const int64_t nn = t->nnodes;
    memcpy(perm, t->perm, sizeof(int64_t) * t->n);
    memcpy(level, t->level, sizeof(int32_t) * nn);
    memcpy(parent, t->parent, sizeof(int32_t) * nn);
    memcpy(child0, t->child0, sizeof(int32_t) * nn);
    memcpy(nchild, t->nchild, sizeof(int32_t) * nn);
    memcpy(start, t->start, sizeof(int64_t) * nn);
    memcpy(count, t->count, sizeof(int64_t) * nn);
    memcpy(bmin, t->bmin, sizeof(double) * 3 * nn);
    memcpy(bmax, t->bmax, sizeof(double) * 3 * nn);
    memcpy(center, t->center, sizeof(double) * 3 * nn);
    memcpy(radius, t->radius, sizeof(double) * nn);
    memcpy(root, t->root, sizeof(double) * 4);
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    free(t->perm);
    free(t->keys);
    free(t->ys);
    free(t->level);
    free(t->parent);
    free(t->child0);
    free(t->nchild);
    free(t->start);
    free(t->count);
    free(t->bmin);
    free(t->bmax);
    free(t->center);
    free(t->radius);
    free(t);
}

/* ------------------------------------------------------------------------- */
/* Cluster moments (Sec. 2: M_j^k and Mt_jl^k), computed directly per node.   */
/* ------------------------------------------------------------------------- */

/* Positions are taken from pos (input order, (n,3)); the membership of each
 * node and its centre come from the tree.  With pos equal to the positions the
 * tree was built from this is the paper's moment; with perturbed positions it
 * is the frozen-plan moment used for finite differences. */
static void moments_at(const orc_tree *t, const double *pos, const double *f, const double *h,
                       const double *nu, int p, double *M, double *Mt)
{
    const int nm = orc_nm(p);
    int32_t *kk = malloc(sizeof(int32_t) * 3 * nm);
    orc_kindex(p, kk);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < t->nnodes; c++) {
        double *Mc = M + (size_t)c * nm * 3;
        double *Tc = Mt + (size_t)c * nm * 9;
        memset(Mc, 0, sizeof(double) * nm * 3);
        memset(Tc, 0, sizeof(double) * nm * 9);
        for (int64_t s = t->start[c]; s < t->start[c] + t->count[c]; s++) {
            const int64_t src = t->perm[s];
            double dy[3];
            for (int a = 0; a < 3; a++) dy[a] = pos[3 * src + a] - t->center[3 * c + a];
            for (int a = 0; a < nm; a++) {
                const double mono = monomial(dy, kk[3 * a], kk[3 * a + 1], kk[3 * a + 2]);
                for (int j = 0; j < 3; j++) Mc[3 * a + j] += mono * f[3 * src + j];
                for (int j = 0; j < 3; j++)
                    for (int l = 0; l < 3; l++)
                        Tc[9 * a + 3 * j + l] += mono * (h[3 * src + j] * nu[3 * src + l]);
            }
        }
    }
    free(kk);
}

/* M: (nnodes, nm, 3); Mt: (nnodes, nm, 9) with index j*3+l. */
void orc_moments(const orc_tree *t, const double *src, const double *f, const double *h,
                 const double *nu, int p, double *M, double *Mt)
{
    moments_at(t, src, f, h, nu, p, M, Mt);
}

/* ------------------------------------------------------------------------- */
/* Treecode (Sec. 5, Algorithm 1)                                             */
/* ------------------------------------------------------------------------- */

typedef struct {
    const orc_tree *t;
    const double *pos, *f, *h, *nu, *M, *Mt;
    int p, explicit_far;
    double theta;
    const int32_t *kk;
} tc_ctx;

typedef struct {
    double u[3];
    int64_t nfar, nnear, npairs;
    double *b;   /* scratch for the b coefficients */
} tc_acc;

static int mac_accept(const orc_tree *t, int64_t c, const double x[3], double theta)
{
    const double dx = x[0] - t->center[3 * c];
    const double dy = x[1] - t->center[3 * c + 1];
    const double dz = x[2] - t->center[3 * c + 2];
    const double R = sqrt(dx * dx + dy * dy + dz * dz);
    return R > 0.0 && t->radius[c] <= theta * R;
}

/* compute-velocity(x, C) of Algorithm 1 */
static void compute_velocity(const tc_ctx *cx, const double x[3], int64_t c, tc_acc *acc)
{
    const orc_tree *t = cx->t;
    if (mac_accept(t, c, x, cx->theta)) {
        const int nm = orc_nm(cx->p);
        double d[3];
        for (int a = 0; a < 3; a++) d[a] = x[a] - t->center[3 * c + a];
        const double *Mc = cx->M + (size_t)c * nm * 3;
        const double *Tc = cx->Mt + (size_t)c * nm * 9;
        if (cx->explicit_far) {
            double v[3];
            orc_far_explicit(d, cx->p, Mc, Tc, v);
            for (int a = 0; a < 3; a++) acc->u[a] += v[a];
        } else {
            double v[3] = {0.0, 0.0, 0.0};
            orc_coulomb_taylor(d, cx->p + 2, acc->b);
            far_contracted_b(d, cx->p, acc->b, cx->p + 2, cx->kk, Mc, Tc, v);
            for (int a = 0; a < 3; a++) acc->u[a] += v[a];
        }
        acc->nfar++;
    } else if (t->nchild[c] == 0) {
        for (int64_t s = t->start[c]; s < t->start[c] + t->count[c]; s++) {
            const int64_t n = t->perm[s];
            pair_contracted(x, cx->pos + 3 * n, cx->f + 3 * n, cx->h + 3 * n, cx->nu + 3 * n, acc->u);
        }
        acc->nnear++;
        acc->npairs += t->count[c];
    } else {
        for (int32_t ch = 0; ch < t->nchild[c]; ch++) compute_velocity(cx, x, t->child0[c] + ch, acc);
    }
}

/* Treecode velocity at arbitrary targets (disjoint or not).  f, h, nu and the
 * source positions are in input order; M, Mt come from orc_moments.  Per-target
 * interaction counts are written when the pointers are non-null. */
void orc_treecode(const orc_tree *t, const double *src, const double *f, const double *h, const double *nu,
                  const double *M, const double *Mt, int p, double theta, const double *tgt, int64_t m,
                  double *u, int64_t *nfar, int64_t *nnear, int64_t *npairs, int explicit_far)
{
    const int nm = orc_nm(p);
    int32_t *kk = malloc(sizeof(int32_t) * 3 * nm);
    orc_kindex(p, kk);
    tc_ctx cx = {t, src, f, h, nu, M, Mt, p, explicit_far, theta, kk};
    const int S = p + 3;
#pragma omp parallel
    {
        double *b = malloc(sizeof(double) * S * S * S);
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < m; i++) {
            tc_acc acc = {{0.0, 0.0, 0.0}, 0, 0, 0, b};
            compute_velocity(&cx, tgt + 3 * i, 0, &acc);
            for (int a = 0; a < 3; a++) u[3 * i + a] = acc.u[a];
            if (nfar) nfar[i] = acc.nfar;
            if (nnear) nnear[i] = acc.nnear;
            if (npairs) npairs[i] = acc.npairs;
        }
        free(b);
    }
    free(kk);
}

/* ------------------------------------------------------------------------- */
/* Frozen plan: interaction lists of Algorithm 1, kept and re-applied         */
/* ------------------------------------------------------------------------- */

static void list_walk(const orc_tree *t, const double x[3], int64_t c, double theta, int32_t *far,
                      int64_t *nf, int32_t *near, int64_t *nn)
{
    if (mac_accept(t, c, x, theta)) {
        if (far) far[*nf] = (int32_t)c;
        (*nf)++;
    } else if (t->nchild[c] == 0) {
        if (near) near[*nn] = (int32_t)c;
        (*nn)++;
    } else {
        for (int32_t ch = 0; ch < t->nchild[c]; ch++) list_walk(t, x, t->child0[c] + ch, theta, far, nf, near, nn);
    }
}

/* Two calls: with far_nodes == NULL only the CSR pointers are filled (counts,
 * then an inclusive scan); the second call fills the node lists. */
void orc_lists(const orc_tree *t, double theta, const double *tgt, int64_t m, int64_t *far_ptr,
               int32_t *far_nodes, int64_t *near_ptr, int32_t *near_nodes)
{
    if (!far_nodes) {
        far_ptr[0] = near_ptr[0] = 0;
        for (int64_t i = 0; i < m; i++) {
            int64_t nf = 0, nn = 0;
            list_walk(t, tgt + 3 * i, 0, theta, NULL, &nf, NULL, &nn);
            far_ptr[i + 1] = far_ptr[i] + nf;
            near_ptr[i + 1] = near_ptr[i] + nn;
        }
        return;
    }
    for (int64_t i = 0; i < m; i++) {
        int64_t nf = 0, nn = 0;
        list_walk(t, tgt + 3 * i, 0, theta, far_nodes + far_ptr[i], &nf, near_nodes + near_ptr[i], &nn);
    }
}

/* Frozen-plan operator: the lists, node membership and centres are fixed;
 * moments and kernels are re-evaluated from the given positions and weights. */
void orc_frozen_apply(const orc_tree *t, const double *src, const double *f, const double *h,
                      const double *nu, int p, const double *tgt, int64_t m, const int64_t *far_ptr,
                      const int32_t *far_nodes, const int64_t *near_ptr, const int32_t *near_nodes, double *u)
{
    const int nm = orc_nm(p);
    double *M = malloc(sizeof(double) * (size_t)t->nnodes * nm * 3);
    double *Mt = malloc(sizeof(double) * (size_t)t->nnodes * nm * 9);
    moments_at(t, src, f, h, nu, p, M, Mt);
    int32_t *kk = malloc(sizeof(int32_t) * 3 * nm);
    orc_kindex(p, kk);
    const int S = p + 3;
#pragma omp parallel
    {
        double *b = malloc(sizeof(double) * S * S * S);
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < m; i++) {
            double acc[3] = {0.0, 0.0, 0.0};
            const double *x = tgt + 3 * i;
            for (int64_t e = far_ptr[i]; e < far_ptr[i + 1]; e++) {
                const int64_t c = far_nodes[e];
                double d[3];
                for (int a = 0; a < 3; a++) d[a] = x[a] - t->center[3 * c + a];
                orc_coulomb_taylor(d, p + 2, b);
                far_contracted_b(d, p, b, p + 2, kk, M + (size_t)c * nm * 3, Mt + (size_t)c * nm * 9, acc);
            }
            for (int64_t e = near_ptr[i]; e < near_ptr[i + 1]; e++) {
                const int64_t c = near_nodes[e];
                for (int64_t s = t->start[c]; s < t->start[c] + t->count[c]; s++) {
                    const int64_t n = t->perm[s];
                    pair_contracted(x, src + 3 * n, f + 3 * n, h + 3 * n, nu + 3 * n, acc);
                }
            }
            for (int a = 0; a < 3; a++) u[3 * i + a] = acc[a];
        }
        free(b);
    }
    free(kk);
    free(Mt);
    free(M);
}

/* Gradient of w . u for one near pair (the analytic derivative of the
 * contracted direct-sum terms of Sec. 4.1).  Adds d/df, d/dh of the source and
 * d/dx of the target; d/dy of the source is the negative of d/dx. */
static void pair_grad(const double x[3], const double y[3], const double f[3], const double h[3],
                      const double nu[3], const double w[3], double gf[3], double gh[3], double gx[3])
{
    const double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) {
        gx[0] = gx[1] = gx[2] = 0.0;
        return;
    }
    const double r = sqrt(r2), r3 = r2 * r, r5 = r3 * r2;
    const double df = d[0] * f[0] + d[1] * f[1] + d[2] * f[2];
    const double dh = d[0] * h[0] + d[1] * h[1] + d[2] * h[2];
    const double dn = d[0] * nu[0] + d[1] * nu[1] + d[2] * nu[2];
    const double wd = w[0] * d[0] + w[1] * d[1] + w[2] * d[2];
    const double wf = w[0] * f[0] + w[1] * f[1] + w[2] * f[2];
    const double s = df / r3, tt = dh * dn / r5;
    for (int j = 0; j < 3; j++) {
        gf[j] += w[j] / r + wd * d[j] / r3;
        gh[j] += wd * d[j] * dn / r5;
    }
    for (int q = 0; q < 3; q++)
        gx[q] = -wf * d[q] / r3 + w[q] * (s + tt) +
                wd * (f[q] / r3 - 3.0 * s * d[q] / r2 + (h[q] * dn + dh * nu[q]) / r5 - 5.0 * tt * d[q] / r2);
}

/* Gradient of L = sum_m w^m . u^m for the direct sum, with respect to f, h,
 * source positions and target positions (all (.,3), input order). */
void orc_direct_grad(const double *tgt, int64_t m, const double *src, int64_t n, const double *f,
                     const double *h, const double *nu, const double *w, double *gf, double *gh,
                     double *gsrc, double *gtgt)
{
    memset(gf, 0, sizeof(double) * 3 * n);
    memset(gh, 0, sizeof(double) * 3 * n);
    memset(gsrc, 0, sizeof(double) * 3 * n);
    memset(gtgt, 0, sizeof(double) * 3 * m);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < n; s++) {
        for (int64_t i = 0; i < m; i++) {
            double gx[3];
            pair_grad(tgt + 3 * i, src + 3 * s, f + 3 * s, h + 3 * s, nu + 3 * s, w + 3 * i, gf + 3 * s,
                      gh + 3 * s, gx);
            for (int q = 0; q < 3; q++) gsrc[3 * s + q] -= gx[q];
        }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; i++) {
        for (int64_t s = 0; s < n; s++) {
            double gx[3], junk_f[3] = {0, 0, 0}, junk_h[3] = {0, 0, 0};
            pair_grad(tgt + 3 * i, src + 3 * s, f + 3 * s, h + 3 * s, nu + 3 * s, w + 3 * i, junk_f, junk_h,
                      gx);
            for (int q = 0; q < 3; q++) gtgt[3 * i + q] += gx[q];
        }
    }
}

/* d/dx_s of b^q for fixed source point: -(q_s+1) b^{q+e_s}. */
static double dbx(const double *b, int P, int q0, int q1, int q2, int s)
{
    int e[3];
    ev(s, e);
    const int qs = s == 0 ? q0 : (s == 1 ? q1 : q2);
    return -(qs + 1) * bget(b, P, q0 + e[0], q1 + e[1], q2 + e[2]);
}

/* Transpose of the frozen-plan operator (its adjoint), written out from the
 * particle-cluster form eq. pc_interaction with the explicit coefficients of
 * recurrence_2 / recurrence_3.  For L = sum_m w^m . u^m returns dL/df, dL/dh,
 * dL/d(source positions), dL/d(target positions).  Centres are held fixed. */
void orc_frozen_adjoint(const orc_tree *t, const double *src, const double *f, const double *h,
                        const double *nu, int p, const double *tgt, int64_t m, const int64_t *far_ptr,
                        const int32_t *far_nodes, const int64_t *near_ptr, const int32_t *near_nodes,
                        const double *w, double *gf, double *gh, double *gsrc, double *gtgt)
{
    const int64_t n = t->n, nnodes = t->nnodes;
    const int nm = orc_nm(p);
    const int P = p + 3, S = P + 1;
    double *M = malloc(sizeof(double) * (size_t)nnodes * nm * 3);
    double *Mt = malloc(sizeof(double) * (size_t)nnodes * nm * 9);
    moments_at(t, src, f, h, nu, p, M, Mt);
    double *LM = calloc((size_t)nnodes * nm * 3, sizeof(double));
    double *LT = calloc((size_t)nnodes * nm * 9, sizeof(double));
    int32_t *kk = malloc(sizeof(int32_t) * 3 * nm);
    orc_kindex(p, kk);
    double *b = malloc(sizeof(double) * S * S * S);
    double *a = malloc(sizeof(double) * nm * 9);
    double *at = malloc(sizeof(double) * nm * 27);
    memset(gf, 0, sizeof(double) * 3 * n);
    memset(gh, 0, sizeof(double) * 3 * n);
    memset(gsrc, 0, sizeof(double) * 3 * n);
    memset(gtgt, 0, sizeof(double) * 3 * m);

    /* far-field target-position derivative: it writes only target i's gradient, so the
     * targets run in parallel; the weight adjoints and the near field follow serially */
#pragma omp parallel
    {
        double *bp = malloc(sizeof(double) * S * S * S);
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < m; i++) {
            const double *x = tgt + 3 * i, *wi = w + 3 * i;
            for (int64_t e = far_ptr[i]; e < far_ptr[i + 1]; e++) {
                const int64_t c = far_nodes[e];
                double d[3];
                for (int q = 0; q < 3; q++) d[q] = x[q] - t->center[3 * c + q];
                orc_coulomb_taylor(d, P, bp);
                const double *b = bp;
                const double *Mc = M + (size_t)c * nm * 3, *Tc = Mt + (size_t)c * nm * 9;
                for (int q = 0; q < nm; q++) {
                    const int k[3] = {kk[3 * q], kk[3 * q + 1], kk[3 * q + 2]};
                    /* target-position derivative of the coefficients */
                    for (int s = 0; s < 3; s++) {
                        double g = 0.0;
                        for (int ii = 0; ii < 3; ii++) {
                            int ei[3];
                            ev(ii, ei);
                            for (int j = 0; j < 3; j++) {
                                int ej[3];
                                ev(j, ej);
                                const double da = delta(ii, j) * dbx(b, P, k[0], k[1], k[2], s) +
                                                  delta(j, s) * (k[ii] + 1) * bsh(b, P, k, ei[0], ei[1], ei[2]) +
                                                  d[j] * (k[ii] + 1) * dbx(b, P, k[0] + ei[0], k[1] + ei[1], k[2] + ei[2], s) -
                                                  (k[ii] + 1 - delta(ii, j)) *
                                                      dbx(b, P, k[0] + ei[0] - ej[0], k[1] + ei[1] - ej[1], k[2] + ei[2] - ej[2], s);
                                g += wi[ii] * da * Mc[3 * q + j];
                                for (int l = 0; l < 3; l++) {
                                    int el[3];
                                    ev(l, el);
                                    const double cij = (k[ii] + 1) * (k[j] + 1 + delta(ii, j));
                                    const double dat =
                                        (delta(l, s) * cij * bsh(b, P, k, ei[0] + ej[0], ei[1] + ej[1], ei[2] + ej[2]) +
                                         d[l] * cij * dbx(b, P, k[0] + ei[0] + ej[0], k[1] + ei[1] + ej[1], k[2] + ei[2] + ej[2], s) -
                                         (k[ii] + 1 - delta(ii, l)) * (k[j] + 1 + delta(ii, j) - delta(j, l)) *
                                             dbx(b, P, k[0] + ei[0] + ej[0] - el[0], k[1] + ei[1] + ej[1] - el[1],
                                                 k[2] + ei[2] + ej[2] - el[2], s) +
                                         delta(ii, j) * (k[l] + 1) * dbx(b, P, k[0] + el[0], k[1] + el[1], k[2] + el[2], s)) /
                                        3.0;
                                    g += wi[ii] * dat * Tc[9 * q + 3 * j + l];
                                }
                            }
                        }
                        gtgt[3 * i + s] += g;
                    }
                }
            }
        }
        free(bp);
    }

    for (int64_t i = 0; i < m; i++) {
        const double *x = tgt + 3 * i, *wi = w + 3 * i;
        for (int64_t e = far_ptr[i]; e < far_ptr[i + 1]; e++) {
            const int64_t c = far_nodes[e];
            double d[3];
            for (int q = 0; q < 3; q++) d[q] = x[q] - t->center[3 * c + q];
            orc_coulomb_taylor(d, P, b);
            stokeslet_coeffs_from_b(d, p, b, P, a);
            stresslet_coeffs_from_b(d, p, b, P, at);
            double *LMc = LM + (size_t)c * nm * 3, *LTc = LT + (size_t)c * nm * 9;
            for (int q = 0; q < nm; q++) {
                for (int ii = 0; ii < 3; ii++) {
                    for (int j = 0; j < 3; j++) {
                        LMc[3 * q + j] += wi[ii] * a[(q * 3 + ii) * 3 + j];
                        for (int l = 0; l < 3; l++) LTc[9 * q + 3 * j + l] += wi[ii] * at[((q * 3 + ii) * 3 + j) * 3 + l];
                    }
                }
            }
        }
        for (int64_t e = near_ptr[i]; e < near_ptr[i + 1]; e++) {
            const int64_t c = near_nodes[e];
            for (int64_t s = t->start[c]; s < t->start[c] + t->count[c]; s++) {
                const int64_t nn = t->perm[s];
                double gx[3];
                pair_grad(x, src + 3 * nn, f + 3 * nn, h + 3 * nn, nu + 3 * nn, wi, gf + 3 * nn, gh + 3 * nn, gx);
                for (int q = 0; q < 3; q++) {
                    gtgt[3 * i + q] += gx[q];
                    gsrc[3 * nn + q] -= gx[q];
                }
            }
        }
    }
    /* moment adjoints back to every source of every node.  Nodes are numbered level by
     * level and the nodes of one level hold disjoint sources, so the nodes of a level run
     * in parallel while every source still receives its terms root first, in node order. */
    for (int64_t c0 = 0; c0 < nnodes;) {
        int64_t c1 = c0;
        while (c1 < nnodes && t->level[c1] == t->level[c0]) c1++;
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = c0; c < c1; c++) {
            const double *LMc = LM + (size_t)c * nm * 3, *LTc = LT + (size_t)c * nm * 9;
            for (int64_t s = t->start[c]; s < t->start[c] + t->count[c]; s++) {
                const int64_t nn = t->perm[s];
                double dy[3];
                for (int q = 0; q < 3; q++) dy[q] = src[3 * nn + q] - t->center[3 * c + q];
                for (int q = 0; q < nm; q++) {
                    const int k[3] = {kk[3 * q], kk[3 * q + 1], kk[3 * q + 2]};
                    const double mono = monomial(dy, k[0], k[1], k[2]);
                    double pf = 0.0;
                    for (int j = 0; j < 3; j++) {
                        gf[3 * nn + j] += mono * LMc[3 * q + j];
                        pf += f[3 * nn + j] * LMc[3 * q + j];
                        for (int l = 0; l < 3; l++) {
                            gh[3 * nn + j] += mono * nu[3 * nn + l] * LTc[9 * q + 3 * j + l];
                            pf += h[3 * nn + j] * nu[3 * nn + l] * LTc[9 * q + 3 * j + l];
                        }
                    }
                    for (int sx = 0; sx < 3; sx++) {
                        if (k[sx] == 0) continue;
                        int e[3];
                        ev(sx, e);
                        const double dm = k[sx] * monomial(dy, k[0] - e[0], k[1] - e[1], k[2] - e[2]);
                        gsrc[3 * nn + sx] += dm * pf;
                    }
                }
            }
        }
        c0 = c1;
    }
    free(at);
    free(a);
    free(b);
    free(kk);
    free(LT);
    free(LM);
    free(Mt);
    free(M);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count for the parallel loops above (timing only; results do not depend on it). */
void orc_set_num_threads(int k)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(k > 0 ? k : 1);
#else
    (void)k;
#endif
}

/* ------------------------------------------------------------------------- */
/* Regularized Stokeslets and stresslets (the extension Sec. 7 names as      */
/* future work; Cortez 2001, Cortez-Fauci-Medovikov 2005).                    */
/* ------------------------------------------------------------------------- */
/*
 * Kernels, with the paper's normalisation (no 1/(8 pi); at eps = 0 they are
 * eqs. Stokeslet and stresslet exactly), R^2 = |d|^2 + eps^2:
 *   S^eps_ij  = delta_ij (|d|^2 + 2 eps^2) / R^3 + d_i d_j / R^3
 *               (the regularized Stokeslet of the 3D method of regularized
 *               Stokeslets, blob 15 eps^4 / (8 pi R^7));
 *   T^eps_ijl = [d_i d_j d_l + (eps^2/2)(delta_ij d_l + delta_jl d_i + delta_il d_j)] / R^5
 *               (-1/6 of the stress tensor -delta_il p_j + d_l S_ij + d_i S_lj of
 *               that flow, p_j = d_j (2|d|^2 + 5 eps^2) / R^5; at eps = 0 this is
 *               -1/6 of the classical -6 d_i d_j d_l / r^5).
 * With eps > 0 both are finite at d = 0, so every pair is summed (the self
 * pair adds 2 f / eps); with eps = 0 the pair d = 0 is skipped as above.
 *
 * Far field: the order-p Taylor expansion in y about the cluster centre,
 *   u_i = sum_k a^k_ij M_j^k + at^k_ijl Mt_jl^k,
 * the particle-cluster form of Sec. 3 with the regularized kernels.  With
 * phi_nu = R^(-2 nu) and g^k_nu its coefficients (1/k!) D_y^k phi_nu at y_c,
 * the product rule on the linear factors d = x - y (D_y d_i = -e_i) gives
 *   a^k_ij  = delta_ij (g^k_1/2 + eps^2 g^k_3/2)
 *             + d_i d_j g^k - d_i g^(k-e_j) - d_j g^(k-e_i) + g^(k-e_i-e_j)   (g = g_3/2)
 *   at^k_ijl = d_i d_j d_l e^k - d_j d_l e^(k-e_i) - d_i d_l e^(k-e_j) - d_i d_j e^(k-e_l)
 *             + d_l e^(k-e_i-e_j) + d_j e^(k-e_i-e_l) + d_i e^(k-e_j-e_l) - e^(k-e_i-e_j-e_l)
 *             + (eps^2/2) [delta_ij L_l + delta_jl L_i + delta_il L_j],  L_m = d_m e^k - e^(k-e_m)
 * (e = g_5/2; terms with a negative index vanish).  The coefficients of phi_nu
 * follow recurrence_1 generalised to R^2 = |d|^2 + eps^2 and exponent nu:
 *   n R^2 g^k = (2n + 2nu - 2) sum_i d_i g^(k-e_i) - (n + 2nu - 2) sum_i g^(k-2e_i),  n = ||k||,
 * which for nu = 1/2, eps = 0 is recurrence_1.
 */

/* coefficients of (|d|^2 + eps^2)^(-nu2/2) for ||k|| <= P, dense (P+1)^3 as b */
void orc_reg_taylor(const double d[3], double eps, int nu2, int P, double *a)
{
    const int S = P + 1;
    const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
    for (int i = 0; i < S * S * S; i++) a[i] = 0.0;
    a[0] = pow(R2, -0.5 * nu2);
    for (int n = 1; n <= P; n++)
        for (int k1 = n; k1 >= 0; k1--)
            for (int k2 = n - k1; k2 >= 0; k2--) {
                const int k3 = n - k1 - k2;
                double s1 = 0.0, s2 = 0.0;
                for (int i = 0; i < 3; i++) {
                    int q[3] = {k1, k2, k3};
                    q[i] -= 1;
                    if (q[i] >= 0) s1 += d[i] * bget(a, P, q[0], q[1], q[2]);
                    q[i] -= 1;
                    if (q[i] >= 0) s2 += bget(a, P, q[0], q[1], q[2]);
                }
                a[(k1 * S + k2) * S + k3] = ((2.0 * n + nu2 - 2.0) * s1 - (n + nu2 - 2.0) * s2) / (n * R2);
            }
}

/* g^(k - sum of shifts), 0 when an index goes negative */
static double rget(const double *a, int P, const int k[3], int i0, int i1, int i2)
{
    int q[3] = {k[0], k[1], k[2]};
    if (i0 >= 0) q[i0]--;
    if (i1 >= 0) q[i1]--;
    if (i2 >= 0) q[i2]--;
    if (q[0] < 0 || q[1] < 0 || q[2] < 0) return 0.0;
    return bget(a, P, q[0], q[1], q[2]);
}

/* a^k_ij (nm,3,3) and at^k_ijl (nm,3,3,3) of the regularized kernels at d, ||k|| <= p */
void orc_reg_coeffs(const double d[3], double eps, int p, double *a, double *at)
{
    const int nm = orc_nm(p), S = p + 1;
    double *g1 = malloc(sizeof(double) * S * S * S);
    double *g3 = malloc(sizeof(double) * S * S * S);
    double *g5 = malloc(sizeof(double) * S * S * S);
    orc_reg_taylor(d, eps, 1, p, g1);
    orc_reg_taylor(d, eps, 3, p, g3);
    orc_reg_taylor(d, eps, 5, p, g5);
    int32_t *kk = malloc(sizeof(int32_t) * 3 * nm);
    orc_kindex(p, kk);
    const double e2 = eps * eps;
    for (int q = 0; q < nm; q++) {
        const int k[3] = {kk[3 * q], kk[3 * q + 1], kk[3 * q + 2]};
        const double G1 = bget(g1, p, k[0], k[1], k[2]), G3 = bget(g3, p, k[0], k[1], k[2]);
        const double E = bget(g5, p, k[0], k[1], k[2]);
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double v = d[i] * d[j] * G3 - d[i] * rget(g3, p, k, j, -1, -1) - d[j] * rget(g3, p, k, i, -1, -1) +
                           rget(g3, p, k, i, j, -1);
                if (i == j) v += G1 + e2 * G3;
                a[(q * 3 + i) * 3 + j] = v;
                for (int l = 0; l < 3; l++) {
                    double w = d[i] * d[j] * d[l] * E - d[j] * d[l] * rget(g5, p, k, i, -1, -1) -
                               d[i] * d[l] * rget(g5, p, k, j, -1, -1) - d[i] * d[j] * rget(g5, p, k, l, -1, -1) +
                               d[l] * rget(g5, p, k, i, j, -1) + d[j] * rget(g5, p, k, i, l, -1) +
                               d[i] * rget(g5, p, k, j, l, -1) - rget(g5, p, k, i, j, l);
                    double lin = 0.0;
                    if (i == j) lin += d[l] * E - rget(g5, p, k, l, -1, -1);
                    if (j == l) lin += d[i] * E - rget(g5, p, k, i, -1, -1);
                    if (i == l) lin += d[j] * E - rget(g5, p, k, j, -1, -1);
                    at[((q * 3 + i) * 3 + j) * 3 + l] = w + 0.5 * e2 * lin;
                }
            }
    }
    free(kk);
    free(g5);
    free(g3);
    free(g1);
}

/* far-field velocity of one cluster: sum_k a^k_ij M_j^k + at^k_ijl Mt_jl^k */
void orc_reg_far(const double d[3], double eps, int p, const double *M, const double *Mt, double u[3])
{
    const int nm = orc_nm(p);
    double *a = malloc(sizeof(double) * nm * 9);
    double *at = malloc(sizeof(double) * nm * 27);
    orc_reg_coeffs(d, eps, p, a, at);
    u[0] = u[1] = u[2] = 0.0;
    for (int q = 0; q < nm; q++)
        for (int i = 0; i < 3; i++) {
            for (int j = 0; j < 3; j++) {
                u[i] += a[(q * 3 + i) * 3 + j] * M[3 * q + j];
                for (int l = 0; l < 3; l++) u[i] += at[((q * 3 + i) * 3 + j) * 3 + l] * Mt[9 * q + 3 * j + l];
            }
        }
    free(at);
    free(a);
}

/* one source's regularized contribution, contracted:
 *   u_i += f_i (|d|^2 + 2 eps^2)/R^3 + d_i (d.f)/R^3
 *        + [d_i (d.h)(d.nu) + (eps^2/2)(h_i (d.nu) + d_i (h.nu) + nu_i (d.h))] / R^5 */
static void reg_pair(const double x[3], const double y[3], const double f[3], const double h[3],
                     const double nu[3], double eps, double u[3])
{
    const double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (r2 == 0.0 && eps == 0.0) return;
    const double e2 = eps * eps;
    const double R2 = r2 + e2;
    const double R = sqrt(R2);
    const double R3 = R2 * R, R5 = R3 * R2;
    const double df = d0 * f[0] + d1 * f[1] + d2 * f[2];
    const double dh = d0 * h[0] + d1 * h[1] + d2 * h[2];
    const double dn = d0 * nu[0] + d1 * nu[1] + d2 * nu[2];
    const double hn = h[0] * nu[0] + h[1] * nu[1] + h[2] * nu[2];
    const double cs = (r2 + 2.0 * e2) / R3;
    const double dd[3] = {d0, d1, d2};
    for (int i = 0; i < 3; i++)
        u[i] += f[i] * cs + dd[i] * df / R3 +
                (dd[i] * dh * dn + 0.5 * e2 * (h[i] * dn + dd[i] * hn + nu[i] * dh)) / R5;
}

/* regularized direct sum over all sources, for each target */
void orc_reg_direct(const double *tgt, int64_t m, const double *src, int64_t n, const double *f,
                    const double *h, const double *nu, double eps, double *u)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; t++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t s = 0; s < n; s++)
            reg_pair(tgt + 3 * t, src + 3 * s, f + 3 * s, h + 3 * s, nu + 3 * s, eps, acc);
        u[3 * t + 0] = acc[0];
        u[3 * t + 1] = acc[1];
        u[3 * t + 2] = acc[2];
    }
}

/* the same sum with S^eps and T^eps formed as tensors */
void orc_reg_direct_tensor(const double *tgt, int64_t m, const double *src, int64_t n, const double *f,
                           const double *h, const double *nu, double eps, double *u)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; t++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t s = 0; s < n; s++) {
            double d[3];
            for (int a = 0; a < 3; a++) d[a] = tgt[3 * t + a] - src[3 * s + a];
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 == 0.0 && eps == 0.0) continue;
            const double R2 = r2 + eps * eps, R = sqrt(R2);
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    const double Sij = (i == j ? (r2 + 2.0 * eps * eps) / (R2 * R) : 0.0) + d[i] * d[j] / (R2 * R);
                    acc[i] += Sij * f[3 * s + j];
                    for (int l = 0; l < 3; l++) {
                        const double Tijl = (d[i] * d[j] * d[l] + 0.5 * eps * eps *
                                                                      ((i == j ? d[l] : 0.0) + (j == l ? d[i] : 0.0) +
                                                                       (i == l ? d[j] : 0.0))) /
                                            (R2 * R2 * R);
                        acc[i] += Tijl * h[3 * s + j] * nu[3 * s + l];
                    }
                }
        }
        for (int a = 0; a < 3; a++) u[3 * t + a] = acc[a];
    }
}

typedef struct {
    const orc_tree *t;
    const double *pos, *f, *h, *nu, *M, *Mt;
    int p;
    double theta, eps;
} reg_ctx;

/* compute-velocity(x, C) of Algorithm 1 with the regularized kernels */
static void reg_velocity(const reg_ctx *cx, const double x[3], int64_t c, tc_acc *acc)
{
    const orc_tree *t = cx->t;
    if (mac_accept(t, c, x, cx->theta)) {
        const int nm = orc_nm(cx->p);
        double d[3], v[3];
        for (int a = 0; a < 3; a++) d[a] = x[a] - t->center[3 * c + a];
        orc_reg_far(d, cx->eps, cx->p, cx->M + (size_t)c * nm * 3, cx->Mt + (size_t)c * nm * 9, v);
        for (int a = 0; a < 3; a++) acc->u[a] += v[a];
        acc->nfar++;
    } else if (t->nchild[c] == 0) {
        for (int64_t s = t->start[c]; s < t->start[c] + t->count[c]; s++) {
            const int64_t n = t->perm[s];
            reg_pair(x, cx->pos + 3 * n, cx->f + 3 * n, cx->h + 3 * n, cx->nu + 3 * n, cx->eps, acc->u);
        }
        acc->nnear++;
        acc->npairs += t->count[c];
    } else {
        for (int32_t ch = 0; ch < t->nchild[c]; ch++) reg_velocity(cx, x, t->child0[c] + ch, acc);
    }
}

/* regularized treecode velocity at arbitrary targets (same tree, moments and MAC) */
void orc_reg_treecode(const orc_tree *t, const double *src, const double *f, const double *h, const double *nu,
                      const double *M, const double *Mt, int p, double theta, double eps, const double *tgt,
                      int64_t m, double *u, int64_t *nfar, int64_t *nnear, int64_t *npairs)
{
    reg_ctx cx = {t, src, f, h, nu, M, Mt, p, theta, eps};
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < m; i++) {
        tc_acc acc = {{0.0, 0.0, 0.0}, 0, 0, 0, NULL};
        reg_velocity(&cx, tgt + 3 * i, 0, &acc);
        for (int a = 0; a < 3; a++) u[3 * i + a] = acc.u[a];
        if (nfar) nfar[i] = acc.nfar;
        if (nnear) nnear[i] = acc.nnear;
        if (npairs) npairs[i] = acc.npairs;
    }
}
