/*
 * octree_oracle.c -- plain, slow, FP64 reference of the Lagrangian-point
 * tracking step (host-cell search, 3-point regularized-delta interpolation,
 * force spreading, gradient with respect to point positions).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code with the GPU path.
 *
 * What it follows (Jiang, Calzavarini & Krug, "Simulations of particle-laden
 * flows with large dispersed-phase size disparities using highly scalable
 * parallel adaptive methods"):
 *   - leaves of the octree kept in an array sorted by Morton (Z-order) index
 *     (Sec. 3.1, grid management; Sec. 3.2, Lagrangian data management);
 *   - host-cell search: Algorithm 1 (search_host_cell / get_cell_at), and the
 *     naive linear containment scan that Sec. 3.2 contrasts it with;
 *   - interpolation of the Eulerian velocity to a Lagrangian point and
 *     spreading of a point force back to the grid (Sec. 2.2, the
 *     interpolation and spreading equations of the multi-direct-forcing
 *     scheme);
 *   - the weighting function W = product of three 1-D 3-point discrete delta
 *     functions phi (Sec. 2.2, the W and phi equations).
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - integer coordinates are kept at the tree's finest level L instead of
 *     p4est's MAXLEVEL; get_cell_at(x, l) = floor(x 2^l) 2^(L-l), which equals
 *     (floor(x 2^L) >> (L-l)) << (L-l) exactly for binary floating point;
 *   - a cell is the half-open box [a, a + 2^(L-l)) on each axis;
 *   - a leaf id is its rank in the Morton-sorted leaf array, -1 = not found;
 *   - phi takes the dimensionless distance r = (x - X)/dx_l, so its branch
 *     bounds are 1/2 and 3/2;
 *   - the 3x3x3 stencil is taken at the host leaf's level l; the value of a
 *     stencil node (a level-l cell) is read from the leaf that contains the
 *     node's centre (half-open rule, so a centre on a corner of finer cells
 *     belongs to the upper child);
 *     PARITY UNPINNED for stencils that cross a level jump: the paper gives
 *     no value there.  The tests pin this reading's implementation by
 *     geometry (the node's leaf contains its centre) and by self-consistency
 *     (conservation, the adjoint identity, constants reproduced);
 *   - spread is the exact transpose of interpolate: both use the weights
 *     phi(rx) phi(ry) phi(rz) without a cell-volume factor (the (dx)^D of the
 *     sums cancels the 1/dx^D of W);
 *   - periodic domains wrap integer coordinates; otherwise stencil nodes
 *     outside the unit cube are dropped with their weight.
 *
 * Floating-point sums use Neumaier-compensated accumulation in a fixed order
 * (stencil z outer, y, x inner; points in ascending index order).
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t n_leaves;
    const uint64_t *keys;    /* Morton keys of leaf anchors, ascending        */
    const uint8_t *levels;   /* level of each leaf                             */
    int32_t l_min;           /* coarsest level any leaf may have               */
    int32_t l_max;           /* finest level L; integer coordinates in 2^-L    */
    int32_t periodic;        /* 1: unit cube is periodic in x, y and z         */
} orc_tree;

/* ---------------------------------------------------------------------------
 * Morton (Z-order) index: bit b of x goes to bit 3b, of y to 3b+1, of z to
 * 3b+2 (Sec. 3.1: the Z-curve linearises the tree).  Written as a plain loop
 * over bits.
 * ------------------------------------------------------------------------- */
uint64_t orc_morton_encode(uint32_t x, uint32_t y, uint32_t z, int32_t L)
{
    uint64_t k = 0;
    for (int b = 0; b < L; ++b) {
        k |= (uint64_t)((x >> b) & 1u) << (3 * b);
        k |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
        k |= (uint64_t)((z >> b) & 1u) << (3 * b + 2);
    }
    return k;
}

void orc_morton_decode(uint64_t k, int32_t L, uint32_t *x, uint32_t *y, uint32_t *z)
{
    uint32_t a = 0, b2 = 0, c = 0;
    for (int b = 0; b < L; ++b) {
        a |= (uint32_t)((k >> (3 * b)) & 1u) << b;
        b2 |= (uint32_t)((k >> (3 * b + 1)) & 1u) << b;
        c |= (uint32_t)((k >> (3 * b + 2)) & 1u) << b;
    }
    *x = a; *y = b2; *z = c;
}

void orc_encode_keys(int64_t n, const uint32_t *anchors, int32_t L, uint64_t *keys)
{
    for (int64_t i = 0; i < n; ++i)
        keys[i] = orc_morton_encode(anchors[3 * i], anchors[3 * i + 1], anchors[3 * i + 2], L);
}

/* ---------------------------------------------------------------------------
 * Sorting the leaves by Morton index (the sorted quadrant array of a p4est
 * tree, Sec. 3.1).  perm[sorted position] = input position.
 * ------------------------------------------------------------------------- */
static const uint64_t *g_sort_keys;
static int cmp_idx(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (g_sort_keys[a] < g_sort_keys[b]) return -1;
    if (g_sort_keys[a] > g_sort_keys[b]) return 1;
    return (a < b) ? -1 : (a > b);
}

void orc_sort_leaves(int64_t n, const uint64_t *keys, int64_t *perm)
{
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    g_sort_keys = keys;
    qsort(perm, (size_t)n, sizeof(int64_t), cmp_idx);
    g_sort_keys = NULL;
}

/* Validity of a sorted leaf array as a partition of the unit cube.
 * Returns 0 when valid, 1 when the leaves do not tile the cube exactly,
 * 2 when two leaves share an anchor, 3 when a level is outside [l_min, L]
 * or a key has bits above 3L. */
int32_t orc_check_partition(const orc_tree *t)
{
    int L = t->l_max;
    if (L < 0 || L > 21 || t->l_min < 0 || t->l_min > L) return 3;
    if (t->n_leaves <= 0) return 1;
    for (int64_t j = 0; j < t->n_leaves; ++j) {
        int l = t->levels[j];
        if (l < t->l_min || l > L) return 3;
        if ((t->keys[j] >> (3 * L)) != 0) return 3;
    }
    uint64_t expect = 0; /* first Morton index not yet covered */
    for (int64_t j = 0; j < t->n_leaves; ++j) {
        uint64_t vol = (uint64_t)1 << (3 * (L - t->levels[j]));
        if (j > 0 && t->keys[j] == t->keys[j - 1]) return 2;
        if (t->keys[j] != expect) return 1;        /* gap or overlap          */
        if (t->keys[j] % vol != 0) return 1;       /* anchor not cell-aligned */
        expect = t->keys[j] + vol;
    }
    return (expect == ((uint64_t)1 << (3 * L))) ? 0 : 1;
}

/* ---------------------------------------------------------------------------
 * Point -> integer coordinates at level L:  I = floor(x 2^L) in FP64.
 * Returns 0 for points that have no host cell: NaN/inf, |x 2^L| >= 2^52, or
 * (non-periodic) outside [0, 1).  Periodic domains wrap I modulo 2^L.
 * ------------------------------------------------------------------------- */
static int point_cell(const orc_tree *t, const double x[3], int64_t I[3])
{
    const double scale = ldexp(1.0, t->l_max);
    const int64_t M = (int64_t)1 << t->l_max;
    for (int d = 0; d < 3; ++d) {
        double s = x[d] * scale;
        if (!(fabs(s) < 4503599627370496.0)) return 0; /* 2^52; false for NaN */
        int64_t v = (int64_t)floor(s);
        if (t->periodic) {
            v %= M;
            if (v < 0) v += M;
        } else if (v < 0 || v >= M) {
            return 0;
        }
        I[d] = v;
    }
    return 1;
}

/* Exact-match binary search over the sorted keys; -1 when absent. */
static int64_t binary_search(const orc_tree *t, uint64_t K)
{
    int64_t lo = 0, hi = t->n_leaves - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (t->keys[mid] == K) return mid;
        if (t->keys[mid] < K) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* get_cell_at(point, level) of Algorithm 1 on integer coordinates:
 * the anchor of the level-l cell that contains I. */
static void get_cell_at(const int64_t I[3], int l, int L, uint32_t a[3])
{
    int sh = L - l;
    for (int d = 0; d < 3; ++d) a[d] = (uint32_t)((I[d] >> sh) << sh);
}

/* Algorithm 1 (search_host_cell) for one point: for each level from l_min to
 * L build the test cell and binary-search the Z-sorted leaves for it; the
 * first exact hit (same anchor and same level) is the host cell.  The forest
 * here has a single tree. */
int64_t orc_search_host_cell(const orc_tree *t, const int64_t I[3])
{
    for (int l = t->l_min; l <= t->l_max; ++l) {
        uint32_t a[3];
        get_cell_at(I, l, t->l_max, a);
        uint64_t K = orc_morton_encode(a[0], a[1], a[2], t->l_max);
        int64_t idx = binary_search(t, K);
        if (idx >= 0 && t->levels[idx] == l) return idx;
    }
    return -1;
}

/* The naive linear search of Sec. 3.2: test every leaf for containment.
 * Returns the unique containing leaf, -1 if none, -2 if several contain it. */
int64_t orc_linear_search(const orc_tree *t, const int64_t I[3])
{
    int64_t found = -1;
    for (int64_t j = 0; j < t->n_leaves; ++j) {
        uint32_t a[3];
        orc_morton_decode(t->keys[j], t->l_max, &a[0], &a[1], &a[2]);
        int64_t size = (int64_t)1 << (t->l_max - t->levels[j]);
        int inside = 1;
        for (int d = 0; d < 3; ++d)
            if (!(I[d] >= (int64_t)a[d] && I[d] < (int64_t)a[d] + size)) inside = 0;
        if (inside) {
            if (found >= 0) return -2;
            found = j;
        }
    }
    return found;
}

/* Host ids of n points.  method 0: Algorithm 1, method 1: linear search. */
void orc_locate(const orc_tree *t, const double *pos, int64_t n, int32_t method, int64_t *ids)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        int64_t I[3];
        if (!point_cell(t, pos + 3 * k, I)) { ids[k] = -1; continue; }
        ids[k] = method == 0 ? orc_search_host_cell(t, I) : orc_linear_search(t, I);
    }
}

/* ---------------------------------------------------------------------------
 * 3-point discrete delta function phi (Sec. 2.2), on the dimensionless
 * distance r, and its derivative, each branch as printed.
 *
 * They are evaluated in binary128 (__float128) and rounded once to FP64.
 * Near the edge of the support (|r| -> 3/2) the outer branch is a difference
 * of two terms close to 1/2 whose result goes to zero quadratically, so the
 * printed formula evaluated in FP64 is good only to about 2^-53 absolute;
 * in binary128 the same formula, in the same order, is good to about 2^-113
 * absolute, far below any FP64 result it is compared with.
 * ------------------------------------------------------------------------- */
static __float128 phi_q(__float128 r)
{
    __float128 a = r < 0 ? -r : r;
    if (a <= 0.5Q) return (1.0Q + sqrtq(1.0Q - 3.0Q * r * r)) / 3.0Q;
    if (a <= 1.5Q) return (5.0Q - 3.0Q * a - sqrtq(-2.0Q + 6.0Q * a - 3.0Q * r * r)) / 6.0Q;
    return 0.0Q;
}

static __float128 dphi_q(__float128 r)
{
    __float128 a = r < 0 ? -r : r;
    __float128 sg = r < 0 ? -1.0Q : 1.0Q;
    if (a <= 0.5Q) return -r / sqrtq(1.0Q - 3.0Q * r * r);
    if (a < 1.5Q) {
        __float128 g = -2.0Q + 6.0Q * a - 3.0Q * r * r;
        return sg * (-3.0Q - (6.0Q - 6.0Q * a) / (2.0Q * sqrtq(g))) / 6.0Q;
    }
    return 0.0Q;
}

double orc_phi(double r) { return (double)phi_q((__float128)r); }

double orc_dphi(double r) { return (double)dphi_q((__float128)r); }

/* Neumaier-compensated accumulation. */
static inline void nsum(double *s, double *c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *c += (*s - t) + v; else *c += (v - t) + *s;
    *s = t;
}

/* The stencil of one point: host leaf, its level l, per-axis node cell
 * indices at level l (o = 0,1,2 for offsets -1,0,+1), whether each node
 * exists, the per-axis 1-D weights ph[d][o] = phi(r) of the distances
 * r = t_d - 1/2 - (o-1) (and phi'(r) in dph when asked), and the leaf
 * holding each of the 27 nodes.  The offset t_d = x 2^l - floor(x 2^l) and
 * the distance are formed in binary128, where both are exact (also for a
 * point below 0 wrapped by periodicity, whose FP64 offset would round), and
 * phi / phi' are evaluated there and rounded once. */
typedef struct {
    int64_t host;
    int level;
    double ph[3][3];
    double dph[3][3];
    int valid[3][3];
    int64_t leaf[27];   /* index oz*9 + oy*3 + ox */
} stencil;

static int build_stencil(const orc_tree *t, const double x[3], stencil *st, int want_grad)
{
    int64_t I[3];
    st->host = -1;
    if (!point_cell(t, x, I)) return 0;
    st->host = orc_search_host_cell(t, I);
    if (st->host < 0) return 0;
    const int L = t->l_max;
    const int l = t->levels[st->host];
    const int sh = L - l;
    const int64_t Ml = (int64_t)1 << l;
    st->level = l;
    int64_t nidx[3][3];
    for (int d = 0; d < 3; ++d) {
        double s = x[d] * ldexp(1.0, l);     /* position in level-l cell units */
        /* offset inside the host cell, in binary128 so that it is exact
         * also for s < 0 (a periodic wrap), where s - floor(s) in FP64 would
         * round away the distance to the far edge of the support           */
        __float128 frac = (__float128)s - (__float128)floor(s);
        int64_t i0 = I[d] >> sh;             /* host cell index at level l    */
        for (int o = 0; o < 3; ++o) {
            __float128 r = frac - 0.5Q - (__float128)(o - 1);
            st->ph[d][o] = (double)phi_q(r);
            st->dph[d][o] = want_grad ? (double)dphi_q(r) : 0.0;
            int64_t nd = i0 + (o - 1);
            int ok = 1;
            if (t->periodic) { nd %= Ml; if (nd < 0) nd += Ml; }
            else if (nd < 0 || nd >= Ml) ok = 0;
            nidx[d][o] = nd;
            st->valid[d][o] = ok;
        }
    }
    for (int oz = 0; oz < 3; ++oz)
        for (int oy = 0; oy < 3; ++oy)
            for (int ox = 0; ox < 3; ++ox) {
                int q = oz * 9 + oy * 3 + ox;
                if (!(st->valid[0][ox] && st->valid[1][oy] && st->valid[2][oz])) {
                    st->leaf[q] = -1;
                    continue;
                }
                int64_t N[3];
                int64_t nn[3] = {nidx[0][ox], nidx[1][oy], nidx[2][oz]};
                for (int d = 0; d < 3; ++d)  /* node centre at level-L resolution */
                    N[d] = (nn[d] << sh) + (sh > 0 ? ((int64_t)1 << (sh - 1)) : 0);
                st->leaf[q] = orc_search_host_cell(t, N);
            }
    return 1;
}

/* ---------------------------------------------------------------------------
 * Interpolation (Sec. 2.2):  U_k = sum_n W(x_n - X_k) (dx)^3 u(x_n).
 * field: (n_leaves, 3) in Morton order.  U: (n, 3).  scale (nullable):
 * sum_n |w_n| |u_n,c|, the magnitude that bounds the rounding error.
 * Points without a host cell get U = 0.
 * ------------------------------------------------------------------------- */
void orc_interpolate(const orc_tree *t, const double *field, const double *pos, int64_t n,
                     double *U, double *scale)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) {
        stencil st;
        double s[3] = {0, 0, 0}, c[3] = {0, 0, 0}, m[3] = {0, 0, 0};
        if (build_stencil(t, pos + 3 * k, &st, 0)) {
            for (int oz = 0; oz < 3; ++oz)
                for (int oy = 0; oy < 3; ++oy)
                    for (int ox = 0; ox < 3; ++ox) {
                        int q = oz * 9 + oy * 3 + ox;
                        if (st.leaf[q] < 0) continue;
                        double w = st.ph[0][ox] * st.ph[1][oy] * st.ph[2][oz];
                        const double *u = field + 3 * st.leaf[q];
                        for (int e = 0; e < 3; ++e) {
                            nsum(&s[e], &c[e], w * u[e]);
                            m[e] += fabs(w) * fabs(u[e]);
                        }
                    }
        }
        for (int e = 0; e < 3; ++e) {
            U[3 * k + e] = s[e] + c[e];
            if (scale) scale[3 * k + e] = m[e];
        }
    }
}

/* ---------------------------------------------------------------------------
 * Spreading (Sec. 2.2):  f(x_n) = sum_k F_k W(x_n - X_k) (dx)^3, the exact
 * transpose of orc_interpolate.  f, scale: (n_leaves, 3); count: contributions
 * per leaf; fabs_sum: sum of |F_k,c| over the contributions (weight-free).
 * The last three are nullable diagnostics.  f is overwritten.
 *
 * The points are cut into one contiguous block per thread (ascending index
 * order inside each block); every thread sums its block into a private,
 * compensated copy of the field, and the copies are then added leaf by leaf
 * in thread order with the same compensation.
 * ------------------------------------------------------------------------- */
void orc_spread(const orc_tree *t, const double *F, const double *pos, int64_t n,
                double *f, double *scale, int64_t *count, double *fabs_sum)
{
    const int64_t nl = t->n_leaves;
    const size_t n3 = (size_t)(3 * nl);
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
    if ((int64_t)nt > n / 256 + 1) nt = (int)(n / 256 + 1);   /* small inputs: fewer copies */
#endif
    /* per thread: sum, compensation, and the diagnostics when asked */
    double *ps = (double *)calloc((size_t)nt * n3, sizeof(double));
    double *pc = (double *)calloc((size_t)nt * n3, sizeof(double));
    double *pm = scale ? (double *)calloc((size_t)nt * n3, sizeof(double)) : NULL;
    double *pa = fabs_sum ? (double *)calloc((size_t)nt * n3, sizeof(double)) : NULL;
    int64_t *pn = count ? (int64_t *)calloc((size_t)nt * (size_t)nl, sizeof(int64_t)) : NULL;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        const int64_t k0 = n * tid / nt, k1 = n * (tid + 1) / nt;
        double *fs = ps + (size_t)tid * n3, *fc = pc + (size_t)tid * n3;
        for (int64_t k = k0; k < k1; ++k) {
            stencil st;
            if (!build_stencil(t, pos + 3 * k, &st, 0)) continue;
            for (int oz = 0; oz < 3; ++oz)
                for (int oy = 0; oy < 3; ++oy)
                    for (int ox = 0; ox < 3; ++ox) {
                        int q = oz * 9 + oy * 3 + ox;
                        int64_t j = st.leaf[q];
                        if (j < 0) continue;
                        double w = st.ph[0][ox] * st.ph[1][oy] * st.ph[2][oz];
                        for (int e = 0; e < 3; ++e) {
                            nsum(&fs[3 * j + e], &fc[3 * j + e], w * F[3 * k + e]);
                            if (pm) pm[(size_t)tid * n3 + 3 * j + e] += fabs(w * F[3 * k + e]);
                            if (pa) pa[(size_t)tid * n3 + 3 * j + e] += fabs(F[3 * k + e]);
                        }
                        if (pn) pn[(size_t)tid * (size_t)nl + j] += 1;
                    }
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n3; ++i) {
        double s = 0.0, c = 0.0, m = 0.0, a = 0.0;
        for (int th = 0; th < nt; ++th) {
            nsum(&s, &c, ps[(size_t)th * n3 + i]);
            nsum(&s, &c, pc[(size_t)th * n3 + i]);
            if (pm) m += pm[(size_t)th * n3 + i];
            if (pa) a += pa[(size_t)th * n3 + i];
        }
        f[i] = s + c;
        if (scale) scale[i] = m;
        if (fabs_sum) fabs_sum[i] = a;
    }
    if (count) {
        for (int64_t j = 0; j < nl; ++j) {
            int64_t c = 0;
            for (int th = 0; th < nt; ++th) c += pn[(size_t)th * (size_t)nl + j];
            count[j] = c;
        }
    }
    free(ps);
    free(pc);
    free(pm);
    free(pa);
    free(pn);
}

/* ---------------------------------------------------------------------------
 * Gradient with respect to point positions of  sum_k v_k . U_k(X_k)  where
 * U = interpolate(field):
 *   g_k,d = sum_n (v_k . u_n) dW_n/dX_d,
 *   dW_n/dX_d = 2^l phi'(r_d) prod_{e != d} phi(r_e)
 * (r_d = (X_d - x_n,d)/dx_l, so dr_d/dX_d = 2^l).  The host leaf, and with it
 * the level and the node set, is held at its value for X_k.  The same sum,
 * with (field, v) = (upstream leaf gradient, F), is the position gradient of
 * spread.  scale (nullable): sum_n sum_c |v_c u_n,c| |dW_n/dX_d|.
 * ------------------------------------------------------------------------- */
void orc_grad_pos(const orc_tree *t, const double *field, const double *vec, const double *pos,
                  int64_t n, double *g, double *scale)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) {
        stencil st;
        double s[3] = {0, 0, 0}, c[3] = {0, 0, 0}, m[3] = {0, 0, 0};
        if (build_stencil(t, pos + 3 * k, &st, 1)) {
            double h = ldexp(1.0, st.level);
            for (int oz = 0; oz < 3; ++oz)
                for (int oy = 0; oy < 3; ++oy)
                    for (int ox = 0; ox < 3; ++ox) {
                        int q = oz * 9 + oy * 3 + ox;
                        if (st.leaf[q] < 0) continue;
                        const double *u = field + 3 * st.leaf[q];
                        const double *v = vec + 3 * k;
                        double dot = v[0] * u[0] + v[1] * u[1] + v[2] * u[2];
                        double adot = fabs(v[0] * u[0]) + fabs(v[1] * u[1]) + fabs(v[2] * u[2]);
                        double px = st.ph[0][ox], py = st.ph[1][oy], pz = st.ph[2][oz];
                        double dw[3] = {h * st.dph[0][ox] * py * pz,
                                        h * px * st.dph[1][oy] * pz,
                                        h * px * py * st.dph[2][oz]};
                        for (int d = 0; d < 3; ++d) {
                            nsum(&s[d], &c[d], dot * dw[d]);
                            m[d] += adot * fabs(dw[d]);
                        }
                    }
        }
        for (int d = 0; d < 3; ++d) {
            g[3 * k + d] = s[d] + c[d];
            if (scale) scale[3 * k + d] = m[d];
        }
    }
}

/* Host leaf and per-node leaf ids of each point (for tests that check the
 * node -> leaf reading).  nodes: (n, 27), -1 for dropped nodes. */
void orc_stencil_leaves(const orc_tree *t, const double *pos, int64_t n, int64_t *host,
                        int32_t *level, int64_t *nodes)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) {
        stencil st;
        int ok = build_stencil(t, pos + 3 * k, &st, 0);
        host[k] = ok ? st.host : -1;
        level[k] = ok ? st.level : -1;
        for (int q = 0; q < 27; ++q) nodes[27 * k + q] = ok ? st.leaf[q] : -1;
    }
}

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
