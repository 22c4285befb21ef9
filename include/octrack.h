/*
 * octrack.h -- C ABI of the MI355X (gfx950) Lagrangian-point tracking library.
 *
 * The library implements the Lagrangian-point tracking step of an immersed-
 * boundary / lattice-Boltzmann solver on an adaptive octree (Jiang,
 * Calzavarini & Krug, "Simulations of particle-laden flows with large
 * dispersed-phase size disparities using highly scalable parallel adaptive
 * methods"):
 *   - the octree as an array of leaves sorted by Morton (Z-order) index
 *     (Sec. 3.1, grid management);
 *   - host-cell search: every Lagrangian point is associated with the leaf
 *     that contains it (Sec. 3.2; Algorithm 1, search_host_cell);
 *   - interpolation of the leaf velocity field to the points and spreading of
 *     point forces back to the leaves with the 3-point regularized delta
 *     function (Sec. 2.2, the interpolation, spreading, W and phi equations).
 *
 * Conventions (all calls):
 *   - Domain: the unit cube, one root tree.  A leaf at level l with integer
 *     anchor a (units of 2^-L, L = l_max) is the half-open box
 *     [a, a + 2^(L-l)) on each axis.
 *   - Morton key of an anchor (x, y, z): bit b of x goes to bit 3b, of y to
 *     3b+1, of z to 3b+2.  Keys use 3L bits; L <= 21.
 *   - Leaf ids are ranks in the Morton-sorted leaf array (0 .. n_leaves-1).
 *     A point without a host leaf (NaN, outside a non-periodic domain,
 *     |x 2^L| >= 2^52) gets id -1; interpolate returns 0 for it and spread
 *     skips it.  That is not an error.
 *   - Integer coordinates of a point are floor(x 2^L) computed in FP64 for
 *     both precisions; periodic domains wrap them modulo 2^L.
 *   - Stencil: 3x3x3 level-l cells around the host cell, l = host leaf level;
 *     the value at a stencil node is the value of the leaf containing the
 *     node's centre; weight = phi(rx) phi(ry) phi(rz) (no cell-volume factor,
 *     so spread is the exact transpose of interpolate).  Non-periodic: nodes
 *     outside the cube are dropped.
 *   - pos, field, vel, force, grad arrays are row-major (rows, 3) in the
 *     dtype given (OT_F32 = float, OT_F64 = double), device memory.
 *   - Every pointer argument that names an array is a DEVICE pointer unless
 *     stated "host".  All arrays are owned by the caller; the library never
 *     frees them and keeps no reference after the call returns (except the
 *     batch plan, see below).
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls enqueue work
 *     and return; results are ready when the stream reaches them.  Only
 *     ot_build_tree synchronises (once, to report validation errors).
 *   - A tree handle is read-only after ot_build_tree: every call that needs
 *     working memory takes it from the caller (a `work` argument), from its
 *     batch plan, or allocates it on the call's stream, so calls on one tree
 *     may run on several streams at once.
 *   - Host ids (`ids` arguments marked "input"): the host leaf of every point
 *     as ot_locate returns it (Algorithm 1's host_cell_id, which Sec. 3.2
 *     makes the prerequisite of interpolation and spreading).  When given,
 *     the call takes each point's host from it instead of searching the
 *     tree; -1 or an id outside [0, n_leaves) means "no host".  NULL: the
 *     call searches.  Ids that are not the points' hosts give meaningless
 *     (but in-bounds) results.
 *   - Return value: OT_OK (0) or a negative OT_ERR_* code; ot_last_error()
 *     returns a message for the calling thread's last failure.
 */
#ifndef OCTRACK_H
#define OCTRACK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OT_OK                 0
#define OT_ERR_INVALID       -1   /* bad argument (null pointer, n < 0, bad enum, ...)      */
#define OT_ERR_NOT_PARTITION -2   /* leaves do not tile the unit cube exactly                */
#define OT_ERR_UNSORTED_DUP  -3   /* two leaves share a Morton key                           */
#define OT_ERR_LEVEL_RANGE   -4   /* L > 21, l_min > L, a leaf level outside [l_min, L] or a */
                                  /* key with bits above 3L                                  */
#define OT_ERR_OOM           -5   /* device allocation failed                                */
#define OT_ERR_HIP           -6   /* a HIP runtime call failed                               */
#define OT_ERR_CAPACITY      -7   /* more leaves than the id field holds (2^26)              */

#define OT_F32 0
#define OT_F64 1

/* Spreading accumulation.  ATOMIC: atomic adds, order dependent in the last
 * bits; workgroups sum their points' contributions in FP64 (for FP32 inputs
 * the exact products) and add each partial sum to field_out with one atomic
 * in the working precision (FP32 or FP64).  FIXED: every
 * contribution is rounded once to a signed 64-bit fixed-point value
 * q = rint(w F 2^s), ties to even, formed with one FP64 fused multiply-add
 * (exact product for FP32 inputs, the exact FP64 product rounded once for
 * FP64 inputs) and summed with integer adds, so
 * the result does not depend on execution order (bitwise reproducible).
 * s = min(62 - E, 51 - Ef) with 2^E >= n max|F| and 2^Ef >= max|F| (no leaf
 * sum can overflow, no contribution exceeds 2^51); max over finite
 * components.  The absolute error per contribution is at most 2^-(s+1).
 * Non-finite forces: ATOMIC mode carries a NaN or infinite component to the
 * leaves that point reaches, as FP arithmetic does; the integer sums of
 * FIXED mode cannot carry it, so there a force with a non-finite component
 * makes every value of the output field NaN. */
#define OT_SPREAD_ATOMIC 0
#define OT_SPREAD_FIXED  1

/* Operations of a fused / batched pass (bit flags). */
#define OT_OP_LOCATE      1   /* write host ids                       */
#define OT_OP_INTERPOLATE 2   /* write interpolated velocities        */
#define OT_OP_SPREAD      4   /* spread forces into the leaf field    */
/* Position gradient grad[k] = sum_n (force[k] . field[leaf(n)]) dw_kn/dX
 * (as ot_grad_pos with vec = force).  Batched plans only, alone or with one
 * of OT_OP_INTERPOLATE (backward of spreading: field = dLoss/dfield_out,
 * force = the forward forces) and OT_OP_SPREAD (backward of interpolation:
 * field = the forward field, force = dLoss/dvel); run with ot_batch_run_grad. */
#define OT_OP_GRAD_POS    8

typedef struct ot_tree ot_tree;
typedef struct ot_batch_plan ot_batch_plan;

typedef struct {
    int32_t l_min;     /* coarsest leaf level (>= 0)                                  */
    int32_t l_max;     /* finest leaf level L (<= 21); integer coordinates in 2^-L    */
    int32_t periodic;  /* 1: the unit cube is periodic on all three axes               */
} ot_tree_desc;

typedef struct {
    int64_t n_leaves;
    int32_t l_min, l_max, periodic;
    int32_t table_levels;    /* levels of the descent table (root + sub-tables)      */
    int64_t table_bytes;     /* device bytes of the descent table                    */
    int64_t workspace_bytes; /* bytes of a fixed-point spreading workspace (the       */
                             /* caller's `work`), = ot_spread_workspace_bytes        */
} ot_tree_info;

/* Tuning of the batched persistent pass.  Zero fields take defaults: 256
 * threads and 4 points per thread, narrowed (down to 64 threads, 1 point
 * per thread) when the run has too few points for two workgroups per CU;
 * sorted plans take tiles of about 160 x (points per leaf), the nearest
 * power of two between 1 and 4 points per thread. */
typedef struct {
    int32_t block;        /* threads per workgroup (multiple of 64, <= 512)           */
    int32_t tile;         /* points per tile (multiple of block)                      */
    int32_t grid;         /* persistent workgroups; 0 = as many as fit on the chip    */
    int32_t flags;        /* OT_TUNE_* bits                                           */
} ot_tuning;

/* Sort the points by host leaf before the persistent pass: locate, then
 * 8-bit radix passes (all stable but the first) over the host ids down to groups of at most 64
 * consecutive ids (two passes up to 4 M leaves, three above) that carry
 * positions and forces into plan-owned buffers; the pass then visits the
 * points in that order and writes each result at its point's input row.
 * Neighbouring threads then share stencil nodes in cache and in the
 * workgroup's spreading table.  Needs the same ops for every instance. */
#define OT_TUNE_SORT_POINTS 1

/* Host-major pass for sorted plans whose instances interpolate or spread
 * (without gradient ops): each window of 256 sorted points is ranked by
 * host in LDS, every distinct host's 27 node leaves and field values are
 * taken once and shared by its points, and the points' spreading sums for
 * one host are added up in registers before one LDS add per node and
 * component (the same rounded fixed-point contributions, so FIXED results
 * are equal bit for bit).  Windows whose hosts are too spread out go to the
 * per-point pass.  Needs OT_TUNE_SORT_POINTS. */
#define OT_TUNE_HOST_MAJOR 2

/* Replay the plan's kernels through a captured HIP graph: one graph launch
 * per run instead of the plan's kernel launches (4 without point sorting,
 * 12 with it up to about 33 M points and 4 M leaves, more above), which
 * saves host time per run.  Off by default: on this GPU the graph launch
 * made a run about 7 us longer on 11 k points and no faster on 10^7. */
#define OT_TUNE_GRAPH 4

/* Morton keys of leaf anchors (Sec. 3.1: leaves are ordered along the
 * Z-curve).  anchors: (n, 3) uint32, each < 2^l_max.  keys: (n,) uint64.
 * Errors: OT_ERR_INVALID (null with n > 0, n < 0), OT_ERR_LEVEL_RANGE
 * (l_max outside [0, 21]).  Anchors >= 2^l_max are not checked here;
 * ot_build_tree rejects the resulting keys. */
int ot_encode_keys(const uint32_t *anchors, int64_t n, int32_t l_max, uint64_t *keys,
                   void *stream);

/* Build the searchable tree from its leaves (the Z-sorted leaf array of
 * Sec. 3.1 and Algorithm 1, plus a descent table that resolves 3 levels per
 * lookup).  keys: (n_leaves,) Morton keys of the anchors at l_max resolution,
 * any order; levels: (n_leaves,) uint8.  perm_out (nullable, (n_leaves,)
 * int32): perm_out[id] = input row of the leaf with that id, so callers can
 * reorder their leaf fields once.  On success *out receives a handle that
 * owns device copies of everything it needs; the inputs may be freed.
 * Errors: OT_ERR_INVALID, OT_ERR_LEVEL_RANGE, OT_ERR_NOT_PARTITION,
 * OT_ERR_UNSORTED_DUP, OT_ERR_CAPACITY, OT_ERR_OOM, OT_ERR_HIP.  Synchronises
 * `stream` once. */
int ot_build_tree(const uint64_t *keys, const uint8_t *levels, int64_t n_leaves,
                  const ot_tree_desc *desc, int32_t *perm_out, void *stream, ot_tree **out);

/* Release a tree (waits for the device to finish using it). */
int ot_destroy_tree(ot_tree *tree);

/* Sizes and parameters of a tree (host struct). */
int ot_tree_info_get(const ot_tree *tree, ot_tree_info *info);

/* Copy the sorted leaf keys (uint64) and levels (uint8) out; either pointer
 * may be NULL. */
int ot_tree_leaves(const ot_tree *tree, uint64_t *keys_out, uint8_t *levels_out, void *stream);

/* Host-cell search (Sec. 3.2, Algorithm 1): ids[k] = leaf containing
 * pos[k], or -1.  pos: (n, 3) dtype; ids: (n,) int32. */
int ot_locate(const ot_tree *tree, const void *pos, int32_t dtype, int64_t n, int32_t *ids,
              void *stream);

/* Interpolation (Sec. 2.2): vel[k] = sum over the 27 stencil nodes of
 * w_kn field[leaf(n)].  field: (n_leaves, 3) in leaf-id order.  ids: input
 * host ids (nullable, see the conventions). */
int ot_interpolate(const ot_tree *tree, const void *field, const void *pos, const int32_t *ids,
                   int32_t dtype, int64_t n, void *vel, void *stream);

/* Bytes of the workspace of fixed-point spreading on `tree`: a 256-byte
 * header and n_leaves x 3 int64 accumulators (0 for a NULL tree). */
int64_t ot_spread_workspace_bytes(const ot_tree *tree);

/* Spreading (Sec. 2.2): field_out[j] (+)= sum_k sum_{n: leaf(n) = j} w_kn
 * force[k], the exact transpose of ot_interpolate.  accumulate = 0 overwrites
 * field_out, 1 adds to it.  mode: OT_SPREAD_ATOMIC or OT_SPREAD_FIXED.  ids:
 * input host ids (nullable).  work: FIXED mode's workspace, a 256-byte
 * aligned device buffer of ot_spread_workspace_bytes(tree) bytes owned by
 * the caller (calls sharing one must not overlap); NULL: the call allocates
 * it on `stream` (hipMallocAsync) and frees it there.  ATOMIC mode ignores
 * it.  Errors: OT_ERR_INVALID (NULL arrays, bad mode/dtype, n < 0, misaligned
 * work), OT_ERR_OOM, OT_ERR_HIP. */
int ot_spread(const ot_tree *tree, const void *force, const void *pos, const int32_t *ids, int32_t dtype,
              int64_t n, int32_t mode, int32_t accumulate, void *field_out, void *work, void *stream);

/* Fixed-point spreading for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): ot_spread with its workspace taken from a static device array
 * of 256 + 24 * OT_NOALLOC_MAX_LEAVES bytes (about 24 MiB) that the library
 * holds on every device it runs on until the process ends.  The call
 * allocates nothing; the caller still passes inputs and outputs.  Every call
 * on one device shares that device's array: calls that overlap on one
 * device (several streams or threads) race and give wrong results.  The
 * array keeps the last call's contents; each call clears what it needs.
 * FIXED mode only uses the array (ATOMIC mode runs ot_spread, which
 * allocates nothing in that mode).  Errors: as ot_spread, and
 * OT_ERR_CAPACITY for a tree with more than OT_NOALLOC_MAX_LEAVES leaves in
 * FIXED mode, OT_ERR_INVALID when the current device is not the tree's. */
#define OT_NOALLOC_MAX_LEAVES 1048576
int ot_spread_noalloc(const ot_tree *tree, const void *force, const void *pos, const int32_t *ids,
                      int32_t dtype, int64_t n, int32_t mode, int32_t accumulate, void *field_out,
                      void *stream);

/* One fused pass over the points: host search, interpolation of `field`
 * and spreading of `force` share the stencil.  ops: OT_OP_* bits; ids
 * (output of the search), vel, force/field_out may be NULL when their op is
 * off.  field_out is overwritten (accumulate = 0) or added to (1).  work: as
 * ot_spread. */
int ot_track(const ot_tree *tree, int32_t ops, const void *field, const void *force,
             const void *pos, int32_t dtype, int64_t n, int32_t mode, int32_t accumulate,
             int32_t *ids, void *vel, void *field_out, void *work, void *stream);

/* Position gradient through the delta-function derivative (the phi
 * equation of Sec. 2.2, differentiated branch by branch):
 * grad[k, d] = sum_n (vec[k] . field[leaf(n)]) dw_kn/dX_d with
 * dw/dX_d = 2^l phi'(r_d) prod_{e != d} phi(r_e), the host leaf held fixed.
 * ids: input host ids (nullable).  grad: (n, 3).
 *
 * ot_interp_grad_pos: gradient of sum_k grad_vel[k] . vel[k] for
 * vel = ot_interpolate(field) at pos, i.e. ot_grad_pos(field, vec = grad_vel).
 * ot_spread_grad_pos: gradient of sum_j grad_field[j] . field_out[j] for
 * field_out = ot_spread(force) at pos, i.e. ot_grad_pos(grad_field, vec = force). */
int ot_grad_pos(const ot_tree *tree, const void *field, const void *vec, const void *pos,
                const int32_t *ids, int32_t dtype, int64_t n, void *grad, void *stream);
int ot_interp_grad_pos(const ot_tree *tree, const void *field, const void *grad_vel, const void *pos,
                       const int32_t *ids, int32_t dtype, int64_t n, void *grad_pos, void *stream);
int ot_spread_grad_pos(const ot_tree *tree, const void *grad_field, const void *force, const void *pos,
                       const int32_t *ids, int32_t dtype, int64_t n, void *grad_pos, void *stream);

/* Backward of ot_interpolate in one pass over the points (the adjoint pair
 * of Sec. 2.2: spreading is the transpose of interpolation), sharing the
 * host search and the 27 node lookups:
 *   grad_field (+)= spread(grad_vel)            (as ot_spread, mode/accumulate)
 *   grad_pos    = ot_grad_pos(field, grad_vel)   (host leaf held fixed).
 * field: (n_leaves, 3) forward field; grad_vel: (n, 3) dLoss/dvel.  Either
 * output may be NULL (not computed), not both unless n = 0 (then the call
 * only clears grad_field when given and accumulate = 0).  grad_field: (n_leaves, 3);
 * grad_pos: (n, 3).  ids: input host ids (nullable); work: FIXED mode's
 * workspace, as ot_spread.  Errors: OT_ERR_INVALID for NULL inputs that an
 * output needs, a bad mode or dtype, n < 0. */
int ot_interp_backward(const ot_tree *tree, const void *field, const void *grad_vel, const void *pos,
                       const int32_t *ids, int32_t dtype, int64_t n, int32_t mode, int32_t accumulate,
                       void *grad_field, void *grad_pos, void *work, void *stream);

/* Backward of ot_spread in one pass over the points:
 *   grad_force = interpolate(grad_field)          (as ot_interpolate)
 *   grad_pos   = ot_grad_pos(grad_field, force)   (host leaf held fixed).
 * grad_field: (n_leaves, 3) dLoss/dfield_out; force: (n, 3) forward forces.
 * Either output may be NULL, not both unless n = 0 (then nothing is done);
 * both are (n, 3) and overwritten.  ids: input host ids (nullable).  Errors
 * as ot_interp_backward. */
int ot_spread_backward(const ot_tree *tree, const void *grad_field, const void *force, const void *pos,
                       const int32_t *ids, int32_t dtype, int64_t n, void *grad_force, void *grad_pos,
                       void *stream);

/* Multi-direct forcing of the immersed-boundary method (IBM subsection of
 * Sec. 2.2), n_iter iterations of:
 *   u_k = interpolate(field) at the markers pos,
 *   F_k = (target_k - u_k) / dt,
 *   f   = spread(F_k) to the leaves (mode: OT_SPREAD_ATOMIC or FIXED),
 *   field += f / rho.
 * field: (n_leaves, 3), updated in place.  pos, target: (n, 3) markers and
 * their prescribed velocities.  force_lag (nullable, (n, 3)) receives the
 * sum over the iterations of F_k, force_eul (nullable, (n_leaves, 3)) the sum
 * of f (the total forcing of the time step).  work: caller-owned device
 * buffer of ot_mdf_workspace_bytes(tree, n, dtype) bytes, 8-byte aligned;
 * the call allocates nothing and enqueues kernels only (no memset), so it
 * can be captured in a graph.  Once per call every marker's 27 node leaves
 * and weights are computed and kept, the leaves they reach listed and the
 * (marker, node) pairs grouped by leaf; each iteration then gathers through
 * the kept stencils and sums each listed leaf's pairs (no atomic adds).
 * Results are those of the plain composition of ot_interpolate and
 * ot_spread (FIXED: bit for bit; ATOMIC: each leaf's sum in FP64, rounded
 * once).  The tree is only read: calls on one tree may run concurrently
 * with their own workspaces.  At most 159,072,862 markers (OT_ERR_CAPACITY).
 * Errors: OT_ERR_INVALID (null arrays, n < 0, n_iter < 0, dt or rho not
 * positive, bad mode/dtype,
 * misaligned work), OT_ERR_HIP. */
int64_t ot_mdf_workspace_bytes(const ot_tree *tree, int64_t n, int32_t dtype);

/* Per-body sums of the IBM coupling (Sec. 2.3, fully resolved bodies).  For
 * body b = 0..n_body-1, owning points [offsets[b], offsets[b+1]):
 *   sum_out[b]    = sum_k vec_k dV_k,
 *   moment_out[b] = sum_k (pos_k - centres[b]) x vec_k dV_k,
 * with pos_k - centres[b] taken as the nearest periodic image when
 * periodic != 0 (unit cube).  With vec = marker forces these are minus the
 * IBM force and torque on the body; with vec = velocity interpolated at
 * points inside the body, the enclosed fluid's linear and angular momentum
 * divided by rho_f.  vec, pos: (n, 3) dtype; offsets: device (n_body + 1,)
 * int64, ascending (segments are clamped to [0, n]); centres: (n_body, 3)
 * dtype; dv: (n,) dtype, or NULL to use dv_all for every point.  Outputs are
 * FP64 (n_body, 3), summed in FP64 in a fixed order (bitwise reproducible).
 * Errors: OT_ERR_INVALID, OT_ERR_HIP. */
int ot_body_sums(const void *vec, const void *pos, int64_t n, const int64_t *offsets, int32_t n_body,
                 const void *centres, const void *dv, double dv_all, int32_t dtype, int32_t periodic,
                 double *sum_out, double *moment_out, void *stream);

/* Mean IBM-force subtraction (Sec. 5.2: in a fully periodic box the
 * domain average of the IBM forcing is removed at every step, so that the
 * dispersed phase exerts no net force on the fluid).  The leaf field is
 * constant over each leaf's cube, so its average over the unit cube is
 *   mean[c] = sum_j field[j][c] 2^(-3 l_j)
 * (summed in FP64 with a fixed grid and a fixed order: the same bits on
 * every run), and with subtract != 0 every leaf then gets
 * field[j][c] - mean[c] (formed in FP64, rounded once to dtype).  field:
 * (n_leaves, 3) dtype, in place; mean_out: device FP64 (3,), required.
 * work: 8-byte aligned device buffer of ot_force_mean_workspace_bytes()
 * bytes, or NULL (allocated on the stream).  The spreading output of this
 * library is a force density when the forces were scaled by dV_k / dx_l^3
 * (no cell-volume factor in the weights).  Errors: OT_ERR_INVALID,
 * OT_ERR_OOM, OT_ERR_HIP. */
int64_t ot_force_mean_workspace_bytes(void);
int ot_force_mean(const ot_tree *tree, void *field, int32_t dtype, int32_t subtract, double *mean_out,
                  void *work, void *stream);

/* Phase I of the migration of Lagrangian points (Algorithm 2), one device.
 *
 * ot_relocate: ids (n,) holds each point's previous host leaf id (or -1) on
 * entry and its host after the move on exit, identical to ot_locate; moved
 * (nullable, device int64 scalar) receives the number of points whose id
 * changed (the leavers).  Every point descends the table: with one or two
 * table loads per point that is cheaper here than checking the previous
 * host first, which the paper does to skip a binary search.
 *
 * ot_leaf_splitters: the partition of the leaves into P contiguous Morton
 * ranges of equal leaf count (Sec. 3.1): splitters (device int64, P + 1)
 * with splitters[0] = 0, splitters[r] = key of leaf floor(r n_leaves / P),
 * splitters[P] = 8^l_max.  1 <= P <= min(4096, n_leaves).
 *
 * ot_find_owner: owner[k] (n,) = the rank r with splitters[r] <= key <
 * splitters[r+1], key = Morton key of the point's finest-level cell
 * floor(x 2^l_max) (wrapped when periodic); -1 for a point with no cell.
 * counts (nullable, device int64 (P,)) receives the number of points per
 * rank (send-buffer sizes).  1 <= P <= 4096.  Errors: OT_ERR_INVALID,
 * OT_ERR_LEVEL_RANGE, OT_ERR_HIP. */
int ot_relocate(const ot_tree *tree, const void *pos, int32_t dtype, int64_t n, int32_t *ids,
                int64_t *moved, void *stream);
int ot_leaf_splitters(const ot_tree *tree, int32_t P, int64_t *splitters, void *stream);
int ot_find_owner(const int64_t *splitters, int32_t P, int32_t l_max, int32_t periodic, const void *pos,
                  int32_t dtype, int64_t n, int32_t *owner, int64_t *counts, void *stream);

/* Parameters of the point-particle step (physical units). */
typedef struct {
    double dt0;      /* time step at level l_min; level l uses dt0 / 2^(l - l_min)  */
    double r_p;      /* particle radius                                              */
    double rho_p;    /* particle density                                             */
    double rho_f;    /* fluid density                                                */
    double nu;       /* kinematic viscosity                                          */
    double g[3];     /* gravitational acceleration                                   */
    int32_t first;   /* 1: forward Euler (no history yet), 0: Adams-Bashforth 2      */
    int32_t reserved;
} ot_particle_params;

/* One step of point-like particles (Sec. 2.3): host leaf, fluid velocity u
 * by trilinear interpolation at the host level (the 8 level-l cells around
 * x 2^l - 1/2, each read from the leaf containing its centre; periodic wrap,
 * nodes beyond walls dropped), Re = 2 r_p |u - v| / nu,
 * a = (1 + 0.15 Re^0.687)(u - v) / tau + (1 - rho_f / rho_p) g with
 * tau = 2 rho_p r_p^2 / (9 rho_f nu), then
 *   v <- v + dt_l (3/2 a - 1/2 acc_prev),  x <- x + dt_l (3/2 v - 1/2 vel_prev)
 * (forward Euler when params->first), x wrapped into the periodic cube, and
 * ids <- host after the move.  vel_prev and acc_prev receive this step's v
 * and a.  A particle with no host does not move.  All arrays (n, 3) dtype
 * except ids (n,) int32, updated in place; field (n_leaves, 3).  Physical
 * units: the previous acceleration needs no rescale when the host level
 * changes (the paper's lattice-unit rescale is that unit change).
 * Errors: OT_ERR_INVALID, OT_ERR_HIP. */
int ot_particle_step(const ot_tree *tree, const void *field, void *pos, void *vel, void *vel_prev,
                     void *acc_prev, int32_t *ids, int32_t dtype, int64_t n,
                     const ot_particle_params *params, void *stream);

/* Host ordering of point particles: the particle state reordered by host
 * leaf, i.e. in the Z-order of the leaves (Sec. 3.1), so that the particle
 * step's node lookups and field reads of neighbouring particles share cache
 * lines.  A simulation keeps its particles in this order and re-sorts every
 * few steps (particles move by less than a cell per step, Sec. 2.3).
 * Reads the (n, 3) dtype arrays pos, vel, vel_prev, acc_prev and writes them
 * reordered to pos_out, vel_out, vel_prev_out, acc_prev_out (distinct from
 * the inputs and from each other: OT_ERR_INVALID otherwise).  ids_out (n,) int32: the host leaf of each output row, -1 for
 * a particle without one; perm_out (n,) int32: the input row of each output
 * row; either may be NULL.  Stable: particles of one host keep their input
 * order, particles without a host come last.  n < 2^31.  work: 256-byte
 * aligned device buffer of ot_particle_sort_workspace_bytes(n) bytes, or
 * NULL (allocated and freed on the stream).  The state is copied bit for
 * bit.  Errors: OT_ERR_INVALID, OT_ERR_OOM, OT_ERR_HIP. */
int64_t ot_particle_sort_workspace_bytes(int64_t n);
int ot_particle_sort(const ot_tree *tree, int32_t dtype, int64_t n, const void *pos, const void *vel,
                     const void *vel_prev, const void *acc_prev, void *pos_out, void *vel_out,
                     void *vel_prev_out, void *acc_prev_out, int32_t *ids_out, int32_t *perm_out,
                     void *work, void *stream);
int ot_mdf(const ot_tree *tree, void *field, const void *pos, const void *target, int32_t dtype,
           int64_t n, int32_t n_iter, double dt, double rho, int32_t mode, void *force_lag,
           void *force_eul, void *work, void *stream);

/* Batched pass over many point sets of uneven size (bubbles' markers and
 * particle groups) in one persistent launch (with OT_TUNE_GRAPH, the
 * plan's launches replay as one HIP graph).
 * offsets: host (n_inst + 1,) int64, ascending, offsets[0] = 0; instance i
 * owns points [offsets[i], offsets[i+1]).  ops: host (n_inst,) OT_OP_* bits
 * per instance.  Tiles of <= tuning.tile points never straddle instances.
 * The plan copies offsets/ops; it keeps the tree pointer (destroy the plan
 * before the tree).  A FIXED plan that spreads owns its spreading workspace,
 * so plans on one tree may run on different streams at once.  With
 * OT_TUNE_SORT_POINTS an instance with ops = 0 must be empty
 * (OT_ERR_INVALID otherwise). */
int ot_batch_plan_create(const ot_tree *tree, const int64_t *offsets, const int32_t *ops,
                         int32_t n_inst, int32_t dtype, int32_t mode, const ot_tuning *tuning,
                         ot_batch_plan **out);

/* Run a plan: like ot_track over all instances (field_out overwritten).
 * The plan's kernels are enqueued on the stream.  With OT_TUNE_GRAPH the
 * first run with a given set of pointers captures them in a graph, and
 * later runs with the same set replay it on the stream. */
int ot_batch_run(ot_batch_plan *plan, const void *field, const void *force, const void *pos,
                 int32_t *ids, void *vel, void *field_out, void *stream);

/* Run a plan whose instances carry OT_OP_GRAD_POS (ops 8, 10 or 12 each; a
 * plan does not mix them with forward-only ops): as ot_batch_run, and the
 * position gradient of every such point goes to grad ((n, 3) dtype).  With
 * point sorting the per-point vector (force) travels with the positions.
 * Errors: OT_ERR_INVALID for NULL arrays the ops need, or a plan without
 * gradient ops; ot_batch_run refuses plans with them. */
int ot_batch_run_grad(ot_batch_plan *plan, const void *field, const void *force, const void *pos,
                      int32_t *ids, void *vel, void *field_out, void *grad, void *stream);

/* Timing of the persistent kernel: with enable = 1, ot_batch_run enqueues
 * the plan's sequence directly on the caller's stream (not through the
 * graph, whose captured events cannot be timed) with a pair of HIP events
 * recorded just before and after the persistent kernel;
 * ot_batch_last_kernel_ms returns the kernel's duration in the last
 * completed run (OT_ERR_HIP while it is still in flight).  enable = 0 returns
 * to the plan's usual launches (graph replays for OT_TUNE_GRAPH plans). */
int ot_batch_plan_timing(ot_batch_plan *plan, int32_t enable);
int ot_batch_last_kernel_ms(const ot_batch_plan *plan, float *ms);

/* Tiles and workgroups a plan uses (host ints, either may be NULL). */
int ot_batch_plan_shape(const ot_batch_plan *plan, int64_t *n_tiles, int32_t *grid);

/* Host-major plans (OT_TUNE_HOST_MAJOR): the number of 256-point windows
 * (0 for other plans) and how many of them the last completed run handed to
 * the per-point pass (host ints, either may be NULL).  Synchronises with the
 * device to read the count. */
int ot_batch_plan_windows(const ot_batch_plan *plan, int64_t *n_windows, int64_t *handed_over);

int ot_batch_plan_destroy(ot_batch_plan *plan);

/* Static message for an error code; message of this thread's last error. */
const char *ot_strerror(int32_t code);
const char *ot_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* OCTRACK_H */
