/*
 * vecchia.h -- C ABI of the MI355X Vecchia hot path (GraphGP method).
 *
 * The calls follow the statement of the problem in the paper: Alg. 1 takes
 * points X (N x d), a covariance kappa, the dense initial size n0, the
 * neighbour matrix C ((N - n0) x k) and the parallel batches B_1..B_L, and
 * produces v = F(xi) from white noise xi; the abstract lists the inverse
 * application, the log-determinant and kernel-parameter derivatives as the
 * other building blocks.
 *
 * Conventions shared by every call:
 *   - Return value: VECCHIA_OK (0) or a negative status.  The message of the
 *     last failing call on the calling thread is vecchia_last_error().  No C++
 *     exception crosses this boundary.
 *   - Host pointers are marked (host); device pointers (device) are HBM
 *     allocations of the caller: the library allocates no device memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device calls only enqueue work and return; they never synchronise the
 *     stream, except vecchia_status().
 *   - Storage order: every device array is indexed by storage position s in
 *     [0, N): the dense block occupies s < n0 (in tree-slot order) and then the
 *     batches follow in increasing depth.  graph_export() returns the mapping
 *     storage position -> input index ("order").
 *   - Sparse index: s' = s - n0 for s >= n0; Ns = N - n0.
 *   - Tiled layout of the per-point k-vectors (neighbours, coefficients): for
 *     64 consecutive sparse points, entry m of each point is contiguous:
 *     element (s', m) lives at ((s' / 64) * kp + m) * 64 + s' % 64, where kp
 *     is k rounded up to a compiled width (8, 16, 32 or 64); unused entries hold
 *     the neighbour index -1 and the coefficient 0.  Array length:
 *     ceil(Ns / 64) * kp * 64.
 *   - Precision: VECCHIA_FP64 computes everything in double.  VECCHIA_FP32
 *     stores coordinates, coefficients, sigma, v and xi as float and computes
 *     kernel values and level application in float, while the Cholesky
 *     pivots, the conditional variances and the log-determinant stay in
 *     double and each coefficient solve gets one refinement step with a
 *     double-accumulated residual.  The dense block is double in both.
 */
#ifndef VECCHIA_H
#define VECCHIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define VECCHIA_OK            0
#define VECCHIA_EINVAL       -1   /* bad argument, detected on the host before any launch */
#define VECCHIA_ENOMEM       -2   /* host allocation failed or workspace too small */
#define VECCHIA_ENOTPD       -3   /* a covariance block was not positive definite */
#define VECCHIA_EUNSUPPORTED -4   /* valid but not compiled (e.g. k > 64, n0 > 128) */
#define VECCHIA_EHIP         -5   /* a HIP runtime call failed */
#define VECCHIA_EBUDGET      -6   /* serving admission: request exceeds the HBM budget */
#define VECCHIA_EIO          -7   /* a graph file could not be opened, read or written, or is damaged */

#define VECCHIA_FP64 0
#define VECCHIA_FP32 1

#define VECCHIA_KMAX  64          /* largest compiled neighbour count */
#define VECCHIA_N0MAX 128         /* largest dense block (FP64 n0 x n0 in one workgroup's LDS) */

/* ---- covariance ---------------------------------------------------------- */
/* Stationary kernel kappa(r) of Sec. 2.1 (forms named by the workloads, and
 * the Matern family with smoothing nu of Fig. 1):
 *   kind 0 EXP: sigma^2 exp(-r/ell)                                (nu = 1/2)
 *   kind 1 M32: sigma^2 (1 + sqrt3 r/ell) exp(-sqrt3 r/ell)        (nu = 3/2)
 *   kind 2 SE : sigma^2 exp(-r^2/(2 ell^2))                        (nu -> infinity)
 *   kind 3 M52: sigma^2 (1 + a + a^2/3) exp(-a), a = sqrt5 r/ell   (nu = 5/2)
 *   kind 4 MATERN: sigma^2 2^(1-nu)/Gamma(nu) a^nu K_nu(a), a = sqrt(2 nu) r/ell,
 *          any nu in [VECCHIA_NU_MIN, VECCHIA_NU_MAX] (K_nu the modified Bessel
 *          function of the second kind; sigma^2 at r = 0).  Supported by
 *          vecchia_factor on FP64 views and at k = 64 on both precisions (the
 *          factors that evaluate covariances in double; then forward, inverse
 *          and logdet, which do not depend on the kernel); the FP32 factor at
 *          k <= 32, the fused forward, the tangent and both adjoints return
 *          VECCHIA_EUNSUPPORTED for it.
 * `nugget` is added only on the diagonal (a point with itself); `nu` is read
 * by kind 4 only. */
#define VECCHIA_NU_MIN 0.25
#define VECCHIA_NU_MAX 8.0
typedef struct vecchia_kernel {
    int32_t kind;
    double sigma;
    double ell;
    double nugget;
    double nu;
} vecchia_kernel;

/* ---- graph (host, int32) -------------------------------------------------- */
typedef struct vecchia_graph vecchia_graph;   /* opaque, owned by the library */

/* Sec. 2.2 and Sec. 2.1: orders the N points of x (host, row-major N x d,
 * finite doubles) in the bit-reversed left-balanced k-d tree order (split on
 * the dimension of widest extent, median by (coordinate, input index)),
 * finds for every slot i >= n0 the k nearest preceding slots (squared
 * distance ((dx*dx + dy*dy) + dz*dz) in double, ties to the smaller slot;
 * fewer than k predecessors pad with -1), computes the depths
 * d_i = 1 + max_{j in c(i)} d_j (Sec. 2.2, "Batch construction") and the
 * storage order (dense block, then batches by depth; inside a batch, in-order
 * rank of the tree, which is spatially coherent).
 * 1 <= d <= 3, 1 <= k <= VECCHIA_KMAX, 1 <= n0 <= n < 2^31.  n_threads <= 0
 * uses every hardware thread.  On success *out owns the graph; free it with
 * graph_free().  Errors: EINVAL (arguments, non-finite coordinates), ENOMEM. */
int graph_build(const double* x, int64_t n, int32_t d, int32_t k, int32_t n0,
                int32_t n_threads, vecchia_graph** out);

/* The same build with its neighbour search on the device (the preceding
 * k-NN query of Sec. 2.3's last paragraph), in three steps:
 *   graph_build_begin  orders the points (tree, as graph_build) and leaves the
 *                      graph pending; same arguments and errors as graph_build;
 *   graph_knn_nodes    exports the query tree for the device: nodes (host,
 *                      N * VECCHIA_KNN_NODE_BYTES bytes, in-order layout; the
 *                      caller copies them to the device) and rank_of (host,
 *                      N int32: tree slot -> node index);
 *   graph_knn_device   (device, enqueued on `stream`) writes rows (device,
 *                      (N - n0) x k int32, row r for tree slot n0 + r): the k
 *                      slots j < slot with the smallest (D, j), ascending,
 *                      -1 padded -- the rows graph_build computes on the host,
 *                      bit for bit;
 *   graph_build_finish takes the rows back (host, same layout), checks that
 *                      every entry names a preceding slot and that each row
 *                      ascends by (distance, slot) (EINVAL otherwise), then
 *                      computes depths and the storage order.
 * Until graph_build_finish succeeds, graph_export, graph_export_nbr and
 * graph_export_children return EINVAL.  Device buffers are the caller's. */
#define VECCHIA_KNN_NODE_BYTES 40
int graph_build_begin(const double* x, int64_t n, int32_t d, int32_t k, int32_t n0,
                      int32_t n_threads, vecchia_graph** out);
int graph_knn_nodes(const vecchia_graph* g, void* nodes, int32_t* rank_of);
int graph_knn_device(const void* nodes, const int32_t* rank_of, int64_t n, int32_t d, int32_t k, int32_t n0,
                     int32_t* rows, void* stream);
int graph_build_finish(vecchia_graph* g, const int32_t* rows);

/* The depths of Sec. 2.2 on the device, as the parallel fixpoint of their
 * recurrence (Sec. 2.3, last paragraph): the dense block (slots < n0) at 0,
 * every sparse slot i at d_i = 1 + max d_j over its row.  rows (device): as
 * graph_knn_device writes them; depth (device, N int32, tree slot order)
 * receives the depths; scratch (device) holds one int32.  Each sparse slot
 * starts at 1 and the sweeps raise it in place until a sweep changes nothing;
 * the fixpoint is unique, so the result does not depend on the order of the
 * updates.  Neighbours precede their point, so the slots are swept in
 * consecutive blocks, in order, each until it is stable (the blocks before it
 * are final).  The call synchronises `stream` every second sweep to test for
 * a change and returns when the depths are final; *sweeps (may be NULL)
 * receives the number of sweeps.  Errors: EINVAL, EHIP. */
int graph_depth_device(const int32_t* rows, int64_t n, int32_t k, int32_t n0, int32_t* depth, int32_t* scratch,
                       void* stream, int32_t* sweeps);

/* graph_build_finish with the depths given (host, N int32, tree slot order,
 * from graph_depth_device) instead of computed: they are checked against the
 * recurrence (EINVAL naming the first slot that breaks it), then the batches
 * and the storage order follow from them as in graph_build. */
int graph_build_finish_depth(vecchia_graph* g, const int32_t* rows, const int32_t* depth);

/* The bit-reversed left-balanced k-d tree of Sec. 2.2 on the device, by sort
 * passes (Sec. 2.3, last paragraph), one tree level at a time: per level a
 * stable radix sort of the points by their coordinate in their node's split
 * dimension, then by node, makes every node's set a run ordered by
 * (coordinate, input index); its point is the run's middle (rank |S|/2) and
 * the parts below and above are its children's sets.  The split dimension of
 * a node is the widest extent of its set (the lowest on ties).  The result is
 * the tree graph_build makes, bit for bit.
 *   x          (device) N x 3 doubles in input order, zero padded for d < 3;
 *   tree_perm  (device, N int32) receives slot -> input index;
 *   sdim       (device, N int32) receives each slot's split dimension;
 *   scratch    (device, 256-byte aligned) graph_tree_scratch_bytes(N) bytes
 *              (about 64 N bytes: keys, indices, per-node sizes and bounds,
 *              sort temporaries).
 * Enqueued on `stream`; the caller synchronises.  Errors: EINVAL, ENOMEM
 * (scratch too small), EHIP. */
int graph_tree_scratch_bytes(int64_t n, size_t* bytes);
int graph_tree_device(const double* x, int64_t n, int32_t d, int32_t* tree_perm, int32_t* sdim, void* scratch,
                      size_t scratch_bytes, void* stream);

/* graph_build_begin with the tree given (host arrays from graph_tree_device)
 * instead of built: the tree is checked against the points without being
 * rebuilt -- tree_perm a permutation, every split dimension the widest extent
 * of its subtree, every point of a left (right) subtree below (above) its
 * node's point by (coordinate, input index) -- and EINVAL names the first
 * slot that breaks it.  Otherwise as graph_build_begin (the graph is pending
 * until graph_build_finish / graph_build_finish_depth). */
int graph_build_begin_tree(const double* x, int64_t n, int32_t d, int32_t k, int32_t n0, int32_t n_threads,
                           const int32_t* tree_perm, const int32_t* sdim, vecchia_graph** out);

/* Sizes of a built graph (any pointer may be NULL).  kp = padded width of the
 * tiled layout; n_levels = number of sparse batches L. */
int graph_info(const vecchia_graph* g, int64_t* n, int32_t* d, int32_t* k, int32_t* kp,
               int32_t* n0, int32_t* n_levels);

/* Storage maps (host arrays, caller-allocated, any may be NULL):
 *   order[N]          storage position -> input index
 *   slot[N]           storage position -> tree slot (generation order)
 *   level_ptr[L + 2]  batch boundaries: level_ptr[0] = 0, level_ptr[1] = n0,
 *                     batch l (1..L) is [level_ptr[l], level_ptr[l+1])
 *   depth[N]          depth of each storage position (0 for the dense block) */
int graph_export(const vecchia_graph* g, int32_t* order, int32_t* slot, int32_t* level_ptr,
                 int32_t* depth);

/* Neighbour indices in storage positions (host, caller-allocated):
 * layout 0 = row-major Ns x k, rows in sparse-index order, each row in
 * ascending (distance, slot), as Sec. 2.1 selects them; layout 1 = the tiled
 * device layout (length ceil(Ns/64) * kp * 64), each row in ascending
 * storage position with padding (-1) last: the same conditioning sets, in
 * the order that keeps a wave's gathers on few cache lines.  Every device
 * array indexed by a row position (b, the packed children) follows layout 1. */
int graph_export_nbr(const vecchia_graph* g, int32_t layout, int32_t* nbr);

/* Coordinates in storage order, 3 per point (zero padded for d < 3), as
 * double (precision VECCHIA_FP64) or float (VECCHIA_FP32): host, N x 3.
 * EINVAL for a NULL argument, a bad precision or a pending graph. */
int graph_export_points(const vecchia_graph* g, int32_t precision, void* xs);

/* Children lists for the reverse sweep of the adjoint (host): for storage
 * position j, child[child_ptr[j] .. child_ptr[j+1]) are the packed entries
 * s' * kp + m of every sparse point s' whose neighbour at position m of its
 * layout-1 row is j, ascending.
 * child_ptr has N + 1 entries; child has Ns * k entries at most (the exact
 * count is child_ptr[N]).  EUNSUPPORTED if Ns * kp >= 2^31. */
int graph_export_children(const vecchia_graph* g, int64_t* child_ptr, int32_t* child);

/* Host time spent in the phases of graph_build, seconds: tree, neighbours,
 * depth, storage order.  times has 4 entries. */
int graph_build_times(const vecchia_graph* g, double* times);

/* Graph serialisation (host).  A built graph depends only on the points, k and
 * n0 (Sec. 2.1 and 2.2: tree order, preceding k-NN, depth batches), so it can
 * be written once and reused by later processes instead of being rebuilt.
 *   graph_save  writes a finished graph to `path` (created or truncated): a
 *               32-byte header (magic "VCGRAPH1", N int64, d, k, n0 int32,
 *               one reserved int32), then the input coordinates (N x d
 *               double, input order), the tree (slot -> input index, N int32;
 *               split dimension per slot, N int32), the neighbour rows in
 *               slot numbers ((N - n0) x k int32, ascending (distance, slot),
 *               -1 padded) and the depth per slot (N int32), all
 *               little-endian, and last the 64-bit FNV-1a hash of everything
 *               before it.
 *   graph_load  reads such a file into a new graph (*out, freed with
 *               graph_free).  The hash and the sizes are checked first; the
 *               content then goes through graph_build_begin_tree and
 *               graph_build_finish_depth, so the tree, the rows and the
 *               depths are checked as for a device build (a row is checked to
 *               name preceding slots in ascending order, not re-searched).
 *               n_threads as for graph_build.
 * Errors: EINVAL (NULL argument, graph still pending, the content fails a
 * check), EUNSUPPORTED (k above the compiled maximum), ENOMEM, EIO (open,
 * read or write failed, wrong magic, truncated file, hash mismatch). */
int graph_save(const vecchia_graph* g, const char* path);
int graph_load(const char* path, int32_t n_threads, vecchia_graph** out);

void graph_free(vecchia_graph* g);

/* ---- device factor ---------------------------------------------------------- */
/* A view of one factored point set.  Every pointer except level_ptr is a
 * device pointer owned by the caller; the view itself is plain data. */
typedef struct vecchia_view {
    int64_t n;                 /* N */
    int32_t k;                 /* neighbours per point */
    int32_t kp;                /* padded width of the tiled layout (graph_info) */
    int32_t n0;                /* dense block size */
    int32_t n_levels;          /* L */
    int32_t precision;         /* VECCHIA_FP64 or VECCHIA_FP32 */
    int32_t redo_log2;         /* VECCHIA_FP32: a point whose smallest Cholesky pivot is below
                                  2^-redo_log2 * K_ii, or not positive, is recomputed entirely in
                                  double (results stored as float).  0 = default (8); < 0 = only
                                  points whose float factorisation fails.  Ignored for FP64. */
    const void* x;             /* (device) N x 3 coordinates in storage order, double or float */
    const int32_t* nbr;        /* (device) tiled neighbour indices (graph_export_nbr layout 1) */
    const int32_t* level_ptr;  /* (host)   L + 2 batch boundaries (graph_export) */
    const int32_t* level_ptr_dev; /* (device) the same L + 2 boundaries, or NULL.  When set, runs of
                                     consecutive small batches of the forward pass are processed by one
                                     workgroup in a single launch instead of one launch per batch. */
    const int64_t* child_ptr;  /* (device) N + 1, only needed by vecchia_backward, else NULL */
    const int32_t* child;      /* (device) packed children, only for vecchia_backward, else NULL */
    void* workspace;           /* (device) vecchia_workspace_bytes() bytes, 256-byte aligned */
    size_t workspace_bytes;
    vecchia_kernel kernel;     /* written by vecchia_factor */
} vecchia_view;

/* Bytes of device workspace that hold a factor: coefficients b (tiled),
 * sigma, the dense factor L0 (n0 x n0 double), log-determinant partials and a
 * status word. */
int vecchia_workspace_bytes(int64_t n, int32_t k, int32_t n0, int32_t precision, size_t* bytes);

/* Eq. (2) for every sparse point at once, plus the dense initial batch:
 * gathers the coordinates of each point and of its k neighbours, assembles
 * K_cc, k_ci and K_ii, factors K_cc = L L^T, solves y = L^-1 k_ci,
 * b = L^-T y, sigma^2 = K_ii - y.y, and L0 = chol(K[0:n0, 0:n0]).  Writes the
 * workspace and view->kernel.  A non-positive pivot or conditional variance
 * is recorded in the workspace status word (see vecchia_status); nothing is
 * jittered.  Errors: EINVAL (view/kernel), ENOMEM (workspace too small),
 * EUNSUPPORTED, EHIP (launch failure). */
int vecchia_factor(vecchia_view* view, const vecchia_kernel* kern, void* stream);

/* Alg. 1: v[0:n0] = L0 xi[0:n0], then for every batch l = 1..L in order,
 * v_i = b_i . v[c(i)] + sigma_i xi_i.  xi and v are device arrays of N
 * elements (double or float per view->precision) in storage order; they must
 * not overlap.  One launch per batch; with view->level_ptr_dev set, runs of
 * consecutive small batches (<= 512 points) go to one workgroup each, with a
 * workgroup barrier between batches. */
int vecchia_forward(const vecchia_view* view, const void* xi, void* v, void* stream);

/* Alg. 1 as written, fused and on the fly (Sec. 2.3, Implementation: the
 * per-point quantities are computed where they are used instead of being
 * stored): v[0:n0] = L0 xi[0:n0] with L0 = chol(K[0:n0, 0:n0]), then for every
 * batch l = 1..L in order, each point i assembles K_cc, k_ci and K_ii from the
 * coordinates (view->x, view->nbr), factors K_cc = L L^T, solves y = L^-1 k_ci
 * and w = L^-1 v[c(i)] and sets
 *     v_i = y . w + sigma_i xi_i,   sigma_i^2 = K_ii - y . y,
 * which is Eq. (2)'s b_i . v[c(i)] + sigma_i xi_i without forming b_i.  No
 * coefficient or sigma is stored: the workspace (vecchia_fused_workspace_bytes,
 * 256-byte aligned, view->workspace / workspace_bytes) holds L0, per-tile log
 * sigma sums and a status word, O(n0^2 + N/8) bytes instead of the factor's
 * O(N k).  The arithmetic is double for both storage precisions; xi, v and
 * the coordinates are stored per view->precision, in storage order.  If
 * logdet (device, 1 double) is not NULL it receives the log-determinant of the
 * same pass (as vecchia_logdet).  The rest of the view is as for
 * vecchia_forward; view->kernel is not read.  A non-positive pivot or variance
 * is recorded for vecchia_fused_status.  Errors: EINVAL, ENOMEM (workspace
 * too small), EUNSUPPORTED, EHIP. */
int vecchia_fused_workspace_bytes(int64_t n, int32_t k, int32_t n0, int32_t precision, size_t* bytes);
int vecchia_forward_fused(const vecchia_view* view, const vecchia_kernel* kern, const void* xi, void* v,
                          double* logdet, void* stream);
/* As vecchia_status, for a view whose workspace holds a fused forward. */
int vecchia_fused_status(const vecchia_view* view, void* stream, int64_t* first_bad_slot);

/* Inverse application xi = F^-1(v): xi[0:n0] = L0^-1 v[0:n0] and
 * xi_i = (v_i - b_i . v[c(i)]) / sigma_i for every sparse point at once. */
int vecchia_inverse(const vecchia_view* view, const void* v, void* xi, void* stream);

/* log det of the Vecchia covariance F F^T = 2 (sum log L0_jj + sum log sigma_i),
 * summed in double with compensation, written to out (device, 1 double). */
int vecchia_logdet(const vecchia_view* view, double* out, void* stream);

/* Reverse-mode derivatives (Sec. 2.3) of
 *     <v_bar, F xi> + <xi_bar_in, F^-1 v> + logdet_bar * logdet
 * with respect to xi, v and theta = (sigma, ell):
 *   xi_bar  (device, N)   = F^T v_bar              (NULL allowed if v_bar NULL)
 *   v_bar_out (device, N) = F^-T xi_bar_in         (NULL allowed if xi_bar_in NULL)
 *   theta_bar (device, 2 doubles) = d/d(sigma, ell), accumulated in double.
 * xi and v are the forward pair (v = F xi) or the inverse pair; v_bar and
 * xi_bar_in may be NULL.  Needs view->child_ptr and view->child.  scratch is a
 * device buffer of vecchia_backward_scratch_bytes() bytes. */
int vecchia_backward_scratch_bytes(const vecchia_view* view, size_t* bytes);
int vecchia_backward(const vecchia_view* view, const vecchia_kernel* kern,
                     const void* xi, const void* v, const void* v_bar, const void* xi_bar_in,
                     double logdet_bar, void* xi_bar, void* v_bar_out, double* theta_bar,
                     void* scratch, size_t scratch_bytes, void* stream);

/* The same scalar's derivative with respect to the point coordinates
 * (Sec. 2.3: derivatives of the building blocks), at a fixed graph: the
 * order and the neighbour sets are piecewise constant in x and are held.
 * Every covariance entry kappa(|x_p - x_q|) of K_cc, k_ci and the dense block
 * passes its cotangent to both points through
 * d kappa / d x_p = kappa'(r) (x_p - x_q) / r (zero for coincident points).
 *   x_bar (device, N x 3 doubles, storage order, the third column zero for
 *          d < 3): the cotangent of view->x, in double for both precisions.
 * Inputs as vecchia_backward (v_bar, xi_bar_in may be NULL).  Each point's
 * share from the points that condition on it is gathered over the children
 * lists in a fixed order: the result does not depend on scheduling.
 * scratch: vecchia_backward_x_scratch_bytes() bytes (the backward's scratch,
 * the per-point outputs of the sweeps and 24 bytes per neighbour entry),
 * 256-byte aligned.  Errors: EINVAL, ENOMEM (scratch too small),
 * EUNSUPPORTED, EHIP. */
int vecchia_backward_x_scratch_bytes(const vecchia_view* view, size_t* bytes);
int vecchia_backward_x(const vecchia_view* view, const vecchia_kernel* kern, const void* xi, const void* v,
                       const void* v_bar, const void* xi_bar_in, double logdet_bar, double* x_bar, void* scratch,
                       size_t scratch_bytes, void* stream);

/* vecchia_backward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same derivatives, computed by the same kernels, with the scratch taken
 * from a fixed device array inside the library instead of a caller buffer.
 * Every GPU the library runs on holds its own copy of that array (64 MiB,
 * vecchia_backward_noalloc_max_bytes) from the library's load until the
 * process ends; a view whose vecchia_backward_scratch_bytes exceeds it (about
 * 8 million points) is rejected with VECCHIA_ENOMEM before anything is
 * launched.  The call allocates nothing (with per-kernel timing off).  All
 * calls on one GPU share the array and it keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other threads) race; nothing
 * in it needs to start at zero.  Other arguments and errors as
 * vecchia_backward. */
int vecchia_backward_noalloc_max_bytes(size_t* bytes);
int vecchia_backward_noalloc(const vecchia_view* view, const vecchia_kernel* kern,
                             const void* xi, const void* v, const void* v_bar, const void* xi_bar_in,
                             double logdet_bar, void* xi_bar, void* v_bar_out, double* theta_bar, void* stream);

/* Forward-mode derivatives (Sec. 2.3: forward and backward derivatives with
 * respect to the kernel parameters): the tangent of v = F(xi; sigma, ell) and
 * of the logdet in the direction (xi_dot, sigma_dot, ell_dot),
 *     v_dot = F(xi_dot) + (dF/dsigma sigma_dot + dF/dell ell_dot) xi.
 * Per sparse point, with K_dot = sigma_dot dK/dsigma + ell_dot dK/dell
 * (nugget excluded) and the stored b, sigma:
 *     b_dot = K_cc^-1 (k_dot_ci - K_dot_cc b),
 *     sigma_dot_i = (K_dot_ii - 2 k_dot_ci . b + b . K_dot_cc b) / (2 sigma_i),
 * then batch by batch v_dot_i = b_dot . v[c(i)] + b . v_dot[c(i)] +
 * sigma_dot_i xi_i + sigma_i xi_dot_i; the dense block uses the Cholesky
 * tangent L0_dot = L0 Phi(L0^-1 K0_dot L0^-T).  K_cc is recomputed per point
 * (double arithmetic).  xi and v (device, N, storage order) are the forward
 * pair of the factored view; xi_dot may be NULL (zero); v_dot (device, N)
 * receives the tangent; logdet_dot (device, 1 double, nullable) receives
 * 2 sum sigma_dot_i / sigma_i + tr(K0^-1 K0_dot).  scratch: device buffer of
 * vecchia_jvp_scratch_bytes() bytes, 256-byte aligned.  Errors: EINVAL,
 * ENOMEM (scratch too small), EHIP. */
int vecchia_jvp_scratch_bytes(const vecchia_view* view, size_t* bytes);
int vecchia_forward_jvp(const vecchia_view* view, const vecchia_kernel* kern, const void* xi, const void* v,
                        const void* xi_dot, double sigma_dot, double ell_dot, void* v_dot, double* logdet_dot,
                        void* scratch, size_t scratch_bytes, void* stream);

/* Synchronises `stream`, then reports how many points of the last
 * vecchia_factor had a non-positive pivot or variance (not_pd) and, for
 * VECCHIA_FP32, how many were recomputed in double (recomputed). */
int vecchia_factor_counts(const vecchia_view* view, void* stream, int64_t* not_pd, int64_t* recomputed);

/* Synchronises `stream`, then reads the workspace status word.  Returns
 * VECCHIA_OK, or VECCHIA_ENOTPD with *first_bad_slot = the smallest storage
 * position whose pivot or conditional variance was not positive (-1 if
 * none; the dense block reports its first bad pivot row). */
int vecchia_status(const vecchia_view* view, void* stream, int64_t* first_bad_slot);

/* ---- serving: continuous batching of requests on one GPU ----------------- */
/* Not a passage of the paper: a request loop around the calls above.  Each
 * request brings its own points (host, N x 3 doubles, input order), kernel,
 * k, n0 and one operation; the engine builds its graph on a host worker
 * thread, admits it when its whole device footprint fits in the free part of
 * the caller's HBM arena (FIFO in the order graphs become ready, so a slow
 * build does not block the requests behind it), runs upload + vecchia_factor + the
 * operation + download on one of its streams, and frees the arena range at
 * completion.  Requests on different streams overlap on the device.  All
 * computation is FP32 (VECCHIA_FP32).  Thread safety: one thread drives a
 * server (submit/progress/take/result/release); graph workers are internal. */
#define VECCHIA_OP_FORWARD 0   /* result = F(input), input = white noise, input order */
#define VECCHIA_OP_INVERSE 1   /* result = F^-1(input), input = field values */
#define VECCHIA_OP_LOGDET  2   /* result = log det (no input) */

typedef struct vecchia_server vecchia_server;

typedef struct vecchia_serve_stats {
    size_t arena_bytes, bytes_in_use, peak_bytes, largest_free;
    int64_t building, queued, running, admitted, completed, failed, rejected, cancelled;
    int64_t peak_running;   /* most requests resident on the device at once */
    int64_t graphs_on_device; /* graphs built through the device path (serve_set_graph_device) */
} vecchia_serve_stats;

/* arena: (device) 256-byte aligned buffer of arena_bytes owned by the caller
 * and not touched by it while the server lives (the HBM budget).  n_streams
 * in 1..64 (default priority), graph_workers host threads each running
 * graph_build; a request of n points builds with min(graph_threads,
 * max(1, n / 2^16)) threads, so that small graphs start no threads and large
 * ones (the tail of the latency) are built in parallel.  mock != 0: no
 * device calls at all
 * (arena may be NULL); a running request completes after 3 serve_progress
 * calls and returns its input (host tests of the scheduler). */
int serve_create(void* arena, size_t arena_bytes, int32_t n_streams, int32_t graph_workers, int32_t graph_threads,
                 int32_t mock, vecchia_server** out);

/* Device graph builds (Sec. 2.3, last paragraph: tree, neighbour search and
 * depths on the GPU): buffer (device, 256-byte aligned, owned by the caller
 * and not touched by it while the server lives) is split into one slice per
 * graph worker; a worker then builds the graph of a request of at least 2^15
 * points whose device build fits its slice (graph_tree_device,
 * graph_knn_device, graph_depth_device on a stream of its own, about
 * 64 N + 4 N k bytes), and every other graph on the host.  The graphs are the
 * same bit for bit.  NULL turns it off.  EINVAL for a mock server. */
int serve_set_graph_device(vecchia_server* s, void* buffer, size_t bytes);

/* Device bytes a request of N points needs (coordinates, tiled neighbours,
 * workspace, input, output). */
int serve_request_bytes(int64_t n, int32_t k, int32_t n0, size_t* bytes);

/* Copies x (host, N x 3) and input (host, N floats, input order; NULL for
 * logdet) and queues the request.  EBUDGET if it can never fit in the arena;
 * EINVAL on bad arguments.  *id > 0 identifies the request. */
int serve_submit(vecchia_server* s, const double* x, int64_t n, int32_t k, int32_t n0, const vecchia_kernel* kern,
                 int32_t op, const float* input, int64_t* id);

/* Non-blocking step of the engine: retires finished requests (frees their
 * arena ranges), admits queued ones in FIFO order while the head fits, and
 * enqueues their device work.  *n_completed = requests waiting in serve_take. */
int serve_progress(vecchia_server* s, int32_t* n_completed);

/* Pops the id of one finished request (0 if none). */
int serve_take(vecchia_server* s, int64_t* id);

/* Result of a finished request: out (host, N floats, input order) for
 * forward/inverse, *logdet for logdet; times[4] (seconds) = graph build,
 * queue wait, device time (admission to completion), total.  Returns the
 * request's own error if it failed. */
int serve_result(vecchia_server* s, int64_t id, float* out, double* logdet, double* times);

/* Frees the host copies of a finished or cancelled request. */
int serve_release(vecchia_server* s, int64_t id);

/* Cancels a request that is not yet admitted. */
int serve_cancel(vecchia_server* s, int64_t id);

int serve_stats(vecchia_server* s, vecchia_serve_stats* out);

/* Waits for the device work in flight, stops the workers, frees everything
 * except the caller's arena. */
void serve_destroy(vecchia_server* s);

/* Padded width used for a neighbour count k (8, 16, 32 or 64), or -1. */
int32_t vecchia_padded_k(int32_t k);

/* Per-kernel timing: when enabled, every launch made by the library is
 * bracketed by HIP events on its stream and its duration is accumulated per
 * kernel name (milliseconds).  Reading the totals synchronises the device.
 * names: buffer of `cap` bytes receiving '\n'-separated names. */
int vecchia_profile_enable(int32_t on);
int vecchia_profile_read(char* names, size_t cap, double* total_ms, int64_t* launches, int32_t max_kernels,
                         int32_t* n_kernels);
int vecchia_profile_reset(void);

/* sizeof(vecchia_view) and sizeof(vecchia_kernel) as compiled, for bindings
 * that mirror the structs (ABI check). */
int vecchia_abi_sizes(size_t* view_bytes, size_t* kernel_bytes);

const char* vecchia_last_error(void);
const char* vecchia_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VECCHIA_H */
