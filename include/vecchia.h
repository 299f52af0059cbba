/* vecchia.h -- C ABI of the MI355X (gfx950) block Vecchia library.
 *
 * The library evaluates the block Vecchia approximation of a zero-mean
 * Gaussian-process log-likelihood with a Matern covariance:
 *
 *   l(theta) = sum_i log p(y_{B_i} | y_{N_i})                 eq. (vecchia-vector)
 *
 * where B_1..B_bc is an ordered partition of the points into blocks
 * (K-means clusters in random order, Section 2.1) and N_i holds the m_i
 * points of earlier blocks nearest to the centroid of B_i (Alg. 1,
 * preprocessing).  Each block term is computed by the chain of Alg. 1
 * (Cholesky of the neighbour covariance, triangular solves, Schur update,
 * Cholesky of the conditional covariance, log-determinant and quadratic
 * form), fused into one workgroup per block.
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - All work is enqueued on `stream` (a hipStream_t passed as void*;
 *     NULL = the default stream).  Calls return after enqueueing; outputs are
 *     valid once the stream has been synchronised.  Entry points that must
 *     know a device-side count on the host (noted below) synchronise the
 *     stream themselves.
 *   - Locations are row-major n x d doubles, d in {1, 2, 3}.  Index arrays
 *     are int32 (n < 2^31) unless typed otherwise.
 *   - The caller owns every buffer, including the workspaces; the library
 *     keeps no global state (apart from compiled kernels) and does not
 *     allocate device memory.  Calls on different streams with different
 *     workspaces may run concurrently.
 *   - Return value: VECCHIA_OK or a negative vecchia_status for argument or
 *     launch errors only.  Numerical outcomes (non-positive-definite
 *     blocks, FP32 re-factorisations) are reported in-band through the
 *     `counters` output.
 */
#ifndef VECCHIA_H
#define VECCHIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VECCHIA_OK = 0,
  VECCHIA_EINVAL = -1,        /* bad argument (size, pointer, ordering) */
  VECCHIA_ENOMEM = -2,        /* workspace or output capacity too small */
  VECCHIA_EHIP = -3,          /* a HIP runtime call or launch failed */
  VECCHIA_EUNSUPPORTED = -4   /* valid input outside what this build supports */
} vecchia_status;

typedef enum {
  VECCHIA_FP64 = 0,       /* all arithmetic in FP64 */
  VECCHIA_FP32_BULK = 1,  /* covariance, factorisations and solves in FP32; per-block
                             log-det and quadratic form accumulated in FP64; cross-block
                             sum in FP64; blocks whose FP32 pivots fall below the guard
                             are re-factorised in FP64 */
  VECCHIA_FP32_BULK_FORCE_REFACTOR = 2  /* test hook: FP32-bulk with every block flagged,
                                           so every block is re-factorised in FP64 */
} vecchia_precision;

/* Matern parameters, eq. (maternkernel), plus a nugget and per-axis ranges:
 *   C(s_i, s_j) = sigma2 * rho_nu(h / range) + nugget * [i == j],
 *   h = || (s_i - s_j) / aniso ||  (componentwise division; aniso = {1,1,1}
 *   is isotropic).  nu = 0.5, 1.5, 2.5 use the closed forms rho = e^-x,
 *   (1+x) e^-x, (1 + x + x^2/3) e^-x; any other nu in [0.05, 10] uses
 *   rho = 2^(1-nu)/Gamma(nu) x^nu K_nu(x), evaluated in FP64 (Temme's series
 *   for x <= 2, the trapezoidal rule on the integral representation of K for
 *   x > 2, upward recurrence in the order) by the one-wave kernels
 *   only: other engines, blocks above VECCHIA_MAX_JOINT and the simulator
 *   return VECCHIA_EUNSUPPORTED for it, as for nu outside [0.05, 10].  The
 *   nugget applies to same-index pairs only (not to distinct points at
 *   distance zero). */
typedef struct {
  double sigma2;
  double range;
  double nugget;
  double nu;
  double aniso[3];
} vecchia_theta;

/* Version of this ABI (major*10000 + minor*100 + patch). */
int vecchia_version(void);

/* Text for a vecchia_status value (static storage). */
const char* vecchia_status_string(int status);

/* ---------------------------------------------------------------- blocks --
 * Clustering g and block permutation zeta (Section 2.1; Alg. 1, preprocessing).
 * Lloyd's K-means in metric-scaled coordinates x = s * metric_scale, started
 * from the points init_idx[0..bc) and run until no assignment changes or
 * max_iter iterations.  An empty cluster is re-seeded with the point farthest
 * from its centroid.  Clusters are then ordered by block_perm (position i
 * holds cluster block_perm[i]; empty clusters are dropped) and points inside
 * a block keep ascending original index.
 *   locs         n x d, original order
 *   metric_scale host, d doubles (NULL = all ones)
 *   init_idx     bc int64 distinct point indices
 *   block_perm   bc int64, a permutation of 0..bc-1
 *   perm         out, n int64: re-ordered position -> original index
 *   block_ptr    out, bc+1 int32 CSR offsets of blocks in re-ordered points
 *   bc_out       host out: number of non-empty blocks (<= bc)
 *   iters_out    host out (may be NULL): Lloyd iterations run
 *   workspace    >= vecchia_blocks_workspace_size(n, bc, d) bytes
 * Synchronises `stream` (the block count is needed on the host). */
size_t vecchia_blocks_workspace_size(int64_t n, int64_t bc, int32_t d);
int vecchia_blocks(const double* locs, int64_t n, int32_t d, const double* metric_scale,
                   const int64_t* init_idx, const int64_t* block_perm, int64_t bc, int32_t max_iter,
                   int64_t* perm, int32_t* block_ptr, int64_t* bc_out, int32_t* iters_out,
                   void* workspace, size_t ws_bytes, void* stream);

/* Row gather dst[i, :] = src[perm[i], :] for an n x d double array (locations
 * or, with d = 1, data) -- the re-ordering of points into block order.
 * Asynchronous. */
int vecchia_permute(const double* src, int64_t n, int32_t d, const int64_t* perm, double* dst, void* stream);

/* ------------------------------------------------------------- neighbors --
 * Conditioning sets (Alg. 1, nearest neighbours; Section 2.2): for block i,
 * the m_i = min(m, block_ptr[i]) points of blocks 0..i-1 nearest to the
 * block centroid, sorted by (squared distance, index).  The centroid is the
 * mean of the block's metric-scaled points summed in order; squared
 * distances are FP64 sums (c_k - s_k*w_k)^2, k ascending, without fused
 * multiply-add, so results are reproducible bit for bit.  m = -1 selects
 * every earlier point (ascending index).
 *   locs_perm    n x d, block order (locs[perm])
 *   block_ptr    bc+1 int32
 *   nbr_ptr      out, bc+1 int32 CSR offsets (written by the call)
 *   nbr_idx      out, capacity nbr_cap int32 indices into the re-ordered points
 *   workspace    >= vecchia_neighbors_workspace_size(n, bc, d, m) bytes
 * Returns VECCHIA_ENOMEM if sum_i m_i exceeds nbr_cap.  Synchronises `stream`. */
size_t vecchia_neighbors_workspace_size(int64_t n, int64_t bc, int32_t d, int32_t m);
int vecchia_neighbors(const double* locs_perm, int64_t n, int32_t d, const double* metric_scale,
                      const int32_t* block_ptr, int64_t bc, int32_t m,
                      int32_t* nbr_ptr, int32_t* nbr_idx, int64_t nbr_cap,
                      void* workspace, size_t ws_bytes, void* stream);

/* Block orderings (Section 2.1): instead of the random order of
 * vecchia_blocks, order the blocks by their centroids (mean of the block's
 * metric-scaled points).
 *   VECCHIA_ORDER_MORTON  Z order: each centroid coordinate to a cell of a 2^B
 *                         grid over the centroids' bounding box (B = 63, 32,
 *                         21 for d = 1, 2, 3), bits interleaved with axis 0
 *                         lowest, sorted by key then block index
 *   VECCHIA_ORDER_MAXMIN  first the block nearest the mean centroid (summed in
 *                         block order), then each next block maximises the
 *                         minimum squared distance to the blocks placed (ties:
 *                         lowest index); O(bc^2) work, one workgroup up to
 *                         8,192 blocks, one launch pair per step above
 *   VECCHIA_ORDER_HILBERT the Morton cells, keyed by their distance along the
 *                         Hilbert curve of order B (Skilling's transform; in
 *                         1-D the cell order), sorted by key then block index
 *   VECCHIA_ORDER_KDTREE  leaves of a k-d tree from left to right: median
 *                         splits with the axis cycling with depth (depth mod
 *                         d); a node's blocks sorted by (coordinate, block
 *                         index), the first floor(k/2) to the left child
 * vecchia_reorder_blocks takes points already grouped into blocks (locs_perm,
 * block_ptr) and returns
 *   block_order    out, bc int64: position -> current block index
 *   point_perm     out, n int64: new point order as indices into locs_perm
 *   block_ptr_out  out, bc+1 int32 for the new order
 * Apply point_perm with vecchia_permute, then search neighbours.
 *   workspace  >= vecchia_reorder_blocks_workspace_size(n, bc, d) bytes
 * Synchronises `stream` (Morton, Hilbert: the bounding box goes through the
 * host). */
#define VECCHIA_ORDER_MORTON 1
#define VECCHIA_ORDER_MAXMIN 2
#define VECCHIA_ORDER_HILBERT 3
#define VECCHIA_ORDER_KDTREE 4
size_t vecchia_reorder_blocks_workspace_size(int64_t n, int64_t bc, int32_t d);
int vecchia_reorder_blocks(const double* locs_perm, int64_t n, int32_t d, const double* metric_scale,
                           const int32_t* block_ptr, int64_t bc, int32_t method, int64_t* block_order,
                           int64_t* point_perm, int32_t* block_ptr_out, void* workspace, size_t ws_bytes,
                           void* stream);

/* Kernel families.
 * VECCHIA_ENGINE_MFMA (default): each block's bordered joint matrix lives in
 *   16 x 16 matrix-core accumulator tiles of ONE wave (a 64-thread workgroup).
 *   The Cholesky runs in panels of four columns with rank-4 MFMA updates; the
 *   adjoint's back-substitution and contraction are MFMA products.  Up to
 *   G = 9 tile rows (FP64) or G = 10 (FP32) the factor stays in the registers
 *   through the adjoint (the inverses of its diagonal tiles are formed during
 *   the factorisation) and the l_i + 2 right-hand sides run in passes of 28
 *   (32 at G = 10); at G = 9 only when they fit one pass.  Otherwise the
 *   factor goes to the auxiliary tile buffer (FP32 G = 11: a factorisation
 *   launch, then an adjoint launch; FP64 G = 10, 11: the same with a
 *   left-looking factorisation that holds one tile column in the registers at
 *   a time) and the right-hand sides run in passes of up to 32, so any l_i
 *   fits the LDS.  The FP64 value kernels above G = 9 exceed the register
 *   file and spill part of the tiles.
 * VECCHIA_ENGINE_MFMA_WG: the same tiles spread over the four waves of a
 *   workgroup, for every size class (two barriers per panel).
 * VECCHIA_ENGINE_TILES: one register tile per thread, one barrier per column
 *   (vector ALU only). */
typedef enum { VECCHIA_ENGINE_MFMA = 0, VECCHIA_ENGINE_TILES = 1, VECCHIA_ENGINE_MFMA_WG = 2 } vecchia_engine;

/* ------------------------------------------------------------------ plan --
 * Launch schedule for one (block_ptr, nbr_ptr) pair: blocks are grouped into
 * size classes by p_i = m_i + l_i so that each class runs the kernel
 * configuration that fits it.  Build once per data set, reuse for every
 * likelihood evaluation.  The struct is host memory owned by the caller; its
 * device arrays live in the caller's workspace, which must stay allocated
 * while the plan is used.  Synchronises `stream`.
 *   max_theta    largest ntheta that later calls will pass
 *   workspace    >= vecchia_plan_workspace_size(bc, max_theta) bytes
 * Blocks with m_i + l_i above VECCHIA_MAX_JOINT (up to 16383) form a size class
 * of their own: each is generated into a global workspace slot and factored
 * left-looking in 16-column panels with MFMA panel updates;
 * vecchia_loglik_grad and vecchia_loglik_grad_nu return VECCHIA_EUNSUPPORTED
 * for plans that contain such blocks (their adjoint kernel is built but
 * switched off).
 * Auxiliary workspace: plan->aux_ws_bytes bytes (0 when not needed), attached
 * with vecchia_plan_attach_aux before the first evaluation, holds the large
 * blocks' slots and, after them, for engine MFMA, the per-block factor tiles of the
 * size classes whose adjoint goes through the tile buffer (at most 4 GiB;
 * the adjoint launches in chunks that fit it).  A smaller
 * buffer is accepted down to the size that holds every large-block slot and
 * one work item's FP64 factor tiles of the largest class that uses the tile
 * buffer (else
 * VECCHIA_ENOMEM): the size classes then run one after another, the adjoint
 * in as many launches as the buffer needs, and plan->aux_ws_bytes is lowered
 * to the attached size.  One plan's calls must not overlap in time (they
 * share both workspaces). */
#define VECCHIA_MAX_BUCKETS 24
#define VECCHIA_MAX_JOINT 175  /* largest m_i + l_i (both engines) */
typedef struct {
  int64_t n, bc;
  int32_t max_theta;
  int32_t nbuckets;
  int32_t pmax, lmax, mmax;
  int32_t bucket_cfg[VECCHIA_MAX_BUCKETS];     /* kernel configuration of each class */
  int64_t bucket_off[VECCHIA_MAX_BUCKETS + 1]; /* class ranges in the schedule array */
  int64_t lsum;                                /* sum of l_i (= n when blocks cover all points) */
  double flops_la;                             /* sum_i (p_i^3/3 + p_i^2): algorithmic LA flops */
  double cov_entries;                          /* sum_i p_i (p_i + 1) / 2 */
  void* ws;
  size_t ws_bytes;
  size_t off_sched, off_partial, off_flag, off_list, off_count, off_chunk, off_grad;
  void* timing;   /* NULL unless vecchia_plan_set_timing enabled per-launch timing */
  int32_t engine; /* vecchia_engine of the kernels this plan schedules */
  int64_t nlarge;            /* blocks with m_i + l_i > VECCHIA_MAX_JOINT */
  int32_t large_slots;       /* large blocks factored concurrently */
  int64_t large_slot_elems;  /* elements per large-block slot */
  size_t aux_ws_bytes;       /* auxiliary workspace needed (vecchia_plan_attach_aux) */
  void* aux_ws;
  int32_t bucket_lmax[VECCHIA_MAX_BUCKETS];  /* largest l_i of each class */
  int32_t lds_bytes;                          /* device LDS limit per workgroup */
  int32_t bucket_main;                        /* class with the most blocks */
  void* exec;      /* side streams and events of concurrent size classes (vecchia_plan_destroy) */
  int32_t kind;    /* 0 likelihood plan, 1 prediction plan (VECCHIA_PLAN_PREDICT) */
} vecchia_plan;

/* Layout of vecchia_plan as compiled into the library, for bindings that
 * mirror the struct (for instance through ctypes): out[0] = sizeof(vecchia_plan),
 * out[1 + k] = offsetof of the k-th field in declaration order.  Writes at most
 * cap entries (out may be NULL) and returns the number of entries.  Host only;
 * a binding compares these with its own mirror at load and refuses to run on
 * a mismatch. */
int32_t vecchia_plan_layout(int64_t* out, int32_t cap);
size_t vecchia_plan_workspace_size(int64_t bc, int32_t max_theta);
/* Name of the kernel that size class q of a plan runs for a value call
 * (with_grad = 0) or a value + gradient call in the given precision, for
 * profiles and benchmark reports, e.g. "bv_wave_kernel<float,9,5>" (one-wave
 * kernel, FP32, G = 9 tile rows, mode 5: gradient with the factor kept in
 * registers; mode 1: through the tile buffer; "...,2>+...,3>": the split
 * gradient, factorisation then adjoint; "...,6>+...,3>": the same with the
 * left-looking factorisation).  Host only.  VECCHIA_EINVAL for a bad
 * class index, VECCHIA_ENOMEM if cap bytes cannot hold the name. */
int vecchia_plan_class_kernel(const vecchia_plan* plan, int32_t q, int32_t precision, int32_t with_grad,
                              char* name, int32_t cap);
/* Tile configuration of a size class (plan->bucket_cfg[q]) of an engine: tile
 * size R and tile-grid order G (joint capacity R*G; the matrix-core engine has
 * R = 16 and holds the bordered matrix, p + 1 <= 16 G).  VECCHIA_EINVAL for an
 * unknown configuration. */
int vecchia_tile_config(int32_t engine, int32_t cfg, int32_t* R, int32_t* G);
/* engine may carry VECCHIA_PLAN_PREDICT (with VECCHIA_ENGINE_MFMA and
 * max_theta = 1): a plan for vecchia_predict over blocks of new locations,
 * sized by pred_rows(m_i) + l_i where pred_rows rounds m_i up to a multiple
 * of 4 (every block must fit VECCHIA_MAX_JOINT, else VECCHIA_EUNSUPPORTED).
 * The likelihood entry points reject prediction plans. */
#define VECCHIA_PLAN_PREDICT 16
int vecchia_plan_init(vecchia_plan* plan, const int32_t* block_ptr, const int32_t* nbr_ptr,
                      int64_t n, int64_t bc, int32_t max_theta, int32_t engine,
                      void* workspace, size_t ws_bytes, void* stream);
int vecchia_plan_attach_aux(vecchia_plan* plan, void* aux_workspace, size_t bytes);
/* Releases what vecchia_plan_init created on the host side (side streams,
 * events, timing records); call it before re-initialising or dropping a plan.
 * The workspaces stay the caller's. */
int vecchia_plan_destroy(vecchia_plan* plan);

/* Per-launch timing for benchmarks.  When enabled, vecchia_loglik and
 * vecchia_loglik_grad bracket every size-class kernel launch with hipEvents
 * recorded on the call's stream (host-side objects; no device memory).
 * vecchia_plan_timing synchronises those events and returns, per size class
 * q < plan->nbuckets, the summed milliseconds of its main kernel launches and
 * their count, and at index plan->nbuckets the summed span from the first
 * class launch to the last of each call (the classes run concurrently on the
 * plan's side streams), so ms and launches need nbuckets + 1 entries;
 * reset != 0 clears the record.  Disabling frees the events. */
int vecchia_plan_set_timing(vecchia_plan* plan, int enable);
int vecchia_plan_timing(vecchia_plan* plan, double* ms, int64_t* launches, int reset);

/* ---------------------------------------------------------------- loglik --
 * Block Vecchia log-likelihood (Alg. 1) for ntheta parameter vectors.
 *   plan         from vecchia_plan_init on the same block_ptr / nbr_ptr
 *   locs_perm    n x d, block order;  y_perm: n doubles, block order
 *   nbr_idx      neighbour indices (every index of block i < block_ptr[i])
 *   theta        host, ntheta values (ntheta <= plan->max_theta)
 *   precision    vecchia_precision
 *   loglik       out, ntheta doubles
 *   counters     out or NULL, 2*ntheta int32: [t*2+0] blocks re-factorised in
 *                FP64 by the FP32 guard, [t*2+1] blocks that were not positive
 *                definite even in FP64 (then loglik[t] is NaN)
 *   partial      out or NULL, ntheta*bc doubles: per-block terms l_i,
 *                [t*bc + i]
 * The FP32 guard flags a block when a pivot d_k (the diagonal before the
 * square root, in either Cholesky) is not finite or falls below
 * max(nugget/2, p_i * 2^-23 * (sigma2 + nugget)). */
int vecchia_loglik(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                   const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                   const vecchia_theta* theta, int32_t ntheta, int32_t precision,
                   double* loglik, int32_t* counters, double* partial, void* stream);

/* -------------------------------------------------------- loglik_noalloc --
 * For callers that cannot allocate device memory at call time (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * value path of vecchia_loglik, same arguments and results bit for bit, but
 * the per-call buffers (per-block terms, guard flags, the FP64 re-run list and
 * its counters) live in a static device array of the library instead of the
 * plan's workspace.  The call itself allocates nothing.
 *   - The array holds VECCHIA_NOALLOC_SCRATCH_BYTES bytes (about 16 MiB) on
 *     each GPU the library runs on, until the process ends; its device
 *     address is resolved once per device by vecchia_plan_init (or by the
 *     first call on that device).
 *   - plan->bc * ntheta above VECCHIA_NOALLOC_MAX_ITEMS: VECCHIA_ENOMEM.
 *   - Plans with blocks above VECCHIA_MAX_JOINT: VECCHIA_EUNSUPPORTED (those
 *     blocks are factored in the auxiliary workspace).  No auxiliary
 *     workspace is needed otherwise.
 *   - Every call on one GPU uses that GPU's one array: calls that overlap in
 *     time on the same GPU (other streams, other threads, other plans) race
 *     and must be serialised by the caller.  The plan's workspace still
 *     provides the block schedule (read only). */
#define VECCHIA_NOALLOC_MAX_ITEMS (1 << 20)
#define VECCHIA_NOALLOC_SCRATCH_BYTES ((size_t)16777472)
size_t vecchia_noalloc_scratch_bytes(void);
int vecchia_loglik_noalloc(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                           const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                           const vecchia_theta* theta, int32_t ntheta, int32_t precision,
                           double* loglik, int32_t* counters, double* partial, void* stream);

/* ----------------------------------------------------------- loglik_grad --
 * Log-likelihood and its gradient w.r.t. (sigma2, range, nugget) for each
 * theta.  The gradient is the adjoint of the per-block chain of Alg. 1,
 * evaluated without storing any factor: each workgroup re-factorises its
 * block, back-substitutes once with L_J^T for [alpha | b | R^T] and contracts
 * against the covariance derivatives regenerated on the fly, where
 *   d l_i = 1/2 [alpha^T dK_J alpha - b^T dK_N b - <K_J^-1 - K_N^-1, dK_J>].
 * "range" is the common scale: with anisotropy, d/d(range) scales every axis.
 * Arguments as vecchia_loglik, plus
 *   grad      out, 3*ntheta doubles [t*3 + k], k = (sigma2, range, nugget)
 *   gpartial  out or NULL, ntheta*bc*3 doubles, per-block gradient rows
 * The FP32-bulk path re-runs guard-flagged blocks (value and gradient) in FP64. */
int vecchia_loglik_grad(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                        const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                        const vecchia_theta* theta, int32_t ntheta, int32_t precision,
                        double* loglik, double* grad, int32_t* counters, double* partial, double* gpartial,
                        void* stream);

/* -------------------------------------------------------- loglik_grad_nu --
 * Log-likelihood and its gradient w.r.t. (sigma2, range, nugget) and the
 * Matern smoothness nu (eq. (maternkernel)), as estimated in Section 3: the
 * adjoint of vecchia_loglik_grad with one more contraction,
 *   d l_i / d nu = 1/2 <W, sigma2 d rho / d nu>,
 * where d rho / d nu = 2^(1-nu)/Gamma(nu) x^nu [K_nu (log x - log 2 -
 * psi(nu)) + d K_nu / d nu], and d K_nu / d nu is the trapezoidal rule on
 * int_0^inf t exp(-x cosh t) sinh(nu t) dt (at the reduced order, raised by
 * the differentiated recurrence).  Every nu in [0.05, 10], including the
 * half-integers, goes through the Bessel-form kernels, so the plan must use
 * engine VECCHIA_ENGINE_MFMA with no block above VECCHIA_MAX_JOINT (else
 * VECCHIA_EUNSUPPORTED).  Arguments as vecchia_loglik_grad, plus
 *   dnu          out, ntheta doubles: d l / d nu
 *   gpartial_nu  out or NULL, ntheta*bc doubles: per-block d l_i / d nu */
int vecchia_loglik_grad_nu(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                           const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                           const vecchia_theta* theta, int32_t ntheta, int32_t precision,
                           double* loglik, double* grad, double* dnu, int32_t* counters, double* partial,
                           double* gpartial, double* gpartial_nu, void* stream);

/* ------------------------------------------------------------ loglik_dnu --
 * Derivative of the log-likelihood w.r.t. the Matern smoothness nu (eq.
 * (maternkernel)), for estimating nu together with the other parameters as
 * in Section 3.  A central difference of two FP64 evaluations at
 * nu (1 + rel_step) and nu (1 - rel_step), each clipped to [0.05, 10]; both
 * use the Bessel form, so the plan must use engine VECCHIA_ENGINE_MFMA with
 * no block above the one-wave limit.  Truncation error is of order
 * (rel_step nu)^2 |d3 l / d nu3| / 6, rounding error of order
 * 1e-16 |l| / (rel_step nu); rel_step = 1e-4 balances them for FP64.
 * (vecchia_loglik_grad_nu gives the same derivative from the adjoint.)
 *   theta, ntheta   host, as vecchia_loglik (precision is always FP64)
 *   rel_step        relative step, in (0, 0.1]
 *   dnu             out, device, ntheta doubles
 *   tmp             device scratch owned by the caller, 2*ntheta doubles
 *                   (the two log-likelihoods of each theta)
 * Returns VECCHIA_EINVAL for NULL pointers or rel_step outside (0, 0.1], and
 * the status vecchia_loglik gives for the shifted theta otherwise. */
int vecchia_loglik_dnu(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                       const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                       const vecchia_theta* theta, int32_t ntheta, double rel_step, double* dnu, double* tmp,
                       void* stream);

/* ------------------------------------------------------------ prediction --
 * Block Vecchia prediction (Section 2.4, Alg. 2).  The n_new new locations
 * are grouped into blocks B*_1..B*_bc (for instance vecchia_blocks on them,
 * then vecchia_permute into block order), and each block conditions on the m
 * observations nearest its centroid.
 *
 * vecchia_pred_neighbors: as vecchia_neighbors (same centroid, distance and
 * tie rule), but every observation is a candidate of every block:
 * m_i = min(m, n_obs); m = -1 selects all observations (exact kriging).
 *   locs_obs   n_obs x d observed locations
 *   locs_new   n_new x d new locations in block order
 *   block_ptr  bc+1 int32 offsets into locs_new (block_ptr[bc] = n_new)
 *   nbr_ptr    out, bc+1 int32;  nbr_idx: out, indices into locs_obs
 *   workspace  >= vecchia_pred_neighbors_workspace_size(n_obs, n_new, bc, d, m)
 * Synchronises `stream`. */
size_t vecchia_pred_neighbors_workspace_size(int64_t n_obs, int64_t n_new, int64_t bc, int32_t d, int32_t m);
int vecchia_pred_neighbors(const double* locs_obs, int64_t n_obs, const double* locs_new, int64_t n_new,
                           int32_t d, const double* metric_scale, const int32_t* block_ptr, int64_t bc, int32_t m,
                           int32_t* nbr_ptr, int32_t* nbr_idx, int64_t nbr_cap,
                           void* workspace, size_t ws_bytes, void* stream);

/* vecchia_predict: per block, in FP64, the conditional mean and covariance of
 * the new values given the neighbours' observations,
 *   mu_B = K(B,N) K(N,N)^-1 y_N,   Sigma_B = K(B,B) - K(B,N) K(N,N)^-1 K(N,B),
 * with the nugget on the diagonal of K(N,N) and K(B,B) (new noisy
 * observations) and never in K(B,N).  One wave per block eliminates only the
 * neighbour columns of the bordered joint matrix [[K(N,N), .], [K(B,N),
 * K(B,B)], [y_N^T, 0]]; the remaining Schur complement holds Sigma_B and -mu_B.
 *   plan       vecchia_plan_init(block_ptr, nbr_ptr, n_new, bc, 1,
 *              VECCHIA_ENGINE_MFMA | VECCHIA_PLAN_PREDICT, ...)
 *   y_obs      n_obs observed values
 *   theta      host, one parameter vector
 *   mean, var  out, n_new doubles each, in the block order of locs_new
 *   cov        out or NULL: bc * ldc * ldc doubles; block i's l_i x l_i
 *              covariance, row-major, at cov + i * ldc * ldc (ldc >= plan->lmax)
 * A block whose neighbour covariance is not positive definite gets NaN
 * outputs. */
int vecchia_predict(const vecchia_plan* plan, const double* locs_obs, const double* y_obs,
                    const double* locs_new, int32_t d, const int32_t* block_ptr, const int32_t* nbr_ptr,
                    const int32_t* nbr_idx, const vecchia_theta* theta, double* mean, double* var,
                    double* cov, int32_t ldc, void* stream);

/* vecchia_condsim: univariate conditional simulation (Section 2.4): R draws
 * mean_j + sqrt(var_j) z_rj per location; their sample mean and standard
 * deviation (divisor R - 1), the interval mean -/+ 1.959964 sd, and, when
 * y_true is given, stats = (PICP, MSPE): the fraction of true values inside
 * their interval and the mean squared difference between sample mean and
 * truth (Section 3).  The random numbers are inputs.
 *   z          R x n doubles, draw r of location j at z[r * n + j]; R >= 2
 *   smean, ssd, lo, hi   out or NULL, n doubles each
 *   stats      out, 2 doubles (required with y_true)
 *   workspace  >= vecchia_condsim_workspace_size(n) bytes */
size_t vecchia_condsim_workspace_size(int64_t n);
int vecchia_condsim(const double* mean, const double* var, int64_t n, const double* z, int32_t R,
                    const double* y_true, double* smean, double* ssd, double* lo, double* hi, double* stats,
                    void* workspace, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------- simulate --
 * Sequential Vecchia simulator (data generator of the synthetic workloads):
 * points in the given order, y_i = c_i^T y_{N(i)} + sqrt(s_i) z_i, where N(i)
 * (nbr_ptr / nbr_idx, every index < i) are earlier points, c_i = K_NN^-1 k_Ni and
 * s_i = k_ii - k_Ni^T c_i (FP64).  Neighbour lists for it come from
 * vecchia_neighbors with unit blocks (block_ptr = 0..n).  ntheta <= 24 data sets
 * that share the design (locations and neighbours) are drawn in one call.
 *   locs_ord  n x d, simulation order
 *   theta     host, ntheta parameter vectors
 *   z         ntheta x n innovations;  y: out, ntheta x n values
 *   workspace >= vecchia_simulate_workspace_size(n, nbr_ptr[n], ntheta) bytes
 * Every neighbour set must satisfy m_i + 1 <= VECCHIA_MAX_JOINT.
 * Synchronises `stream`. */
size_t vecchia_simulate_workspace_size(int64_t n, int64_t nnz, int32_t ntheta);
int vecchia_simulate(const double* locs_ord, int64_t n, int32_t d, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                     const vecchia_theta* theta, int32_t ntheta, const double* z, double* y,
                     void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------- warm start --
 * Kernels of the learned warm start (variogram features -> MLP -> theta_0).
 *
 * vecchia_variogram: binned empirical semivariogram of nsets data sets, each a
 * subset of k two-dimensional points (locs: nsets blocks of k x 2 doubles at
 * stride locs_stride elements, stride 0 = one shared design; y: nsets x k at
 * stride y_stride).  Pair (i, j), i < j, with 0 < h <= hmax goes to bin
 * floor(h / hmax * nbins) (FP64, clamped to nbins - 1); gamma_b = sum (y_i - y_j)^2 /
 * (2 N_b) (0 if N_b = 0).  features: out, nsets x (nslots * nbins) FP32, zero except
 * slot nu_slot[s]: gamma / subset variance.  gamma: out or NULL, nsets x nbins FP64.
 * nchunks: workgroups per data set (partial sums reduced in a fixed order).
 * nbins <= 64. */
size_t vecchia_variogram_workspace_size(int32_t nsets, int32_t nbins, int32_t nchunks);
int vecchia_variogram(const double* locs, int64_t locs_stride, const double* y, int64_t y_stride, int32_t nsets,
                      int32_t k, int32_t nbins, double hmax, const int32_t* nu_slot, int32_t nslots,
                      float* features, double* gamma, int32_t nchunks, void* workspace, size_t ws_bytes,
                      void* stream);

/* vecchia_gemm: C (M x N, row-major, ld ldc) = op(A) op(B) [+ bias] with
 * optional epilogue: act = 1 applies ReLU (Z, if non-NULL, receives the
 * pre-activation); mask != NULL zeroes entries where mask <= 0 (ReLU backward);
 * accumulate = 1 adds into C.  op(A) = A (M x K, ld lda) or A^T if ta (A stored
 * K x M); op(B) = B (K x N, ld ldb) or B^T if tb (B stored N x K).  use_bf16 = 1
 * rounds operands to BF16 (nearest even) and multiplies on the matrix cores
 * with FP32 accumulation; 0 uses FP32 FMAs.  All FP32 device arrays. */
int vecchia_gemm(const float* A, const float* B, float* C, const float* bias, const float* mask, float* Z,
                 int32_t M, int32_t N, int32_t K, int32_t lda, int32_t ldb, int32_t ldc, int32_t ta, int32_t tb,
                 int32_t act, int32_t accumulate, int32_t use_bf16, void* stream);

/* vecchia_mse: mean squared error over `total` entries; dout = 2 (out - target) /
 * total; loss_part[g] = workgroup g's share of the mean (sum them). */
int vecchia_mse(const float* out, const float* target, int32_t total, float* dout, double* loss_part,
                int32_t nparts, void* stream);

/* vecchia_colsum: out[n] = sum_m X[m * ld + n] (bias gradients). */
int vecchia_colsum(const float* X, int32_t M, int32_t N, int32_t ld, float* out, void* stream);

/* vecchia_adam: one Adam step (bias-corrected, step >= 1) on n FP32 parameters. */
int vecchia_adam(float* param, const float* grad, float* m, float* v, int64_t n, double lr, double beta1,
                 double beta2, double eps, int64_t step, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* VECCHIA_H */
