/*
 * h2.h -- C ABI of the MI355X H^2-ULV dense solver.
 *
 * Solves A x = b for a dense symmetric positive definite kernel matrix
 * A_ij = G(x_i, x_j) over points x_i, following Ma & Yokota, "An inherently
 * parallel H^2-ULV factorization for solving dense linear systems on GPUs"
 * (arXiv 2502.02395):
 *   h2_build   -- H^2 construction with pre-factorization (Algorithm 1,
 *                 Sections 3.4-3.5): cluster tree, shared bases whose span
 *                 includes the Schur-complement fill-ins, couplings, dense
 *                 near blocks;
 *   h2_factor  -- the level-by-level ULV factorization (Algorithm 4,
 *                 Section 4.4, Eq. 21, Eq. 32);
 *   h2_solve   -- the inherently parallel forward and backward substitution
 *                 (Section 3.7, Eq. 24-31), optionally followed by iterative
 *                 refinement / PCG against the FP64 H^2 operator;
 *   h2_matvec  -- the FP64 H^2 matrix-vector product.
 *
 * Conventions (all entry points):
 *   - Every call returns an h2_status; no exception or abort crosses the ABI.
 *   - Matrices are column-major.  Points are row-major (n x dim).
 *   - "host" pointers are read during the call only; "device" pointers must be
 *     HIP device allocations on the current device.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it; the call returns after the work that the
 *     call needs to inspect on the host (ranks during build, the breakdown flag
 *     after factor, residual norms during refinement) has completed.
 *   - The handle owns every device buffer it allocates (through
 *     h2_params.allocator, else hipMalloc) and frees them in h2_destroy.  A handle must not be used from two threads or two
 *     streams at once.
 *   - After an error other than H2_ERR_ARG the handle may only be inspected
 *     (h2_stats, getters) or destroyed.
 */
#ifndef H2_H
#define H2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  H2_OK = 0,
  H2_ERR_ARG = 1,         /* invalid argument (synchronous, handle unchanged)   */
  H2_ERR_ALLOC = 2,       /* device or host allocation failed                   */
  H2_ERR_HIP = 3,         /* a HIP runtime call failed                          */
  H2_ERR_NOT_SPD = 4,     /* Cholesky breakdown (LU variant: a zero or
                             non-finite pivot); h2_stats gives (level, box)    */
  H2_ERR_STATE = 5,       /* call out of order (e.g. solve before factor)       */
  H2_ERR_NOCONV = 6,      /* refinement did not reach the tolerance             */
  H2_ERR_UNSUPPORTED = 7  /* option not available in this library               */
} h2_status;

/* Kernel functions (Eq. 35, Eq. 36 regularised; covariance kernels). */
typedef enum {
  H2_K_LAPLACE_REG = 0,   /* 1/(r + delta)                                       */
  H2_K_YUKAWA_REG = 1,    /* exp(-kappa r)/(r + delta)                           */
  H2_K_GAUSSIAN = 2,      /* exp(-r^2/ell^2) + nugget [i == j]                   */
  H2_K_MATERN32 = 3,      /* (1 + sqrt3 r/ell) exp(-sqrt3 r/ell) + nugget [i==j] */
  H2_K_YUKAWA_DRIFT = 4   /* exp(-kappa r)/(r + delta) (1 + beta (x_0 - y_0)/(r + delta)):
                             the Yukawa kernel plus a skew part along the first
                             axis; non-symmetric for beta != 0                 */
} h2_kernel_id;

typedef struct {
  int32_t id;             /* h2_kernel_id */
  double delta, kappa, ell, nugget;
  double beta;            /* H2_K_YUKAWA_DRIFT only (ignored otherwise)          */
} h2_kernel;

/* Precision of the basis-transform GEMMs (h2_params.gemm_prec):
 *   FP64    FP64 MFMA on the FP64 factors;
 *   FP32    FP32 copies of the operands in HBM, FP32 MFMA, FP32 accumulation;
 *   BF16    the same FP32 copies rounded to BF16 on their way into LDS, BF16
 *           MFMA (16x16x32), FP32 accumulation (8-bit operands);
 *   BF16X3  the same FP32 copies split into BF16 high and low parts, three
 *           BF16 MFMAs per product (high*high + high*low + low*high), FP32
 *           accumulation: about 17-bit operands at a third of the BF16 rate.
 * The Cholesky factors, the root, the H^2 matvec and refinement stay FP64. */
typedef enum { H2_PREC_FP64 = 0, H2_PREC_FP32 = 1, H2_PREC_BF16 = 2, H2_PREC_BF16X3 = 3 } h2_prec;

/* Device memory of a handle.  Every device buffer the handle owns and every
 * temporary of the build comes from alloc(bytes, user), which returns NULL
 * on failure (the call then returns H2_ERR_ALLOC), and goes back through
 * free(ptr, user), which the library calls only after the device work that
 * used the buffer has completed (h2_destroy and failed builds synchronize
 * the device first).  The callbacks and `user` must stay valid until
 * h2_destroy.  A Python caller passes PyTorch's caching allocator here. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} h2_allocator;

typedef struct {
  int32_t dim;            /* 2 or 3                                              */
  int32_t leaf;           /* max points per leaf box (>= 2)                      */
  double eta;             /* admissibility: far iff |c_a-c_b| > eta (rho_a+rho_b) */
  double eps;             /* ID truncation: keep |R_jj| > eps |R_00|             */
  int32_t max_rank;       /* 0 = no cap                                          */
  int32_t s_far, s_near;  /* sample sizes per box; -1 = every candidate point    */
  int32_t gemm_prec;      /* h2_prec of the basis-transform / Schur GEMMs.  Every
                             reduced precision keeps the transforms' operands
                             and results in FP32 (FP32 copies of the bases and
                             near blocks), so the substitution then reads the
                             FP32 copies whatever solve_prec says; the Schur
                             update runs on FP32 MFMA                          */
  int32_t ir_max_iter;    /* 0 = plain direct solve                              */
  double ir_tol;          /* relative residual target of refinement              */
  int32_t use_pcg;        /* 1 = PCG instead of stationary refinement            */
  int32_t use_graph;      /* 1 = capture the factorization's launches in a hipGraph
                             (on the first h2_factor; replayed after), and in an
                             untimed h2_solve the launches of each substitution
                             and H^2 product (one graph per shape, captured on
                             first use).  Captures and replays run on a stream
                             of the handle, ordered after and before the
                             caller's stream by events.  h2_solve_noalloc
                             never captures                                   */
  const float* rank_model;/* host, 4801 MLP weights; NULL = plain pivoted QR    */
  double rank_margin;     /* predicted-rank buffer margin (fraction, e.g. 0.25) */
  int32_t timing;         /* 1 = time factor phases and solve gathers (events)   */
  int32_t no_autotune;    /* 1 = skip the tile-shape autotuner (64x64 tiles)     */
  int32_t solve_prec;     /* h2_prec (FP64, FP32 or BF16) in which the
                             substitution reads the factors: FP32 or BF16
                             copies of the transformed near blocks and bases
                             are made at the end of h2_factor (with a reduced
                             gemm_prec, FP32 copies exist anyway); products and
                             sums, the root, the H^2 matvec and the refinement
                             stay FP64.  The substitution is then a fixed
                             symmetric preconditioner of PCG                  */
  int32_t gs_sweeps;      /* pre-factorization of h2_build (Section 3.5): 0 =
                             exact Cholesky solve with the near-sample block
                             A_cc (LU variant: pivot-free LU); n > 0 = n
                             Gauss-Seidel sweeps (from zero) approximating
                             A_Close = G(B_i, S_C) A_cc^{-1} (LU variant: and
                             the column side with A_cc^T).
                             Range 0..64 (else H2_ERR_ARG); a non-positive
                             diagonal entry of A_cc returns H2_ERR_NOT_SPD
                             with the box in h2_stats                          */
  const h2_allocator* allocator; /* host; copied at build; NULL = hipMalloc and
                             hipFree                                          */
  int32_t matvec_prec;    /* h2_prec (FP64 or FP32) of the leaf near blocks and
                             couplings that PCG's iterations multiply with.
                             FP32: FP32 copies made at build, products and sums
                             FP64; when PCG's own residual reaches ir_tol the
                             residual is recomputed with the FP64 H^2 operator,
                             and PCG restarts from it while that one is above
                             ir_tol (at most 8 restarts).  The returned
                             residual is always the FP64 operator's.  Stationary
                             refinement ignores it                            */
  int32_t factor_lu;      /* 1 = the LU variant of the factorization and the
                             substitution (below) for a symmetric kernel too;
                             a handle with any non-symmetric kernel
                             (H2_K_YUKAWA_DRIFT, beta != 0) always uses it.
                             LU variant (the method stated for non-symmetric
                             matrices): one basis per box for its rows and
                             columns, from an interpolative decomposition of
                             the far field and the fill-in seen from both
                             sides; a pivot-free LU of every redundant block
                             with left and right bases
                             P_i = [Q_i^S | Q_i^R L(r)_ii^{-T}] and
                             P'_i = [Q_i^S | Q_i^R U(r)_ii^{-1}]; near blocks,
                             couplings and factors stored for every ordered
                             pair; the forward sweep of Eq. 31 with the lower
                             and the backward sweep with the upper factor.
                             It takes any gemm_prec, solve_prec FP64 or FP32
                             (the right basis has its own FP32 copy),
                             matvec_prec FP64 and use_pcg 0 (refinement is
                             stationary), else H2_ERR_ARG                     */
} h2_params;

typedef struct h2_ctx* h2_handle;

/* Per-handle statistics (h2_stats). */
typedef struct {
  int64_t n;              /* total points (all instances)                        */
  int32_t n_inst, levels; /* instances, max tree depth L                         */
  int64_t n_boxes;        /* boxes of levels 1..L over all instances             */
  int64_t near_pairs;     /* unordered near pairs incl. diagonal, all levels     */
  int64_t far_pairs;      /* unordered far pairs, all levels                     */
  int64_t leaf_near_blocks; /* ordered dense near blocks at the leaves (N_NZB)   */
  int32_t max_rank_seen, max_m_seen, root_n;
  double flops_factor;    /* canonical algorithmic flops of one factorization
                             (LU variant: the LU counts, every ordered pair)    */
  double flops_solve;     /* canonical flops of one solve, per right-hand side   */
  double bytes_factors;   /* bytes of the stored factors                         */
  double t_build, t_factor, t_solve; /* seconds of the last call (host clock)    */
  int32_t ir_iters;       /* refinement iterations of the last solve             */
  double ir_residual;     /* last relative residual against the H^2 operator     */
  int32_t fail_level, fail_box, fail_inst; /* location of a Cholesky breakdown   */
  int32_t rank_fallbacks; /* boxes whose predicted rank fell back to full QR     */
  double t_pair_gemm;     /* seconds in the near-pair transform launches of the
                             last factor (HIP events; params.timing = 1)         */
  double flops_pair_gemm; /* canonical flops of those launches: sum over
                             unordered near pairs of 2 m_i m_j (m_i + m_j)
                             (LU variant: over ordered pairs)                  */
  int32_t pair_launches;  /* number of those launches per factor                */
  double bytes_basis;     /* bytes allocated for the bases U_i (predicted
                             capacities plus fallbacks, or m_i^2 per box)       */
  int32_t tuned_lists;    /* GEMM work lists timed by the autotuner             */
  int32_t tuned_cfg_hist[4]; /* how many chose 64x64x16, 128x64x16, 128x128x16,
                                64x64x32 tiles (BM x BN x K-step)               */
  double t_gather[3];     /* seconds in the neighbour-gather launches of the last
                             solve: [0] block products on FP64 blocks, [1] on
                             FP32 copies, [2] per-box reductions (HIP events
                             around each launch; params.timing = 1)           */
  double bytes_gather[3]; /* algorithmic bytes of those launches: every stored
                             block once plus x slices and partial products;
                             for [2] partials, base and y once                */
  int32_t gather_launches[3]; /* number of timed launches of each kind           */
  double t_factor_phase[9]; /* seconds of the last factor per phase (HIP events;
                               params.timing = 1, no graph): basis QR, diagonal
                               transform, RR Cholesky + inverse, V and Schur
                               update, near-pair transforms, far couplings,
                               merge, root, FP32 copies for the substitution  */
  int64_t gather_partials;  /* doubles of gather partial products that one
                               right-hand side of a solve or matvec needs
                               (h2_solve_noalloc: at most H2_NOALLOC_PARTIALS) */
  double flops_factor_phase[9]; /* canonical flops of flops_factor by phase, in
                               the order of t_factor_phase: GEQRF + ORGQR_full,
                               4 m^3, r^3/3, m r^2 + k r^2 + k^2 r, near pairs
                               (2 m_i m_j (m_i + m_j) + r_i r_j^2 + k_i r_j^2 +
                               k_j r_i^2), far pairs k_i k_j (k_i + k_j), 0,
                               n0^3/3, 0.  LU variant: 2 r^3/3, 2 m r^2 +
                               2 k r^2 + 2 k^2 r, every ordered near and far
                               pair, 2 n0^3/3                                  */
  double flops_schur;       /* the k^2 r of phase 3 (the Schur update SS -=
                               L(s) L(s)^T, FP32 MFMA under a reduced
                               gemm_prec)                                      */
  double t_build_id;        /* seconds of the build spent in the pivoted-QR IDs
                               (host clock around each level's launch and the
                               rank readback that ends it)                     */
  double flops_prefactor;   /* canonical flops of the build's pre-factorization
                               (Section 3.5), summed over boxes with a near
                               sample of size c: c^3/3 + 2 c^2 m, or
                               2 c^2 m per Gauss-Seidel sweep                  */
  int32_t ir_fp64_matvecs;  /* FP64 H^2 products of the last solve (PCG with
                               matvec_prec FP32: the initial and every
                               recomputed residual)                            */
  double t_gather_mv32;     /* as t_gather, bytes_gather, gather_launches for
                               the products on FP32 copies of the near blocks
                               and couplings (matvec_prec FP32)                */
  double bytes_gather_mv32;
  int32_t gather_launches_mv32;
  int32_t lu_variant;       /* 1 if the handle uses the LU variant (factor_lu) */
} h2_stats_t;

/* Capacity, in doubles, of the fixed device array that h2_solve_noalloc uses
 * for its gather partial products (64 MiB per GPU). */
#define H2_NOALLOC_PARTIALS (1 << 23)

/* Build the H^2 representation of one kernel matrix (Algorithm 1).
 *  pts:   host, n x dim row-major points (copied).
 *  perm:  host, n int64, the sampling permutation pi of 0..n-1; S_F / S_C take
 *         the candidates that come first in pi.  NULL = identity.
 *  out:   receives the new handle.
 * Errors: H2_ERR_ARG for n < 1, a non-finite coordinate, leaf < 2, dim not 2/3,
 *         bad kernel id, eps < 0, an allocator without both callbacks;
 *         H2_ERR_ALLOC when a device allocation fails (everything allocated
 *         so far is freed);
 *         H2_ERR_NOT_SPD if a near-sample matrix G(S_C, S_C) is not SPD (LU
 *         variant: its pivot-free LU meets a zero or non-finite pivot): then
 *         *out receives a handle in the failed state whose h2_stats give the
 *         (level, box, instance); it accepts only h2_stats and h2_destroy.
 *         On every other error *out is NULL. */
h2_status h2_build(const double* pts, int64_t n, const h2_kernel* kernel,
                   const h2_params* params, const int64_t* perm, void* stream,
                   h2_handle* out);

/* Build many independent systems in one handle (same params, own points,
 * kernel and permutation each); every level of every instance is processed in
 * the same batched launches, instances aligned by height above the leaves.
 * pts[t]: host n[t] x dim; perms[t]: host or NULL. */
h2_status h2_build_batched(int32_t n_inst, const double* const* pts,
                           const int64_t* n, const h2_kernel* kernels,
                           const h2_params* params, const int64_t* const* perms,
                           void* stream, h2_handle* out);

/* Build with a prescribed skeleton selection instead of pivoted QR: for every
 * box of levels L..1 (level-major from the leaves, box-minor), ranks[b] and
 * skel[...] = the k_b skeleton positions into that box's active rows, in pivot
 * order, concatenated.  The ID coefficients are then computed on the device.
 * Single instance only.  Used to run the factorization on an identical H^2
 * matrix as an external reference. */
h2_status h2_build_fixed(const double* pts, int64_t n, const h2_kernel* kernel,
                         const h2_params* params, const int64_t* perm,
                         const int32_t* ranks, const int32_t* skel,
                         void* stream, h2_handle* out);

/* Factor (Algorithm 4; the LU variant for handles with factor_lu).  Returns
 * H2_ERR_NOT_SPD with the location in h2_stats if a redundant diagonal block
 * or the root is not positive definite (LU variant: meets a zero or
 * non-finite pivot). */
h2_status h2_factor(h2_handle h, void* stream);

/* x = A~^{-1} b through the parallel substitution (Eq. 31 and its transpose);
 * with ir_max_iter > 0 refined until max_col ||b - A~ x||/||b|| <= ir_tol
 * (H2_ERR_NOCONV if not reached).  b, x: device, n x nrhs, leading dimension
 * ld >= n, original point order (instances concatenated); b == x allowed.
 * H2_ERR_STATE before a successful h2_factor. */
h2_status h2_solve(h2_handle h, const double* b, double* x, int64_t nrhs,
                   int64_t ld, void* stream);

/* y = A~ x, the FP64 H^2 operator (upward pass, couplings, downward pass,
 * dense near field).  x, y: device, n x nrhs, ld >= n, original order; x != y. */
h2_status h2_matvec(h2_handle h, const double* x, double* y, int64_t nrhs,
                    int64_t ld, void* stream);

/* h2_solve for callers that cannot allocate device memory during the call
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, same kernels and results as h2_solve (with
 * the handle's params.timing ignored), but no hipMalloc, hipFree or other
 * allocating call: the gather partial products go to a fixed device array of
 * H2_NOALLOC_PARTIALS doubles (64 MiB), one per GPU, held until the process
 * ends; right-hand sides are processed in passes of
 * min(16, H2_NOALLOC_PARTIALS / h2_stats.gather_partials) columns.  The
 * handle's own buffers come from its build.  Every call on one GPU shares that
 * GPU's array, so calls that overlap on one GPU (other streams, other
 * threads, other handles) race and must be serialized by the caller.
 * Errors: as h2_solve, plus H2_ERR_UNSUPPORTED when one right-hand side
 * needs more than H2_NOALLOC_PARTIALS doubles of partials (the handle is
 * unchanged), and H2_ERR_HIP if the array's device address cannot be
 * looked up. */
h2_status h2_solve_noalloc(h2_handle h, const double* b, double* x, int64_t nrhs,
                           int64_t ld, void* stream);

h2_status h2_stats(h2_handle h, h2_stats_t* out);

/* Structure export (host buffers, sizes from h2_stats / h2_get_counts).
 *  perm:   n int64, the original index of each tree position (instances
 *          concatenated, each instance's indices local to it).
 *  ranks:  n_boxes int32, levels L..1 level-major, box-minor (instance-major
 *          within a level when batched: instance t's boxes in order).
 *  ms:     n_boxes int32, active sizes m in the same order.
 *  skel:   sum(ranks) int64, skeleton point ids (instance-local) per box.   */
h2_status h2_get_counts(h2_handle h, int64_t* n_boxes, int64_t* n_skel);
h2_status h2_get_structure(h2_handle h, int64_t* perm, int32_t* ranks,
                           int32_t* ms, int64_t* skel);
/* Near / far pairs of one level of instance 0 (ordered pairs, both orders):
 * pairs is 2*count int32; pass NULL to query count only. */
h2_status h2_get_pairs(h2_handle h, int32_t level, int32_t far, int32_t* pairs,
                       int64_t* count);
/* The two-sided basis P_i = [Q_i^S | Q_i^R L(r)_ii^{-1}^T] of box `box` at
 * tree level `level` (1..L) of instance `inst`, after h2_factor: m x m
 * column-major into host `p` (pass NULL to query m and k only).  Q_i is the
 * orthogonal completion of D_i U_i (Section 4.4, Eq. 32), so the last m - k
 * columns are V_i = Q_i^R L(r)_ii^{-T} of Algorithm 4.  H2_ERR_STATE before
 * a successful h2_factor.  LU variant: the left basis P_i (the right one,
 * [Q_i^S | Q_i^R U(r)_ii^{-1}], is not exported). */
h2_status h2_get_basis(h2_handle h, int32_t inst, int32_t level, int32_t box, double* p,
                       int32_t* m, int32_t* k);
/* The root matrix after factor: A_00 (before Cholesky) of instance t, n0 x n0
 * column-major into host `a` (n0 from h2_stats.root_n for t == 0). */
h2_status h2_get_root(h2_handle h, int32_t inst, double* a, int64_t* n0);

/* Rank-predictor MLP 8 -> 64 -> 64 -> 1 (ReLU), FP32, hand-written kernels.
 * Weights: 4801 floats W1(64x8) b1 W2(64x64) b2 W3(1x64) b3, row-major.
 * All pointers device.  Not part of the paper: sizes buffers before
 * compression; pivoted QR remains the fallback. */
h2_status h2_mlp_forward(const float* w, const float* x, float* y, int64_t n,
                         void* stream);
/* One full-batch Adam step on mean((y - t)^2): updates w, m, v in place,
 * writes the loss to *loss (device, 1 float) and the gradient to g (4801). */
h2_status h2_mlp_train_step(float* w, float* m, float* v, float* g,
                            const float* x, const float* t, int64_t n,
                            int32_t step, float lr, float* loss, void* stream);
/* Box features (8 per box, levels L..1 order as ranks) of a built handle. */
h2_status h2_box_features(h2_handle h, float* feats /* device, n_boxes x 8 */,
                          void* stream);

void h2_destroy(h2_handle h);
const char* h2_status_str(h2_status s);

#ifdef __cplusplus
}
#endif
#endif /* H2_H */
