/* Randomized generalized SVD of a matrix pair on one AMD Instinct MI355X
 * (gfx950).  C ABI: plain pointers and sizes, no framework types.
 *
 * Method (arXiv 2404.09459, "Fast randomized algorithms for low-rank matrix
 * approximations with applications in global comparative analysis of a class
 * of data sets"):
 *   - reduced GSVD G1 = U diag(alpha) R, G2 = V diag(beta) R with
 *     alpha^2 + beta^2 = 1, alpha descending ........ Sec. 1, eqs. (gsvd1), (ab)
 *   - randomized basis extraction Q_i of G_i ........ Sec. 2, Algorithm 1
 *     (fixed sketch of k + p columns as in Sec. 3, Theorem "projector";
 *      adaptive blocks of b columns with the cumulative residual test)
 *   - compressed pair Q_i^T G_i, stacked factorisation, SVD of L1, beta,
 *     recovery of U, V, R ............................. Sec. 2, Algorithm 2 and
 *                                                      the recovery after it
 *   - antisymmetric angular distance theta, generalized fractions of
 *     eigenexpression P1, P2, generalized normalized Shannon entropy
 *     D1, D2 ........................................... Sec. 1, the three
 *                                                      defining equations
 * Additions beyond the paper: q subspace (power) iterations
 * W = orth(G^T Q), Q = orth(G W) after the sketch; CholeskyQR2
 * orthonormalisation with FP64 Gram and Cholesky; mixed precision (BF16
 * MFMA for the sketch and early power iterations, FP32 for the last power
 * iteration and the projection, FP64 for the small steps).
 *
 * Truncation: when l1 + l2 < n the stacked factorisation of Algorithm 2 has
 * orthonormal rows and every alpha would be 1; the library keeps the dominant
 * rank-t joint row space of [Q1^T G1; Q2^T G2] (t = k) and applies
 * Algorithm 2's CS step to it.  In RGSVD_FULL mode t = n (needs l1 + l2 >= n)
 * and the result is Algorithm 2's.
 *
 * Gaussian test matrix: Philox4x32-10 (Salmon et al., SC'11) + Box-Muller,
 * key = (seed mod 2^32, seed >> 32), counter = (row, column >> 2, stream, 0),
 * words (x0,x1) -> columns 4j,4j+1 and (x2,x3) -> 4j+2,4j+3,
 * u1 = (xa+1) 2^-32, u2 = xb 2^-32, z = sqrt(-2 ln u1) (cos, sin)(2 pi u2);
 * stream 1 for G1, 2 for G2.
 *
 * Errors: every entry point returns RGSVD_OK (0) or a negative code for
 * problems detected on the host before anything is enqueued; nothing is
 * enqueued on error.  Numerical conditions found on the device are written
 * to the info array (read it after synchronising the stream).  No C++
 * exception crosses this interface.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default
 * stream).  Runs are asynchronous: calls only enqueue work.
 */
#ifndef RGSVD_H
#define RGSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------- codes ---- */
#define RGSVD_OK 0
#define RGSVD_EINVAL (-1)      /* bad argument (null, sizes, k + p > min(m, n), ld < n) */
#define RGSVD_ENOTGMP (-2)     /* full mode requested with l1 + l2 < n               */
#define RGSVD_EHIP (-3)        /* a HIP runtime call failed                          */
#define RGSVD_ENOMEM (-4)      /* host allocation failed                             */
#define RGSVD_EWORKSPACE (-5)  /* workspace null or misaligned (needs 256-byte base) */
#define RGSVD_ENOMODEL (-6)    /* learned sizing requested without a sizing model    */
#define RGSVD_EUNSUPPORTED (-7)/* combination not provided by this build             */
#define RGSVD_ETOOBIG (-8)     /* workspace exceeds RGSVD_STATIC_SCRATCH_BYTES        */

/* storage type of G */
#define RGSVD_F64 0
#define RGSVD_F32 1
/* arithmetic of the basis extraction */
#define RGSVD_PREC_FP64 0      /* every product in FP64 (FP64 MFMA)                  */
#define RGSVD_PREC_FP32 1      /* FP32 MFMA products, FP64 Gram/Cholesky/small step  */
#define RGSVD_PREC_MIXED 2     /* BF16 MFMA sketch + early power iterations, FP32
                                  last power iteration and projection, FP64 small   */
/* sketch sizing */
#define RGSVD_SIZE_FIXED 0     /* l = k + oversample columns, q power iterations      */
#define RGSVD_SIZE_ADAPTIVE 1  /* Algorithm 1: blocks of `block` columns until the
                                  cumulative residual ||(I-QQ^T)G||_F < tol           */
#define RGSVD_SIZE_LEARNED 2   /* sizing network picks l and q from a 16-column probe */
/* truncation */
#define RGSVD_TRUNCATED 0      /* t = k GSV pairs                                      */
#define RGSVD_FULL 1           /* t = n, needs l1 + l2 >= n (fixed or adaptive sizing;
                                  adaptive runs return RGSVD_ENOTGMP from rgsvd_run
                                  when the widths they reach fall short)              */

/* options: how the block Jacobi of the small step is launched.  By default
 * its first sweeps take one launch per round and its last three sweeps (most
 * often converged or nearly) one launch each, with a barrier between rounds,
 * when all workgroups of a sweep fit on the device at once (else per round).
 * Every choice turns the same pairs in the same order: same results.  The
 * barrier's wait is bounded (about a second): if other work sharing the
 * device keeps a sweep's workgroups from running together that long, the
 * Jacobi ends there and the pair carries the sweep-limit flag; callers that
 * share the device with long kernels can set RGSVD_OPT_JACOBI_ROUNDS. */
#define RGSVD_OPT_JACOBI_ROUNDS 0x1 /* every sweep one launch per round                */
#define RGSVD_OPT_JACOBI_SWEEPS 0x2 /* every sweep one launch, when it fits             */
#define RGSVD_OPT_JACOBI_NOWAIT 0x4 /* for tests of the failure path: the barrier of a
                                       one-launch sweep gives up at its first poll; the
                                       Jacobi ends there and the pair carries the
                                       sweep-limit flag (RGSVD_FLAG_JACOBI_M / _L1)    */

/* info words (int32, device), filled by a run */
#define RGSVD_INFO_STATUS 0
#define RGSVD_INFO_L1 1
#define RGSVD_INFO_L2 2
#define RGSVD_INFO_Q 3
#define RGSVD_INFO_FLAGS 4
#define RGSVD_INFO_SWEEPS_M 5
#define RGSVD_INFO_SWEEPS_L1 6
#define RGSVD_INFO_WORDS 8
/* flag bits of info[RGSVD_INFO_FLAGS] */
#define RGSVD_FLAG_SHIFT_Y 0x1     /* CholeskyQR of an m-side basis needed a shift    */
#define RGSVD_FLAG_SHIFT_W 0x2     /* CholeskyQR of an n-side basis needed a shift    */
#define RGSVD_FLAG_CHOL_FAIL 0x4   /* Cholesky failed even shifted (zero basis)       */
#define RGSVD_FLAG_JACOBI_M 0x8    /* eigen-solver hit its sweep limit                */
#define RGSVD_FLAG_JACOBI_L1 0x10  /* SVD of L1 hit its sweep limit                   */
#define RGSVD_FLAG_BETA_ZERO 0x20  /* some beta < 1e-14: that V column is set to zero */
#define RGSVD_FLAG_ALPHA_ZERO 0x40 /* sum of alpha^2 is zero                          */
#define RGSVD_FLAG_NONFINITE 0x80  /* non-finite values reached a Gram matrix         */
#define RGSVD_FLAG_FALLBACK 0x100  /* learned sizing: the residual judge rejected the
                                      network's sketch and Algorithm 1 ran instead    */

typedef struct rgsvd_plan_s* rgsvd_plan_t;

/* Problem and method parameters.  Sizes are int64; G_i are row-major with
 * leading dimension >= n. */
typedef struct {
  int64_t m, p, n;          /* G1 is m x n, G2 is p x n                               */
  int64_t k;                /* target rank: number t of GSV pairs (truncated mode)    */
  int64_t oversample;       /* p of Theorem "projector"; l_i = k + oversample         */
  int32_t power_iters;      /* q subspace iterations                                   */
  int32_t in_dtype;         /* RGSVD_F64 | RGSVD_F32                                  */
  int32_t precision;        /* RGSVD_PREC_*                                           */
  int32_t sizing;           /* RGSVD_SIZE_*                                           */
  int32_t mode;             /* RGSVD_TRUNCATED | RGSVD_FULL                            */
  int32_t options;          /* RGSVD_OPT_* bits (0: defaults)                           */
  uint64_t seed;            /* Omega seed                                              */
  double tol;               /* adaptive: eps of Algorithm 1 (absolute Frobenius);
                               learned: the judge's eps (0: no judge)                   */
  int64_t block;            /* adaptive, learned fallback: b of Algorithm 1 (0 -> 100) */
  int64_t lmax;             /* adaptive/learned: cap on l_i (0 -> min(m_i, n, 224))    */
} rgsvd_desc;

/* Caller-owned device outputs.  alpha, beta, theta, P1, P2 have t entries,
 * D has 2 (D1, D2), sigma_B has l1 + l2 entries: the t dominant singular
 * values of the stacked compressed pair [Q1^T G1; Q2^T G2] in descending
 * order, then l1 + l2 - t values whose squares sum to the remaining
 * singular values' squares (they are not individually singular values).  U (m x t) and V (p x t) are column-major (column j of U
 * at U + j*ldu, ldu >= m), R (t x n) is row-major (ldr >= n); all FP64.
 * U, V, R, sigma_B may be NULL to skip them.  info: RGSVD_INFO_WORDS int32. */
typedef struct {
  double *alpha, *beta, *theta, *P1, *P2, *D, *sigma_B;
  double *U, *V, *R;
  int64_t ldu, ldv, ldr;
  int32_t* info;
} rgsvd_out;

/* Validate `desc`, build a plan and report the device workspace it needs
 * (bytes, 256-byte aligned base required).  The plan holds only host
 * metadata; destroy it with rgsvd_destroy.  Errors: RGSVD_EINVAL,
 * RGSVD_ENOTGMP, RGSVD_EUNSUPPORTED, RGSVD_ENOMEM. */
int rgsvd_plan(const rgsvd_desc* desc, rgsvd_plan_t* plan, size_t* workspace_bytes);

/* Enqueue one randomized GSVD of (G1, G2) on `stream`.  G1, G2: device
 * pointers of the storage type in the plan, row-major with leading
 * dimensions ld1, ld2 >= n (elements).  workspace: device buffer of the
 * size rgsvd_plan reported, owned by the caller, not used concurrently by
 * another run.  The plan must not be used by two streams at once.
 *
 * Fixed sizing only enqueues.  Adaptive sizing (Sec. 2, Algorithm 1) runs
 * block by block: Omega columns [l, l + block) of each matrix's stream, the
 * block projected against the basis so far and orthonormalised, the new rows
 * of B = Q^T G and their energy; the residual ||G||_F^2 - sum ||B_j||_F^2
 * is compared with tol^2 on the host, so the call synchronises `stream`
 * once after the norms of G and once per block (FP64 precision, truncated
 * mode; blocks rows numerically inside the span of the basis become zero
 * basis vectors).  Learned sizing sketches at the widest width the network
 * can pick (min(2k, capacity)); the first 16 columns of that sketch are the
 * probe (Omega's columns are global, so they are the 16-column sketch), its
 * features go through the attached network, and the call synchronises once
 * to read the choice of l (one of k+4, k+8, k+16, k+32, 2k, capped) and q
 * (0..3); the run then continues on the sketch's first l columns.  The job
 * tables of every grid point are built and uploaded once per binding of
 * pointers.  With tol > 0 a residual judge follows: if
 * ||G_i||_F^2 - ||Q_i^T G_i||_F^2 > tol^2 for either matrix, the pair is
 * redone by Algorithm 1 (FP64, blocks of `block` columns, tolerance tol;
 * the plan's buffers are laid out for it) and RGSVD_FLAG_FALLBACK is set;
 * the judge synchronises once more.  For adaptive and learned sizing
 * info[1], info[2], info[3] report the l1, l2, q used and sigma_B needs
 * room for the capacities l1 + l2 of rgsvd_plan_sizes.
 * Errors: RGSVD_EINVAL, RGSVD_EWORKSPACE, RGSVD_ENOMODEL, RGSVD_EHIP. */
int rgsvd_run(rgsvd_plan_t plan, const void* G1, int64_t ld1, const void* G2, int64_t ld2,
              void* workspace, void* stream, const rgsvd_out* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * run as rgsvd_run, without a workspace argument.  Its workspace is a
 * device array of RGSVD_STATIC_SCRATCH_BYTES (64 MiB) built into the library,
 * one per GPU, held until the process ends.  The call allocates nothing:
 * no hipMalloc, hipFree or pinned host memory (the plan's job tables are
 * copied into that array with hipMemcpyAsync from the plan's host memory).
 * Every static run on a GPU shares that GPU's array and leaves its contents
 * behind; each run clears what it needs.  Static runs that overlap on one
 * GPU (two streams, two threads) race on the array: serialise them.
 * Fixed sizing only.  Errors: RGSVD_EINVAL, RGSVD_EUNSUPPORTED (adaptive or
 * learned plans), RGSVD_ETOOBIG (the plan's workspace, as reported by
 * rgsvd_plan, is above RGSVD_STATIC_SCRATCH_BYTES), RGSVD_EHIP. */
#define RGSVD_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int rgsvd_run_static(rgsvd_plan_t plan, const void* G1, int64_t ld1, const void* G2, int64_t ld2,
                     void* stream, const rgsvd_out* out);

/* t (number of returned pairs) and l1, l2: the sketch widths of fixed
 * sizing, the largest widths (capacities) of adaptive and learned sizing. */
int rgsvd_plan_sizes(rgsvd_plan_t plan, int64_t* t, int64_t* l1, int64_t* l2);

void rgsvd_destroy(rgsvd_plan_t plan);
const char* rgsvd_strerror(int code);

/* Per-stage timing of single-pair runs with HIP events recorded on the run's
 * stream between its launches (enable = 1 before rgsvd_run).  After the
 * stream is synchronised, rgsvd_profile_read returns the stage count and, for
 * up to `max` stages, the elapsed milliseconds and a stage tag:
 *   0 zero fill, 1 info init, 2 Omega generation, 3 G W product,
 *   4 split G^T Q / Q^T G product, 5 partial-sum reduction, 6 Gram (CholeskyQR),
 *   7 Cholesky + inverse, 8 triangular update Q = Y R^{-1}, 9 small FP64 step,
 *   10 recovery products, 11 sign convention, 12 Gram of the compressed pair,
 *   13 block Jacobi sweep (start or round) on a factor of the small step. */
int rgsvd_profile(rgsvd_plan_t plan, int32_t enable);
int rgsvd_profile_read(rgsvd_plan_t plan, int32_t max, float* ms, int32_t* tag, int32_t* count);

/* ------------------------------------------------------ batched runs ---- */
/* Many independent pairs of different sizes in one sequence of grouped
 * launches (one launch per step serves every pair), captured once into a
 * HIP graph and replayed.  Shapes are fixed at plan time; fixed sizing only.
 * shapes: host array of npairs descriptors (m, p, n, k, oversample, seed
 * are read per pair).  in_dtype, precision and mode must agree across the
 * batch (else RGSVD_EINVAL); power_iters must agree too and sizing must be
 * RGSVD_SIZE_FIXED (else RGSVD_EUNSUPPORTED), because each grouped launch
 * serves every pair at the same step of the subspace iteration. */
typedef struct {
  const void* G1; const void* G2; int64_t ld1, ld2;
  rgsvd_out out;
} rgsvd_pair_io;

int rgsvd_batch_plan(const rgsvd_desc* shapes, int32_t npairs, rgsvd_plan_t* plan,
                     size_t* workspace_bytes);
/* Bind device pointers (host array of npairs entries) and the workspace;
 * builds and uploads the job tables and captures the graph on `stream`. */
int rgsvd_batch_bind(rgsvd_plan_t plan, const rgsvd_pair_io* io, void* workspace, void* stream);
/* Replay the bound batch on `stream` (graph launch). */
int rgsvd_batch_run(rgsvd_plan_t plan, void* stream);

/* ---------------------------------------------------------- autotuner --- */
/* Tile shapes of the streaming kernels chosen by measurement on the caller's
 * data:
 * rows per tile of the G W kernel (1 or 4), columns per lane of the G^T Q
 * kernel (2 or 4), the number of row chunks of its split reduction (the
 * heuristic count, half, twice) and, on the mixed path over FP32 storage,
 * the kernels themselves (1: 8-wave workgroups sharing W or Q^T through LDS,
 * whose tile shapes are fixed; 2: the per-wave kernels with the three
 * knobs).  Each valid combination is enqueued
 * reps + 1 times on `stream` (outputs are written, one warm-up) and timed
 * with HIP events; the fastest is kept in the plan and in a per-process cache
 * keyed by the plan's shapes, storage type and precision, which later plans
 * of the same key start from.  choice (4 int32, may be NULL): rt, js, chunk
 * index (0 heuristic, 1 half, 2 twice), kernel family (0 where there is
 * no choice); best_ms (may be NULL): mean run time
 * of the choice.  Synchronises `stream`.  Fixed-size plans only.
 * rgsvd_batch_autotune takes the batch's pointers like rgsvd_batch_bind and
 * must be followed by rgsvd_batch_bind (which captures with the choice). */
int rgsvd_autotune(rgsvd_plan_t plan, const void* G1, int64_t ld1, const void* G2, int64_t ld2,
                   void* workspace, void* stream, const rgsvd_out* out, int32_t reps, int32_t* choice,
                   float* best_ms);
int rgsvd_batch_autotune(rgsvd_plan_t plan, const rgsvd_pair_io* io, void* workspace, void* stream,
                         int32_t reps, int32_t* choice, float* best_ms);

/* ---------------------------------------------------- sizing network ---- */
/* 32-64-64-2 ReLU MLP in FP32.  Parameter layout: W1 (64x32), b1 (64),
 * W2 (64x64), b2 (64), W3 (2x64), b3 (2), row-major W[out][in],
 * concatenated (RGSVD_MLP_PARAMS floats).  Features (32, G1's 16 then
 * G2's, each a log10 ratio floored at -8): log10(s_j / s_1) for
 * j = 2, 4, ..., 16 of the singular values of the probe sketch
 * G Omega[:, :16], then log10(rho_j / rho_1) at the columns ceil(k/4),
 * ceil(k/2), ceil(3k/4), k, k+4, k+8, k+16 and L (clamped to [1, L]) of the
 * sketch G Omega[:, :L] at the widest grid width L, rho_j the j-th diagonal
 * entry of its CholeskyQR factor R.  Outputs: regression targets
 * (log2(l / k), q) of the sketch width l and the power count q. */
#define RGSVD_MLP_PARAMS 6402
#define RGSVD_MLP_IN 32
#define RGSVD_MLP_OUT 2

/* Y[b][0..1] = MLP(X[b][0..31]) for b < batch.  act: device scratch of
 * batch * 128 floats that keeps the hidden activations for the backward
 * pass (may be NULL for inference only). */
int rgsvd_mlp_forward(const float* params, const float* X, int32_t batch, float* Y, float* act,
                      void* stream);
/* Gradient of 0.5 * sum (Y - T)^2 / batch w.r.t. the packed parameters
 * (written to grad, RGSVD_MLP_PARAMS floats) from the forward's act; loss
 * (one float, device) may be NULL. */
int rgsvd_mlp_backward(const float* params, const float* X, const float* T, int32_t batch,
                       const float* act, float* grad, float* loss, void* stream);
/* One Adam step (Kingma & Ba): m, v moment buffers, step counts from 1. */
int rgsvd_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                   float beta1, float beta2, float eps, void* stream);
/* Attach a trained sizing network (device params, copied into the plan's
 * own device buffer on `stream`). */
int rgsvd_set_sizing_model(rgsvd_plan_t plan, const float* params, void* stream);
/* Probe features of a pair for the sizing network (enqueued on `stream`):
 * the 32 features above (the floor at -8 is what an FP64 Gram of a sketch
 * resolves), into feat (device, 32 floats).  Runs the head of a learned
 * run: the sketch at the widest grid width L of the plan's k and capacity,
 * in the plan's own sketch arithmetic (BF16 for mixed plans), its first 16
 * columns as the probe, and the first CholeskyQR pass over all L columns
 * for the profile, so a learned plan of the same shapes, precision, k and
 * seed gets the same numbers in its own runs.  Uses the plan's shapes,
 * storage type and seed and its workspace (any sizing mode; single-pair
 * plans); the grid width follows the plan's capacity, so features for a
 * learned plan are taken with a learned plan. */
int rgsvd_probe_features(rgsvd_plan_t plan, const void* G1, int64_t ld1, const void* G2, int64_t ld2,
                         void* workspace, float* feat, void* stream);

/* ----------------------------------------------------------- checks ---- */
/* Omega[r][col0 + c] (r < rows, c < ncols) into out (row-major, ld >= ncols),
 * FP64 (dtype 0) or FP32 (dtype 1) Box-Muller; the generator spec above. */
int rgsvd_gaussian(uint64_t seed, uint32_t stream_id, int64_t rows, int64_t col0, int64_t ncols,
                   int32_t dtype, void* out, int64_t ld, void* stream);
/* The raw Philox words feeding Omega[r][col0 + c], uint32, row-major. */
int rgsvd_philox_words(uint64_t seed, uint32_t stream_id, int64_t rows, int64_t col0,
                       int64_t ncols, uint32_t* out, int64_t ld, void* stream);
/* Lane-layout self-test of the 16x16 MFMA forms the kernels use: computes
 * D = A B for one 16 x K tile (which = 0: fp64 K=4, 1: fp32 K=4, 2: bf16 K=32)
 * from row-major A (16 x K) and B (K x 16) into D (16 x 16, row-major,
 * fp32 or fp64 as the form accumulates). */
int rgsvd_selftest_mfma(int32_t which, const void* A, const void* B, void* D, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RGSVD_H */
