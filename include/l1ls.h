/*
 * l1ls.h -- C ABI of the MI355X (gfx950) solver for the complex L1-regularised
 * least-squares problem (basis pursuit denoising) used for super-resolving
 * tomographic SAR in Shi, Zhu, Yin, Bamler, arXiv 1805.01759.
 *
 * Per pixel p the library solves Eq. (1) = Eq. (6) of the paper (no factor 1/2):
 *     min_x  ||A x - b_p||_2^2 + lambda_p ||x||_1 ,   x in C^L,
 * where A (N x L) is the irregular Fourier matrix of the TomoSAR imaging model,
 * Eq. (5): A[n, l] = exp(-j 2 pi xi_n s_l), xi_n = 2 b_n / (lambda_w r).
 * The solver is Algorithm 1 of the paper (RBPG with backtracking) with a
 * single block (J = 1): Nesterov extrapolation Eqs. (11)-(12), complex soft
 * thresholding Eq. (10), the backtracking condition Eq. (15) and the monotone
 * acceptance test of the algorithm, followed by an optional FP64 refinement on
 * the support and an FP64 check of the optimality conditions.
 *
 * Conventions shared by every entry point
 *  - Complex values are l1ls_c32 (interleaved float re, im; the layout of
 *    torch.complex64 / numpy.complex64).
 *  - A is row-major: A[n * L + l].  B is pixel-major: B[p * N + n].
 *    X is pixel-major: X[p * L + l].
 *  - Every pointer named "device" is a HIP device pointer; the caller owns the
 *    memory.  The solve, plan-execute and unrolled entry points allocate no
 *    device memory: scratch lives in the caller's workspace (l1ls_solve_noalloc:
 *    in a fixed array of the library).  l1ls_plan_create allocates temporary
 *    buffers while it times candidate kernels.  Work is queued on the given
 *    stream and nothing synchronises the host.
 *  - Argument errors are detected on the host before any launch: the call
 *    returns a negative l1ls_status and l1ls_last_error() describes it.
 *  - Numerical outcomes are not errors: per-pixel results are reported in
 *    l1ls_diag.status and the call returns L1LS_OK.
 *  - Supported sizes: 1 <= N <= 128, 1 <= L <= 4096, 0 <= P < 2^31 (the
 *    wave-per-pixel kernel and the block form take up to 1,024 bins: above
 *    that, WAVE is refused and l1ls_solve_blocks refuses blocks of more than
 *    1,024 columns; the FP64 continuation keeps a pixel's vectors in the
 *    workspace there, 96 KB a workgroup per 1,024 bins, and is much slower).
 */
#ifndef L1LS_H
#define L1LS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } l1ls_c32;

typedef enum {
    L1LS_OK = 0,
    L1LS_ERR_INVALID_ARG = -1,
    L1LS_ERR_UNSUPPORTED_SHAPE = -2,
    L1LS_ERR_WORKSPACE = -3,
    L1LS_ERR_HIP = -4,
    L1LS_ERR_INTERNAL = -5
} l1ls_status;

/* Arithmetic of the two contractions A x and A^H r (the gradient of Eq. (9)).
 * L1LS_FP32: FP32 MFMA.  L1LS_SPLIT_BF16: every operand split into hi + lo
 * bfloat16 parts, three MFMA passes (hi*hi + hi*lo + lo*hi) with FP32
 * accumulation.  Everything else (prox, step, reductions) is FP32; the
 * refinement and the final optimality check are FP64.  Split-BF16 runs on the
 * MFMA tiles (the register-resident tile and the streamed tile, which takes every
 * supported shape); the wave-per-pixel kernel (iteration_kernel WAVE) and the
 * block form take L1LS_FP32 only and refuse L1LS_SPLIT_BF16
 * (L1LS_ERR_UNSUPPORTED_SHAPE, also from l1ls_workspace_size and
 * l1ls_plan_create). */
typedef enum { L1LS_FP32 = 0, L1LS_SPLIT_BF16 = 1 } l1ls_precision;

/* The kernel that runs the iterations of Algorithm 1 (l1ls_options.iteration_kernel).
 *  AUTO    the streamed MFMA tile, except for n <= 64 and l <= 384, which run
 *          the register-resident tile; l1ls_plan_create times the candidates
 *          instead, and l1ls_solve_noalloc takes the register tile where the
 *          streamed tile's state would not fit its scratch
 *  MFMA    the register-resident MFMA tile (n <= 64, l <= 512)
 *  WAVE    the wave-per-pixel kernel (plain FP32 vector arithmetic; FP32 only)
 *  STREAM  the streamed MFMA tile: the same contractions as the register tile
 *          (FP32 or split-BF16), with each 16-pixel tile's iterates and
 *          gradients (two x and three G arrays) kept in the workspace (l_pad x
 *          640 bytes a persistent workgroup, at most 512 of them); any
 *          supported shape
 * A kernel that does not take the shape or precision is refused with
 * L1LS_ERR_UNSUPPORTED_SHAPE.  The three agree to FP32 rounding; the register
 * and streamed tiles give bit-identical results for 384 < l <= 512, in either
 * precision. */
typedef enum {
    L1LS_ITER_AUTO = 0,
    L1LS_ITER_MFMA = 1,
    L1LS_ITER_WAVE = 2,
    L1LS_ITER_STREAM = 3
} l1ls_iteration_kernel;

/* Per-pixel status bits (diag.status). */
enum {
    L1LS_PX_CONVERGED = 1,   /* FP64 KKT residual <= tol at the returned x        */
    L1LS_PX_MAX_ITER = 2,    /* iteration budget spent before the FP32 test passed */
    L1LS_PX_NONFINITE = 4,   /* NaN/Inf met in the data or the iteration           */
    L1LS_PX_POLISHED = 8,    /* FP64 refinement on the support was applied         */
    L1LS_PX_ZERO = 16,       /* returned x is exactly 0                            */
    L1LS_PX_BAD_LAMBDA = 32  /* lambda_p <= 0 or not finite: x = 0 returned        */
};

typedef struct {
    int32_t max_iter;      /* cap on iterations of Algorithm 1 (N_K); >= 0, default 500      */
    float tol;             /* KKT residual target (> 0), default 1e-4                          */
    float c_alpha;         /* backtracking factor C_alpha of Eq. (15), in (0,1); default 0.5   */
    int32_t precision;     /* l1ls_precision, default L1LS_FP32                                */
    int32_t backtracking;  /* 1: Eq. (15) line search; 0: fixed step 1/L_f                     */
    int32_t monotone;      /* 1: accept x-bar only if F(x-bar) <= F(x^k) (Algorithm 1)         */
    int32_t fp64_polish;   /* FP64 active-set Newton refinement: 0 off; 1 pixels whose FP64
                              KKT residual exceeds tol; 2 every pixel (to FP64 precision).
                              Working sets of up to 8 complex unknowns, then passes with up
                              to 16 and 32 for pixels that filled the previous one; a pixel
                              whose minimiser has more nonzeros is returned unsolved (status
                              bits)                                                          */
    int32_t polish_after;  /* hand a pixel to the refinement after this many iterations
                              (<= max_iter; <= 0 means max_iter)                              */
    int32_t warm_start;    /* 0: Algorithm 1 starts at x^(0) = 0; 1: X holds each pixel's
                              initial point x^(0) on entry (the Init of Algorithm 1; x^(1) =
                              x^(0), the step starts at alpha_0).  Not available in
                              l1ls_solve_blocks (L1LS_ERR_UNSUPPORTED_SHAPE)                 */
    int32_t fp64_continue; /* 1: a pixel the refinement leaves above tol (its minimiser has more
                              nonzeros than the 32-slot working set holds, or the active-set
                              walk stalls) continues Algorithm 1 in FP64 from the best point
                              found, until KKT <= tol or max_iter iterations in all (FP32 and
                              FP64 counted together); needs fp64_polish.  Default 1; 0: such a
                              pixel is returned unsolved                                     */
    int32_t iteration_kernel; /* l1ls_iteration_kernel, default L1LS_ITER_AUTO; the workspace
                              size depends on it (the streamed tile's state)                  */
} l1ls_options;

/* Device arrays of length P; any may be NULL.
 *  iters      iterations of Algorithm 1 performed
 *  kkt        KKT residual of the returned x, evaluated in FP64:
 *             KKT(x) = L_f max_l |x_l - S_{lambda/L_f}(x_l - g_l/L_f)| / lambda,
 *             g = 2 A^H (A x - b), L_f = 2 lambda_max(A A^H)
 *  objective  F(x) = ||Ax - b||^2 + lambda ||x||_1 (FP64-evaluated, stored FP32)
 *  status     L1LS_PX_* bits
 *  nnz        number of nonzero entries of x */
typedef struct {
    int32_t *iters;
    float *kkt;
    float *objective;
    uint32_t *status;
    int32_t *nnz;
} l1ls_diag;

/* Defaults: max_iter 500, tol 1e-4, c_alpha 0.5, FP32, backtracking, monotone,
 * FP64 polish after max_iter. */
l1ls_options l1ls_options_default(void);

/* Bytes of device workspace l1ls_solve needs for these sizes and options. */
l1ls_status l1ls_workspace_size(int32_t n, int32_t l, int64_t p, const l1ls_options *opt,
                                size_t *bytes);

/* Solve Eq. (1) for every pixel of one stack.
 *  A        device, n*l, row-major, shared by all pixels
 *  B        device, p*n, pixel-major measurement vectors g_p of Eq. (5)
 *  lambda   device float; lambda_stride 0 = one value for all pixels, else
 *           lambda[p * lambda_stride]
 *  X        device, p*l: output (the pixel's x); with opt->warm_start also the
 *           input (each pixel's initial point), overwritten by the result
 *  diag     host struct of device pointers (may be NULL)
 *  workspace/ws_bytes  device scratch of at least l1ls_workspace_size bytes,
 *           16-byte aligned; its contents on entry are ignored
 * Returns L1LS_OK, or a negative status with no work queued.  p = 0 is a no-op. */
l1ls_status l1ls_solve(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B,
                       const float *lambda, int64_t lambda_stride, const l1ls_options *opt,
                       l1ls_c32 *X, const l1ls_diag *diag, void *workspace, size_t ws_bytes,
                       hipStream_t stream);

/* l1ls_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as l1ls_solve, with the workspace taken from a
 * fixed array of L1LS_NOALLOC_SCRATCH_BYTES in the library's code object, one
 * per device, held until the process ends (its address is looked up on the
 * first call on each device; that lookup is the only set-up).  The caller
 * passes inputs and outputs as for l1ls_solve; no hipMalloc, hipFree or event
 * is created.  The stream must belong to the current device.
 *  - returns L1LS_ERR_WORKSPACE, with no work queued, when l1ls_workspace_size
 *    for (n, l, p) exceeds L1LS_NOALLOC_SCRATCH_BYTES (e.g. n = 25, l = 256
 *    holds about 220,000 pixels, n = 50, l = 512 about 68,000 on the register
 *    tile, which the automatic kernel choice takes here when the streamed
 *    tile's state would not fit); split the pixels or call l1ls_solve.
 *  - every call on one device shares that device's array, which keeps the last
 *    call's contents (the kernels clear what must start at zero): calls that
 *    overlap in time on one device race and give undefined results; serialise
 *    them (one stream, or events).
 *  - timing events (l1ls_timing_enable) are not recorded for these calls. */
#define L1LS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
l1ls_status l1ls_solve_noalloc(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B,
                               const float *lambda, int64_t lambda_stride, const l1ls_options *opt,
                               l1ls_c32 *X, const l1ls_diag *diag, hipStream_t stream);

/* Algorithm 1 with J column blocks (randomized block prox-gradient, Eqs. (13)-(14)).
 * Bins are split into J contiguous blocks of ceil(l/J); iteration k of a pixel
 * updates the block that draws[k-1] selects with P_i = L_i / sum_j L_j,
 * L_i = 2 lambda_max(A_i A_i^H) (the first i with draws[k-1] sum L < L_0 + ... + L_i).
 * Per block: its own update count for the extrapolation weight of Eqs. (11)-(12),
 * its own step for Eq. (15) (start 1/(2 max ||a_l||^2) over its columns, floor
 * 1/L_i), and the monotone test of Algorithm 1 on the objective with the block
 * replaced; the KKT residual is tested every J iterations.  J = 1 is Algorithm 1
 * with one block.  The FP64 refinement and certificate then run as in l1ls_solve
 * (the block products are FP32: precision L1LS_SPLIT_BF16 is refused).
 *  blocks   J, 1 <= J <= min(64, l); n <= 64
 *  draws    device double, at least min(max_iter, polish_after) values in [0, 1),
 *           shared by all pixels (pixel-local iteration k uses draws[k-1])
 *  other arguments as l1ls_solve (same workspace size); l1ls_solve_counters
 *  out[0] then holds the iteration's FP32 flops (8 per complex multiply-add)
 *  instead of a count of products, and out[1] is 0. */
l1ls_status l1ls_solve_blocks(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B,
                              const float *lambda, int64_t lambda_stride, const l1ls_options *opt,
                              int32_t blocks, const double *draws, l1ls_c32 *X, const l1ls_diag *diag,
                              void *workspace, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched stacks of uneven size (each with its own A, N, L and pixel count) in
 * one persistent launch per shape class.  The plan holds host tables and the
 * tile shape chosen for each stack; execute only launches kernels (no
 * allocation, no host synchronisation, no branching on device data), so it may
 * be captured into a HIP graph.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t n, l;
    int64_t p;
    const l1ls_c32 *A;       /* device */
    const l1ls_c32 *B;       /* device */
    const float *lambda;     /* device */
    int64_t lambda_stride;
    l1ls_c32 *X;             /* device */
    l1ls_diag diag;
} l1ls_stack;

typedef struct l1ls_plan l1ls_plan;

/* Build a plan from the shapes (n, l, p) of `stacks` (their pointers are not
 * read).  The options are copied into the plan. */
l1ls_status l1ls_plan_create(const l1ls_stack *stacks, int32_t count, const l1ls_options *opt,
                             l1ls_plan **out);
l1ls_status l1ls_plan_workspace_size(const l1ls_plan *plan, size_t *bytes);
/* `stacks` must have the shapes given at plan creation. */
l1ls_status l1ls_plan_execute(l1ls_plan *plan, const l1ls_stack *stacks, void *workspace,
                              size_t ws_bytes, hipStream_t stream);
void l1ls_plan_destroy(l1ls_plan *plan);
/* Describe the plan (tile class per stack) into buf; returns chars needed. */
int32_t l1ls_plan_describe(const l1ls_plan *plan, char *buf, int32_t buf_len);

/* ---------------------------------------------------------------------------
 * Unrolled fixed-step map and its adjoint (differentiation through K
 * iterations of Eqs. (11)-(12) with constant step alpha, no backtracking and no
 * monotone test).  A is built on the device from xi (N) and the elevation grid
 * s (L) as exp(-j 2 pi xi_n s_l).
 *
 * forward: X_K from x^0 = x^{-1} = 0.  tape (device, tape_bytes >=
 *   l1ls_unrolled_tape_size) receives checkpoints (x^k, x^{k-1}) every
 *   ckpt_every iterations for the backward pass.
 * backward: given dX = dloss/dX_K (complex, dRe + j dIm), writes
 *   dB (p*n complex), dlambda (1 float, device) and dxi (n floats, device).
 *   ws (device) >= l1ls_unrolled_backward_ws_size bytes.
 * ------------------------------------------------------------------------- */
l1ls_status l1ls_unrolled_tape_size(int32_t n, int32_t l, int64_t p, int32_t K,
                                    int32_t ckpt_every, size_t *bytes);
l1ls_status l1ls_unrolled_backward_ws_size(int32_t n, int32_t l, int64_t p, int32_t K,
                                           int32_t ckpt_every, size_t *bytes);
l1ls_status l1ls_unrolled_forward(int32_t n, int32_t l, int64_t p, const float *xi,
                                  const float *s, const l1ls_c32 *B, float lambda, float alpha,
                                  int32_t K, int32_t ckpt_every, l1ls_c32 *X_K, void *tape,
                                  size_t tape_bytes, hipStream_t stream);
l1ls_status l1ls_unrolled_backward(int32_t n, int32_t l, int64_t p, const float *xi,
                                   const float *s, const l1ls_c32 *B, float lambda, float alpha,
                                   int32_t K, int32_t ckpt_every, const void *tape,
                                   size_t tape_bytes, const l1ls_c32 *dX, l1ls_c32 *dB,
                                   float *dlambda, float *dxi, void *ws, size_t ws_bytes,
                                   hipStream_t stream);

/* Work counters of the last l1ls_solve that used `workspace` (synchronises
 * `stream`): out[0] pixel forward products A d, out[1] pixel adjoint products
 * A^H r (each 8 N L real flops), out[2] pixels handed to the FP64 refinement,
 * out[3] FP64 flops of the refinement's algorithm (full gradient passes
 * 8 N L each, working-set residuals and gradients 8 N |S|, Gram entries
 * 8 N, factorisations (2|S|)^3/3, substitutions 2 (2|S|)^2), out[4] the
 * refinement's FP32 flops (its round-end gradient over all L bins, 8 N L a
 * round, runs in FP32 under fp64_polish = 1), counted by the kernels as they
 * run.  `out` holds 5 entries. */
l1ls_status l1ls_solve_counters(int32_t n, int32_t l, int64_t p, const void *workspace,
                                hipStream_t stream, uint64_t out[5]);

/* Step constants of the last l1ls_solve or l1ls_solve_blocks with p > 0 that
 * used `workspace` (synchronises `stream`): out[0] L_f = 2 lambda_max(A A^H),
 * the Lipschitz constant of the gradient of ||Ax - b||^2 (Algorithm 1), found
 * by an FP64 power iteration on the N x N matrix A A^H and used as the step
 * floor 1/L_f of Eq. (15) and in the KKT residual; out[1] the initial step
 * alpha_0 = 1/(2 max_l ||a_l||^2) that Eq. (15)'s backtracking starts from;
 * out[2] the power iterations spent.  `out` holds 3 entries; a workspace that
 * no such solve has used holds no meaningful values. */
l1ls_status l1ls_solve_constants(int32_t n, int32_t l, int64_t p, const void *workspace,
                                 hipStream_t stream, double out[3]);

/* Name of a status code; detail of the last error on the calling thread. */
const char *l1ls_status_string(l1ls_status s);
const char *l1ls_last_error(void);

/* Kernel classes of a solve, for event timing. */
typedef enum {
    L1LS_KERNEL_ITERATION = 0, /* the accelerated proximal-gradient iteration */
    L1LS_KERNEL_REFINE = 1,    /* the FP64 refinement */
    L1LS_KERNEL_CERTIFY = 2    /* the FP64 KKT certificate */
} l1ls_kernel_class;

/* Event timing (opt-in, for measurement): while enabled, every kernel launch of
 * l1ls_solve is bracketed by HIP events on its stream.  l1ls_timing_read_kernel
 * returns the total milliseconds and the number of launches of one kernel
 * class since its last read (and resets that class); -1 for an unknown class.
 * l1ls_timing_read is the same for L1LS_KERNEL_ITERATION. */
void l1ls_timing_enable(int32_t on);
int32_t l1ls_timing_read(double *total_ms, int32_t *launches);
int32_t l1ls_timing_read_kernel(int32_t kernel_class, double *total_ms, int32_t *launches);

#ifdef __cplusplus
}
#endif
#endif
