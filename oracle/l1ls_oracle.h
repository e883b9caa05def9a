/*
 * l1ls_oracle.h -- plain FP64 CPU oracle for the complex L1-regularised least
 * squares problem (basis pursuit denoising) of Shi, Zhu, Yin and Bamler,
 * "A fast and accurate basis pursuit denoising algorithm with application to
 * super-resolving tomographic SAR" (arXiv 1805.01759).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU path under paper_1805_01759_amd/.
 *
 * Problem (Eq. (1) = Eq. (6), no factor 1/2 on the quadratic term):
 *     min_x  F(x) = ||A x - b||_2^2 + lambda ||x||_1,   x in C^L,
 * A in C^{N x L} row-major (A[n*L + l]), b in C^N, lambda > 0.
 * Batched data: B is P x N pixel-major, X is P x L pixel-major.
 * Complex values are C99 `double _Complex` (interleaved re, im), which is the
 * memory layout of numpy complex128.
 *
 * Every function is a direct transcription of a definition or of the steps of
 * Algorithm 1 (RBPG with backtracking) with one block (J = 1).  Where the
 * paper is silent the reading used is stated at the function.
 */
#ifndef L1LS_ORACLE_H
#define L1LS_ORACLE_H

#include <complex.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef double _Complex ocplx;

/* Lipschitz constant of grad f, f(x) = ||Ax - b||^2:  L_f = 2 lambda_max(A A^H).
 * Cyclic Jacobi on the real symmetric 2N x 2N embedding of A A^H (whose
 * spectrum is that of A A^H with every eigenvalue doubled in multiplicity). */
double orc_lipschitz(int n, int l, const ocplx *A);

/* Complex soft threshold  S_tau(v) = v * max(0, 1 - tau/|v|), elementwise;
 * |v| <= tau (ties included) maps to 0.  Eq. (10) in complex form. */
void orc_prox(int m, const ocplx *v, double tau, ocplx *out);

/* F(x) = ||Ax-b||^2 + lambda ||x||_1  (Eq. (1)). */
double orc_objective(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                     const ocplx *x);

/* Natural KKT residual (gradient-mapping form):
 *   KKT_nat(x) = L_f * max_l |x_l - S_{lambda/L_f}(x_l - g_l/L_f)_l| / lambda,
 * with g = 2 A^H (A x - b).  Zero iff x is a minimiser. */
double orc_kkt_nat(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                   double Lf, const ocplx *x);

/* Subgradient KKT residual:
 *   max_l { |g_l + lambda x_l/|x_l|| if x_l != 0 ;  max(0, |g_l| - lambda) if x_l = 0 } / lambda. */
double orc_kkt_sub(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                   const ocplx *x);

/* Duality gap F(x) - D(nu) with the dual point nu = s * 2(Ax - b),
 * s = min(1, lambda / max_l |2 a_l^H (Ax - b)|),
 * D(nu) = -||nu||^2/4 - Re(nu^H b)  (dual of Eq. (1), feasible for |a_l^H nu| <= lambda). */
double orc_dual_gap(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                    const ocplx *x);

/* Gap-safe column screening from the dual point of x (not in the paper): with
 * nu = s 2 (Ax - b) as in orc_dual_gap, D is 1/2-strongly concave, so
 * ||nu - nu*|| <= 2 sqrt(F(x) - D(nu)), and |a_l^H nu*| <= |a_l^H nu| + 2 ||a_l|| sqrt(gap).
 * Where that bound is below lambda (1 - 1e-9), the optimality conditions of
 * Eq. (1) force x*_l = 0: mask[l] = 1 (else 0); the relative margin covers the
 * rounding of the bound.  Returns the number of screened bins; gap_out
 * (may be NULL) receives F(x) - D(nu). */
int orc_gap_screen(int n, int l, const ocplx *A, const ocplx *b, double lambda, const ocplx *x,
                   int *mask, double *gap_out);

/* Options of Algorithm 1 with J = 1 (full gradient). */
typedef struct {
    double alpha0;   /* initial step; <= 0 selects 1/(2 max_l ||a_l||^2)          */
    double c_alpha;  /* backtracking factor C_alpha in (0,1)                        */
    double tol;      /* stop when KKT_nat(x^k) <= tol                               */
    int    max_iter; /* N_K                                                         */
    int    backtracking; /* 0: fixed step alpha0                                    */
    int    monotone;     /* 1: accept x-bar only if F(x-bar) <= F(x^k)               */
    int    warm_start;   /* 1: x holds the initial point x^(0) on entry (orc_rbpg)   */
} orc_rbpg_opts;

typedef struct {
    int    iters;       /* iterations performed                                      */
    int    backtracks;  /* total step reductions                                     */
    double alpha;       /* final step                                                */
    double kkt_nat;     /* KKT_nat at the returned point                              */
    double objective;   /* F at the returned point                                    */
    int    converged;   /* 1 if kkt_nat <= tol                                        */
} orc_rbpg_info;

/* Algorithm 1 with one block, FP64.  x (length L) is the output; it starts at
 * x^(0) = 0, or with opt->warm_start at the x^(0) that x holds on entry (the
 * algorithm's initial point is an input).  x^(1) = x^(0) either way. */
void orc_rbpg(int n, int l, const ocplx *A, const ocplx *b, double lambda, double Lf,
              const orc_rbpg_opts *opt, ocplx *x, orc_rbpg_info *info);

/* Active-set damped Newton on the support of x, then the certificate.
 * x is refined in place.  Returns the number of outer active-set rounds. */
int orc_polish(int n, int l, const ocplx *A, const ocplx *b, double lambda, double Lf,
               ocplx *x);

/* Batched drivers, threads over pixels.  lambda has stride lambda_stride
 * (0 => one scalar for all pixels).  Any diagnostic pointer may be NULL.
 * nthreads <= 0 selects the number of online cores. */
/* Algorithm 1 with J blocks (Eqs. (13)-(14)).  Block j covers bins
 * [j w, min(L, (j+1) w)), w = ceil(L/J); L_j = 2 lambda_max(A_j A_j^H) (the
 * Lipschitz constant of the block gradient, Eq. (14)).  Iteration k updates the
 * block i_k drawn with P_i = L_i / sum L (u[k-1] in [0,1) is the draw: i_k is the
 * first j with u sum L < L_0 + ... + L_j).  Readings where the paper is silent:
 * the extrapolation of Eqs. (11)-(12) uses the block's own update count c
 * (beta = max(0, (c-2)/(c+1))) and the block's value before its last update;
 * each block keeps its own step (start 1/(2 max_{l in j} ||a_l||^2), shrunk by
 * C_alpha while Eq. (15) fails on the block, floored at 1/L_j); the monotone test
 * compares F of x^k with block i_k replaced by x-bar; KKT_nat(x^k) <= tol is
 * tested every J iterations.  J = 1 is orc_rbpg. */
double orc_block_lipschitz(int n, int l, const ocplx *A, int J, int j);
int orc_block_pick(int J, const double *Lb, double u);
void orc_rbpg_blocks(int n, int l, const ocplx *A, const ocplx *b, double lambda, double Lf,
                     int J, const double *Lb, const double *u, const orc_rbpg_opts *opt,
                     ocplx *x, orc_rbpg_info *info);
void orc_rbpg_blocks_batch(int n, int l, int64_t p, const ocplx *A, const ocplx *B,
                           const double *lambda, int64_t lambda_stride, int J, const double *u,
                           const orc_rbpg_opts *opt, int nthreads, ocplx *X, int32_t *iters,
                           double *kkt, int32_t *converged);

void orc_rbpg_batch(int n, int l, int64_t p, const ocplx *A, const ocplx *B,
                    const double *lambda, int64_t lambda_stride,
                    const orc_rbpg_opts *opt, int nthreads, ocplx *X,
                    int32_t *iters, double *kkt, int32_t *converged);

/* The minimiser per pixel: Algorithm 1 to a tight stage tolerance, then the
 * Newton polish, then the certificates (KKT_sub, KKT_nat, duality gap). */
void orc_exact_batch(int n, int l, int64_t p, const ocplx *A, const ocplx *B,
                     const double *lambda, int64_t lambda_stride, int nthreads,
                     ocplx *X, double *kkt_sub, double *kkt_nat, double *gap,
                     double *objective);

/* K iterations of the fixed-step accelerated proximal gradient map
 * (Eqs. (11)-(12) with alpha constant, no backtracking, no monotone test),
 * from x^0 = x^{-1} = 0, scalar lambda.  X is the K-th iterate. */
void orc_unrolled_batch(int n, int l, int64_t p, const ocplx *A, const ocplx *B,
                        double lambda, double alpha, int K, int nthreads, ocplx *X);

/* Number of threads the batched drivers use for nthreads <= 0. */
int orc_default_threads(void);

#ifdef __cplusplus
}
#endif
#endif
