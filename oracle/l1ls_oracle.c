/*
 * l1ls_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see the
 * header).  Slow and direct on purpose: per-pixel loops, no blocking, no
 * fusion.  Shares nothing with the GPU path.
 *
 * Paper: Shi, Zhu, Yin, Bamler, arXiv 1805.01759.
 *   Eq. (1)/(6)   problem                     -> orc_objective
 *   Eq. (7)-(9)   proximal-gradient splitting -> orc_rbpg
 *   Eq. (10)      soft-thresholding prox      -> orc_prox (complex form)
 *   Eq. (11)-(12) Nesterov extrapolation      -> orc_rbpg, orc_unrolled_batch
 *   Eq. (14)      L = ||A^T A|| (block Lipschitz; J = 1 -> whole A) -> orc_lipschitz
 *   Eq. (15)      backtracking condition      -> orc_rbpg
 *   Algorithm 1   RBPG with backtracking, J=1 -> orc_rbpg
 *   Eqs. (13)-(14), Algorithm 1 with J blocks  -> orc_rbpg_blocks, orc_block_lipschitz,
 *                                                orc_block_pick
 */
#define _GNU_SOURCE
#include "l1ls_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------ basics */

static double cabs2(ocplx z) { return creal(z) * creal(z) + cimag(z) * cimag(z); }

/* r = A x - b  (length n) */
static void residual(int n, int l, const ocplx *A, const ocplx *b, const ocplx *x, ocplx *r)
{
    for (int i = 0; i < n; ++i) {
        ocplx s = 0;
        for (int j = 0; j < l; ++j) s += A[(int64_t)i * l + j] * x[j];
        r[i] = s - b[i];
    }
}

/* g = 2 A^H r  (length l) */
static void grad_from_residual(int n, int l, const ocplx *A, const ocplx *r, ocplx *g)
{
    for (int j = 0; j < l; ++j) {
        ocplx s = 0;
        for (int i = 0; i < n; ++i) s += conj(A[(int64_t)i * l + j]) * r[i];
        g[j] = 2.0 * s;
    }
}

static double norm1(int m, const ocplx *x)
{
    double s = 0;
    for (int j = 0; j < m; ++j) s += cabs(x[j]);
    return s;
}

static double sqnorm(int m, const ocplx *x)
{
    double s = 0;
    for (int j = 0; j < m; ++j) s += cabs2(x[j]);
    return s;
}

/* ---------------------------------------------------------------- Eq. (10) */

static ocplx prox1(ocplx v, double tau)
{
    double a = cabs(v);
    if (a <= tau) return 0; /* middle case of Eq. (10), ties included */
    return v * (1.0 - tau / a);
}

void orc_prox(int m, const ocplx *v, double tau, ocplx *out)
{
    for (int j = 0; j < m; ++j) out[j] = prox1(v[j], tau);
}

/* ----------------------------------------------------------------- Eq. (1) */

double orc_objective(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                     const ocplx *x)
{
    ocplx *r = malloc(sizeof(ocplx) * n);
    residual(n, l, A, b, x, r);
    double F = sqnorm(n, r) + lambda * norm1(l, x);
    free(r);
    return F;
}

/* ------------------------------------------------------- L_f = 2 lmax(AA^H) */

double orc_lipschitz(int n, int l, const ocplx *A)
{
    int m = 2 * n;
    double *M = calloc((size_t)m * m, sizeof(double));
    /* H = A A^H, embedded as [[Re H, -Im H], [Im H, Re H]] */
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            ocplx h = 0;
            for (int j = 0; j < l; ++j)
                h += A[(int64_t)i * l + j] * conj(A[(int64_t)k * l + j]);
            M[i * m + k] = creal(h);
            M[(i + n) * m + (k + n)] = creal(h);
            M[i * m + (k + n)] = -cimag(h);
            M[(i + n) * m + k] = cimag(h);
        }
    /* cyclic Jacobi rotations until the off-diagonal mass is negligible */
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, tot = 0;
        for (int p = 0; p < m; ++p)
            for (int q = 0; q < m; ++q) {
                tot += M[p * m + q] * M[p * m + q];
                if (p != q) off += M[p * m + q] * M[p * m + q];
            }
        if (off <= 1e-32 * tot || tot == 0) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                double apq = M[p * m + q];
                if (apq == 0) continue;
                double app = M[p * m + p], aqq = M[q * m + q];
                double theta = (aqq - app) / (2 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1));
                double c = 1 / sqrt(t * t + 1), s = t * c;
                for (int k = 0; k < m; ++k) { /* columns p, q */
                    double mkp = M[k * m + p], mkq = M[k * m + q];
                    M[k * m + p] = c * mkp - s * mkq;
                    M[k * m + q] = s * mkp + c * mkq;
                }
                for (int k = 0; k < m; ++k) { /* rows p, q */
                    double mpk = M[p * m + k], mqk = M[q * m + k];
                    M[p * m + k] = c * mpk - s * mqk;
                    M[q * m + k] = s * mpk + c * mqk;
                }
            }
    }
    double lmax = 0;
    for (int p = 0; p < m; ++p)
        if (M[p * m + p] > lmax) lmax = M[p * m + p];
    free(M);
    return 2.0 * lmax;
}

/* ----------------------------------------------------------- KKT measures */

double orc_kkt_nat(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                   double Lf, const ocplx *x)
{
    ocplx *r = malloc(sizeof(ocplx) * n), *g = malloc(sizeof(ocplx) * l);
    residual(n, l, A, b, x, r);
    grad_from_residual(n, l, A, r, g);
    double worst = 0;
    for (int j = 0; j < l; ++j) {
        ocplx p = prox1(x[j] - g[j] / Lf, lambda / Lf);
        double d = cabs(x[j] - p);
        if (d > worst) worst = d;
    }
    free(r);
    free(g);
    return Lf * worst / lambda;
}

double orc_kkt_sub(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                   const ocplx *x)
{
    ocplx *r = malloc(sizeof(ocplx) * n), *g = malloc(sizeof(ocplx) * l);
    residual(n, l, A, b, x, r);
    grad_from_residual(n, l, A, r, g);
    double worst = 0;
    for (int j = 0; j < l; ++j) {
        double v;
        if (x[j] != 0)
            v = cabs(g[j] + lambda * x[j] / cabs(x[j]));
        else
            v = fmax(0.0, cabs(g[j]) - lambda);
        if (v > worst) worst = v;
    }
    free(r);
    free(g);
    return worst / lambda;
}

double orc_dual_gap(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                    const ocplx *x)
{
    ocplx *r = malloc(sizeof(ocplx) * n), *g = malloc(sizeof(ocplx) * l);
    residual(n, l, A, b, x, r);
    grad_from_residual(n, l, A, r, g);
    double gmax = 0;
    for (int j = 0; j < l; ++j) gmax = fmax(gmax, cabs(g[j]));
    double s = (gmax > lambda) ? lambda / gmax : 1.0;
    double nu2 = 0, renub = 0;
    for (int i = 0; i < n; ++i) {
        ocplx nu = s * 2.0 * r[i];
        nu2 += cabs2(nu);
        renub += creal(conj(nu) * b[i]);
    }
    double D = -nu2 / 4.0 - renub;
    double F = sqnorm(n, r) + lambda * norm1(l, x);
    free(r);
    free(g);
    return F - D;
}

int orc_gap_screen(int n, int l, const ocplx *A, const ocplx *b, double lambda, const ocplx *x,
                   int *mask, double *gap_out)
{
    ocplx *r = malloc(sizeof(ocplx) * n), *g = malloc(sizeof(ocplx) * l);
    residual(n, l, A, b, x, r);
    grad_from_residual(n, l, A, r, g); /* g_l = 2 a_l^H r = a_l^H (2 r) */
    double gmax = 0;
    for (int j = 0; j < l; ++j) gmax = fmax(gmax, cabs(g[j]));
    const double s = (gmax > lambda) ? lambda / gmax : 1.0;
    const double gap = orc_dual_gap(n, l, A, b, lambda, x);
    const double rad = 2.0 * sqrt(fmax(gap, 0.0));
    int count = 0;
    for (int j = 0; j < l; ++j) {
        double an = 0;
        for (int i = 0; i < n; ++i) an += cabs2(A[(int64_t)i * l + j]);
        /* a relative margin of 1e-9 covers the rounding of s |g_l| and of the gap:
         * at a minimiser the support bins sit exactly on |a_l^H nu*| = lambda */
        const int out = s * cabs(g[j]) + sqrt(an) * rad < lambda * (1.0 - 1e-9);
        mask[j] = out;
        count += out;
    }
    if (gap_out) *gap_out = gap;
    free(r);
    free(g);
    return count;
}

/* ---------------------------------------------- Algorithm 1, one block J=1 */

void orc_rbpg(int n, int l, const ocplx *A, const ocplx *b, double lambda, double Lf,
              const orc_rbpg_opts *opt, ocplx *x, orc_rbpg_info *info)
{
    ocplx *xprev = calloc(l, sizeof(ocplx)), *y = malloc(sizeof(ocplx) * l);
    ocplx *g = malloc(sizeof(ocplx) * l), *xb = malloc(sizeof(ocplx) * l);
    ocplx *ry = malloc(sizeof(ocplx) * n), *rb = malloc(sizeof(ocplx) * n);
    double colmax = 0;
    for (int j = 0; j < l; ++j) {
        double c = 0;
        for (int i = 0; i < n; ++i) c += cabs2(A[(int64_t)i * l + j]);
        colmax = fmax(colmax, c);
    }
    double alpha = opt->alpha0 > 0 ? opt->alpha0 : 1.0 / (2.0 * colmax);
    double alpha_floor = 1.0 / Lf;
    if (opt->backtracking && alpha < alpha_floor) alpha = alpha_floor;

    double Fx;
    if (opt->warm_start) {
        /* Init: the given x^(0); x^(1) = x^(0), so the first step is a plain
         * backtracked proximal-gradient step from it */
        memcpy(xprev, x, sizeof(ocplx) * l);
        Fx = orc_objective(n, l, A, b, lambda, x);
    } else {
        memset(x, 0, sizeof(ocplx) * l); /* Init: x^(0) = y^(0) = 0 */
        Fx = sqnorm(n, b);               /* F(0) = ||b||^2 */
    }
    int k = 0, backtracks = 0;
    double kkt = orc_kkt_nat(n, l, A, b, lambda, Lf, x);
    int done = kkt <= opt->tol;

    for (k = 1; k <= opt->max_iter && !done; ++k) {
        /* Eq. (11): beta_k = theta_k (1/theta_{k-1} - 1) with theta_k = 2/(k+1),
         * i.e. (k-2)/(k+1); the negative value at k = 1 is clipped to 0. */
        double beta = fmax(0.0, (double)(k - 2) / (double)(k + 1));
        for (int j = 0; j < l; ++j) y[j] = x[j] + beta * (x[j] - xprev[j]);
        residual(n, l, A, b, y, ry);
        grad_from_residual(n, l, A, ry, g);
        double fy = sqnorm(n, ry);
        double fb;
        for (;;) {
            /* Eq. (12): x-bar = prox_{alpha r}(y - alpha grad f(y)) */
            for (int j = 0; j < l; ++j) xb[j] = prox1(y[j] - alpha * g[j], alpha * lambda);
            residual(n, l, A, b, xb, rb);
            fb = sqnorm(n, rb);
            if (!opt->backtracking) break;
            /* Eq. (15): f(x') <= f(y) + Re<grad f(y), x'-y> + ||x'-y||^2 / (2 alpha) */
            double lin = 0, d2 = 0;
            for (int j = 0; j < l; ++j) {
                ocplx d = xb[j] - y[j];
                lin += creal(conj(g[j]) * d);
                d2 += cabs2(d);
            }
            if (fb <= fy + lin + d2 / (2.0 * alpha)) break;
            if (alpha <= alpha_floor) break; /* the condition holds at 1/L_f */
            alpha = fmax(opt->c_alpha * alpha, alpha_floor);
            ++backtracks;
        }
        double Fb = fb + lambda * norm1(l, xb);
        memcpy(xprev, x, sizeof(ocplx) * l);
        if (!opt->monotone || Fb <= Fx) { /* monotone accept (ties accept) */
            memcpy(x, xb, sizeof(ocplx) * l);
            Fx = Fb;
        }
        kkt = orc_kkt_nat(n, l, A, b, lambda, Lf, x);
        if (kkt <= opt->tol) done = 1;
    }
    if (info) {
        info->iters = done ? k - 1 : opt->max_iter;
        if (info->iters < 0) info->iters = 0;
        info->backtracks = backtracks;
        info->alpha = alpha;
        info->kkt_nat = kkt;
        info->objective = orc_objective(n, l, A, b, lambda, x);
        info->converged = kkt <= opt->tol;
    }
    free(xprev);
    free(y);
    free(g);
    free(xb);
    free(ry);
    free(rb);
}


/* ------------------------------- Algorithm 1 with J blocks, Eqs. (13)-(14) */

/* Block j of J covers bins [j w, min(l, (j+1) w)), w = ceil(l / J). */
static void block_range(int l, int J, int j, int *m0, int *m1)
{
    const int w = (l + J - 1) / J;
    *m0 = j * w < l ? j * w : l;
    *m1 = (j + 1) * w < l ? (j + 1) * w : l;
}

double orc_block_lipschitz(int n, int l, const ocplx *A, int J, int j)
{
    int m0, m1;
    block_range(l, J, j, &m0, &m1);
    const int lb = m1 - m0;
    if (lb <= 0) return 0.0;
    ocplx *Aj = malloc(sizeof(ocplx) * (size_t)n * lb);
    for (int i = 0; i < n; ++i)
        for (int m = 0; m < lb; ++m) Aj[(int64_t)i * lb + m] = A[(int64_t)i * l + m0 + m];
    const double L = orc_lipschitz(n, lb, Aj);  /* 2 lambda_max(A_j A_j^H) */
    free(Aj);
    return L;
}

int orc_block_pick(int J, const double *Lb, double u)
{
    double tot = 0;
    for (int j = 0; j < J; ++j) tot += Lb[j];
    double acc = 0;
    for (int j = 0; j < J; ++j) {
        acc += Lb[j];
        if (u * tot < acc) return j;
    }
    return J - 1;
}

void orc_rbpg_blocks(int n, int l, const ocplx *A, const ocplx *b, double lambda, double Lf,
                     int J, const double *Lb, const double *u, const orc_rbpg_opts *opt,
                     ocplx *x, orc_rbpg_info *info)
{
    ocplx *xprev = calloc(l, sizeof(ocplx)), *y = malloc(sizeof(ocplx) * l);
    ocplx *g = malloc(sizeof(ocplx) * l), *xb = malloc(sizeof(ocplx) * l);
    ocplx *ry = malloc(sizeof(ocplx) * n), *rb = malloc(sizeof(ocplx) * n);
    double *alpha = malloc(sizeof(double) * J), *afloor = malloc(sizeof(double) * J);
    int *cnt = calloc(J, sizeof(int));
    for (int jb = 0; jb < J; ++jb) {
        int m0, m1;
        block_range(l, J, jb, &m0, &m1);
        double colmax = 0;
        for (int m = m0; m < m1; ++m) {
            double c = 0;
            for (int i = 0; i < n; ++i) c += cabs2(A[(int64_t)i * l + m]);
            colmax = fmax(colmax, c);
        }
        alpha[jb] = opt->alpha0 > 0 ? opt->alpha0 : (colmax > 0 ? 1.0 / (2.0 * colmax) : 1.0);
        afloor[jb] = Lb[jb] > 0 ? 1.0 / Lb[jb] : alpha[jb];
        if (opt->backtracking && alpha[jb] < afloor[jb]) alpha[jb] = afloor[jb];
    }

    memset(x, 0, sizeof(ocplx) * l); /* Init: x^(0) = y^(0) = 0 */
    double Fx = sqnorm(n, b);
    int k = 0, backtracks = 0;
    double kkt = orc_kkt_nat(n, l, A, b, lambda, Lf, x);
    int done = kkt <= opt->tol;

    for (k = 1; k <= opt->max_iter && !done; ++k) {
        /* i_k drawn with P_i = L_i / sum_j L_j (Eq. (14)); u[k-1] is the draw */
        const int ib = orc_block_pick(J, Lb, u[k - 1]);
        int m0, m1;
        block_range(l, J, ib, &m0, &m1);
        /* Eqs. (11)-(12) on block i_k with its own update count and its own
         * previous value; the other blocks of y are those of x^k */
        ++cnt[ib];
        const double beta = fmax(0.0, (double)(cnt[ib] - 2) / (double)(cnt[ib] + 1));
        memcpy(y, x, sizeof(ocplx) * l);
        for (int m = m0; m < m1; ++m) y[m] = x[m] + beta * (x[m] - xprev[m]);
        residual(n, l, A, b, y, ry);
        grad_from_residual(n, l, A, ry, g); /* only the block's part is used */
        const double fy = sqnorm(n, ry);
        double fb;
        for (;;) {
            /* Eq. (13): the block's prox-gradient step */
            memcpy(xb, y, sizeof(ocplx) * l);
            for (int m = m0; m < m1; ++m) xb[m] = prox1(y[m] - alpha[ib] * g[m], alpha[ib] * lambda);
            residual(n, l, A, b, xb, rb);
            fb = sqnorm(n, rb);
            if (!opt->backtracking) break;
            /* Eq. (15) on the block */
            double lin = 0, d2 = 0;
            for (int m = m0; m < m1; ++m) {
                ocplx d = xb[m] - y[m];
                lin += creal(conj(g[m]) * d);
                d2 += cabs2(d);
            }
            if (fb <= fy + lin + d2 / (2.0 * alpha[ib])) break;
            if (alpha[ib] <= afloor[ib]) break;
            alpha[ib] = fmax(opt->c_alpha * alpha[ib], afloor[ib]);
            ++backtracks;
        }
        const double Fb = fb + lambda * norm1(l, xb);
        for (int m = m0; m < m1; ++m) xprev[m] = x[m];
        if (!opt->monotone || Fb <= Fx) { /* monotone accept (ties accept) */
            memcpy(x, xb, sizeof(ocplx) * l);
            Fx = Fb;
        }
        /* the KKT test once per J block updates */
        if (k % J == 0) {
            kkt = orc_kkt_nat(n, l, A, b, lambda, Lf, x);
            if (kkt <= opt->tol) done = 1;
        }
    }
    if (info) {
        info->iters = done ? k - 1 : opt->max_iter;
        if (info->iters < 0) info->iters = 0;
        info->backtracks = backtracks;
        info->alpha = alpha[0];
        info->kkt_nat = orc_kkt_nat(n, l, A, b, lambda, Lf, x);
        info->objective = orc_objective(n, l, A, b, lambda, x);
        info->converged = info->kkt_nat <= opt->tol;
    }
    free(xprev);
    free(y);
    free(g);
    free(xb);
    free(ry);
    free(rb);
    free(alpha);
    free(afloor);
    free(cnt);
}

/* ------------------------------------------ active-set Newton polish (FP64) */

/* Cholesky solve of the SPD system H d = rhs (size m, H overwritten).
 * Returns 0 on success, -1 if H is not numerically positive definite. */
static int chol_solve(int m, double *H, double *rhs)
{
    for (int j = 0; j < m; ++j) {
        double s = H[j * m + j];
        for (int k = 0; k < j; ++k) s -= H[j * m + k] * H[j * m + k];
        if (!(s > 0)) return -1;
        double d = sqrt(s);
        H[j * m + j] = d;
        for (int i = j + 1; i < m; ++i) {
            double t = H[i * m + j];
            for (int k = 0; k < j; ++k) t -= H[i * m + k] * H[j * m + k];
            H[i * m + j] = t / d;
        }
    }
    for (int i = 0; i < m; ++i) {
        double t = rhs[i];
        for (int k = 0; k < i; ++k) t -= H[i * m + k] * rhs[k];
        rhs[i] = t / H[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double t = rhs[i];
        for (int k = i + 1; k < m; ++k) t -= H[k * m + i] * rhs[k];
        rhs[i] = t / H[i * m + i];
    }
    return 0;
}

/* phi(z) = ||A_S z - b||^2 + lambda sum |z_s|  on the support list S */
static double phi_on_support(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                             int s, const int *S, const ocplx *z, ocplx *r)
{
    for (int i = 0; i < n; ++i) {
        ocplx acc = 0;
        for (int t = 0; t < s; ++t) acc += A[(int64_t)i * l + S[t]] * z[t];
        r[i] = acc - b[i];
    }
    return sqnorm(n, r) + lambda * norm1(s, z);
}

/* Damped Newton on phi over the support of x (in place).  A coordinate whose
 * Newton step passes through the origin is set to zero and leaves the support. */
static void newton_on_support(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                              double Lf, ocplx *x, int *S, ocplx *z, ocplx *zt, ocplx *r,
                              double *H, double *Hc, double *rhs, double *grd)
{
    int s = 0;
    for (int j = 0; j < l; ++j)
        if (x[j] != 0) { S[s] = j; z[s] = x[j]; ++s; }
    for (int it = 0; it < 100 && s > 0; ++it) {
        double ph = phi_on_support(n, l, A, b, lambda, s, S, z, r);
        /* gradient (real pairs) and Hessian 2 realify(A_S^H A_S) + lambda (I - u u^T)/|z| */
        double gscale = 0;
        for (int t = 0; t < s; ++t) {
            ocplx acc = 0;
            for (int i = 0; i < n; ++i) acc += conj(A[(int64_t)i * l + S[t]]) * r[i];
            ocplx gt = 2.0 * acc + lambda * z[t] / cabs(z[t]);
            grd[t] = creal(gt);
            grd[t + s] = cimag(gt);
            gscale = fmax(gscale, cabs(gt));
        }
        if (gscale <= 1e-15 * lambda) break;
        int m = 2 * s;
        for (int t = 0; t < s; ++t)
            for (int u = 0; u < s; ++u) {
                ocplx gtu = 0;
                for (int i = 0; i < n; ++i)
                    gtu += conj(A[(int64_t)i * l + S[t]]) * A[(int64_t)i * l + S[u]];
                H[t * m + u] = 2 * creal(gtu);
                H[(t + s) * m + (u + s)] = 2 * creal(gtu);
                H[t * m + (u + s)] = -2 * cimag(gtu);
                H[(t + s) * m + u] = 2 * cimag(gtu);
            }
        for (int t = 0; t < s; ++t) {
            double a = cabs(z[t]);
            double ur = creal(z[t]) / a, ui = cimag(z[t]) / a;
            H[t * m + t] += lambda * (1 - ur * ur) / a;
            H[(t + s) * m + (t + s)] += lambda * (1 - ui * ui) / a;
            H[t * m + (t + s)] += -lambda * ur * ui / a;
            H[(t + s) * m + t] += -lambda * ur * ui / a;
        }
        double mu = 0;
        for (;;) {
            memcpy(Hc, H, sizeof(double) * m * m);
            for (int t = 0; t < m; ++t) { Hc[t * m + t] += mu; rhs[t] = -grd[t]; }
            if (chol_solve(m, Hc, rhs) == 0) break;
            mu = mu == 0 ? 1e-14 * Lf : mu * 10;
        }
        /* the coordinate whose Newton step reverses it most (relative to its
         * modulus) leaves the support; one at a time */
        int drop = -1;
        double worst_c = 0;
        for (int t = 0; t < s; ++t) {
            ocplx zn = z[t] + (rhs[t] + I * rhs[t + s]);
            double c = creal(conj(z[t]) * zn) / cabs2(z[t]);
            if (c <= 0 && (drop < 0 || c < worst_c)) { drop = t; worst_c = c; }
        }
        if (drop >= 0) {
            z[drop] = 0;
            int w = 0;
            for (int t = 0; t < s; ++t)
                if (z[t] != 0) { S[w] = S[t]; z[w] = z[t]; ++w; }
            s = w;
            continue;
        }
        /* Armijo backtracking on phi */
        double slope = 0;
        for (int t = 0; t < m; ++t) slope += grd[t] * rhs[t];
        double step = 1.0;
        int accepted = 0;
        for (int ls = 0; ls < 60; ++ls) {
            for (int t = 0; t < s; ++t) zt[t] = z[t] + step * (rhs[t] + I * rhs[t + s]);
            double pn = phi_on_support(n, l, A, b, lambda, s, S, zt, r);
            if (pn <= ph + 1e-4 * step * slope) { accepted = 1; break; }
            step *= 0.5;
        }
        if (!accepted) break;
        memcpy(z, zt, sizeof(ocplx) * s);
    }
    memset(x, 0, sizeof(ocplx) * l);
    for (int t = 0; t < s; ++t) x[S[t]] = z[t];
}

/* Polish: alternate a few proximal-gradient steps at step 1/L_f (which fix the
 * support: they zero coordinates whose optimum is 0 and admit violators) with
 * damped Newton on the resulting support.  The best point by F is kept. */
int orc_polish(int n, int l, const ocplx *A, const ocplx *b, double lambda, double Lf,
               ocplx *x)
{
    int *S = malloc(sizeof(int) * l);
    ocplx *z = malloc(sizeof(ocplx) * l), *zt = malloc(sizeof(ocplx) * l);
    ocplx *r = malloc(sizeof(ocplx) * n), *g = malloc(sizeof(ocplx) * l);
    ocplx *best = malloc(sizeof(ocplx) * l);
    double *H = malloc(sizeof(double) * 4 * (size_t)l * l);
    double *Hc = malloc(sizeof(double) * 4 * (size_t)l * l);
    double *rhs = malloc(sizeof(double) * 2 * l), *grd = malloc(sizeof(double) * 2 * l);
    memcpy(best, x, sizeof(ocplx) * l);
    double Fbest = orc_objective(n, l, A, b, lambda, x);
    int round;
    for (round = 0; round < 40; ++round) {
        for (int t = 0; t < 3; ++t) {
            residual(n, l, A, b, x, r);
            grad_from_residual(n, l, A, r, g);
            for (int j = 0; j < l; ++j) x[j] = prox1(x[j] - g[j] / Lf, lambda / Lf);
        }
        newton_on_support(n, l, A, b, lambda, Lf, x, S, z, zt, r, H, Hc, rhs, grd);
        double F = orc_objective(n, l, A, b, lambda, x);
        if (F <= Fbest) { Fbest = F; memcpy(best, x, sizeof(ocplx) * l); }
        if (orc_kkt_sub(n, l, A, b, lambda, x) <= 1e-13) break;
    }
    memcpy(x, best, sizeof(ocplx) * l);
    free(S);
    free(z);
    free(zt);
    free(r);
    free(g);
    free(best);
    free(H);
    free(Hc);
    free(rhs);
    free(grd);
    return round;
}

/* Homotopy in lambda: follow the solution path from lambda_max (x = 0) down
 * to the target lambda on a geometric grid.  At every grid value the working
 * set is updated until the subgradient conditions hold: damped Newton on the
 * support (a coordinate whose Newton step passes through the origin leaves),
 * then the worst violator enters at its exact coordinate minimiser. */
static void homotopy_solve(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                           double Lf, ocplx *x)
{
    int *S = malloc(sizeof(int) * l);
    ocplx *z = malloc(sizeof(ocplx) * l), *zt = malloc(sizeof(ocplx) * l);
    ocplx *r = malloc(sizeof(ocplx) * n), *g = malloc(sizeof(ocplx) * l);
    double *H = malloc(sizeof(double) * 4 * (size_t)l * l);
    double *Hc = malloc(sizeof(double) * 4 * (size_t)l * l);
    double *rhs = malloc(sizeof(double) * 2 * l), *grd = malloc(sizeof(double) * 2 * l);
    double *cn = malloc(sizeof(double) * l);
    for (int j = 0; j < l; ++j) {
        cn[j] = 0;
        for (int i = 0; i < n; ++i) cn[j] += cabs2(A[(int64_t)i * l + j]);
    }
    memset(x, 0, sizeof(ocplx) * l);
    residual(n, l, A, b, x, r);
    grad_from_residual(n, l, A, r, g);
    double lmax = 0;
    for (int j = 0; j < l; ++j) lmax = fmax(lmax, cabs(g[j]));
    if (lambda < lmax) {
        const int stages = 50;
        double ratio = pow(lambda / lmax, 1.0 / stages);
        for (int st = 1; st <= stages; ++st) {
            double lam = st == stages ? lambda : lmax * pow(ratio, st);
            for (int inner = 0; inner < 4 * l; ++inner) {
                newton_on_support(n, l, A, b, lam, Lf, x, S, z, zt, r, H, Hc, rhs, grd);
                residual(n, l, A, b, x, r);
                grad_from_residual(n, l, A, r, g);
                int worst = -1;
                double wv = lam * (1 + 1e-13);
                for (int j = 0; j < l; ++j)
                    if (x[j] == 0 && cabs(g[j]) > wv) { wv = cabs(g[j]); worst = j; }
                if (worst < 0) break;
                /* exact minimiser of F along coordinate `worst` with the others fixed */
                x[worst] = prox1(-g[worst] / (2 * cn[worst]), lam / (2 * cn[worst]));
                if (x[worst] == 0) break;
            }
        }
    }
    free(S);
    free(z);
    free(zt);
    free(r);
    free(g);
    free(H);
    free(Hc);
    free(rhs);
    free(grd);
    free(cn);
}

/* --------------------------------------------------------- batched drivers */

int orc_default_threads(void)
{
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

typedef struct {
    int kind; /* 0 rbpg, 1 exact, 2 unrolled, 3 rbpg with J blocks */
    int n, l;
    int64_t p0, p1;
    const ocplx *A, *B;
    const double *lambda;
    int64_t lambda_stride;
    const orc_rbpg_opts *opt;
    double Lf, alpha, lam_scalar;
    int K;
    ocplx *X;
    int32_t *iters, *converged;
    double *kkt, *kkt_sub, *kkt_nat, *gap, *objective;
    int J;
    const double *Lb, *u;
} job_t;

static void unrolled_one(int n, int l, const ocplx *A, const ocplx *b, double lambda,
                         double alpha, int K, ocplx *x)
{
    ocplx *xprev = calloc(l, sizeof(ocplx)), *y = malloc(sizeof(ocplx) * l);
    ocplx *g = malloc(sizeof(ocplx) * l), *r = malloc(sizeof(ocplx) * n);
    memset(x, 0, sizeof(ocplx) * l);
    for (int k = 1; k <= K; ++k) {
        double beta = fmax(0.0, (double)(k - 2) / (double)(k + 1));
        for (int j = 0; j < l; ++j) y[j] = x[j] + beta * (x[j] - xprev[j]);
        residual(n, l, A, b, y, r);
        grad_from_residual(n, l, A, r, g);
        memcpy(xprev, x, sizeof(ocplx) * l);
        for (int j = 0; j < l; ++j) x[j] = prox1(y[j] - alpha * g[j], alpha * lambda);
    }
    free(xprev);
    free(y);
    free(g);
    free(r);
}

static void *worker(void *arg)
{
    job_t *j = (job_t *)arg;
    for (int64_t p = j->p0; p < j->p1; ++p) {
        const ocplx *b = j->B + p * j->n;
        ocplx *x = j->X + p * j->l;
        if (j->kind == 2) {
            unrolled_one(j->n, j->l, j->A, b, j->lam_scalar, j->alpha, j->K, x);
            continue;
        }
        double lam = j->lambda[j->lambda_stride * p];
        if (j->kind == 3) {
            orc_rbpg_info info;
            orc_rbpg_blocks(j->n, j->l, j->A, b, lam, j->Lf, j->J, j->Lb, j->u, j->opt, x, &info);
            if (j->iters) j->iters[p] = info.iters;
            if (j->kkt) j->kkt[p] = info.kkt_nat;
            if (j->converged) j->converged[p] = info.converged;
        } else if (j->kind == 0) {
            orc_rbpg_info info;
            orc_rbpg(j->n, j->l, j->A, b, lam, j->Lf, j->opt, x, &info);
            if (j->iters) j->iters[p] = info.iters;
            if (j->kkt) j->kkt[p] = info.kkt_nat;
            if (j->converged) j->converged[p] = info.converged;
        } else {
            /* minimiser: homotopy path; if its certificate is not tight, also try
             * Algorithm 1 followed by the polish, and keep the better point */
            homotopy_solve(j->n, j->l, j->A, b, lam, j->Lf, x);
            orc_polish(j->n, j->l, j->A, b, lam, j->Lf, x);
            if (orc_kkt_sub(j->n, j->l, j->A, b, lam, x) > 1e-11) {
                ocplx *x2 = malloc(sizeof(ocplx) * j->l);
                orc_rbpg_opts o = {0, 0.5, 1e-7, 20000, 1, 1};
                orc_rbpg_info info;
                orc_rbpg(j->n, j->l, j->A, b, lam, j->Lf, &o, x2, &info);
                orc_polish(j->n, j->l, j->A, b, lam, j->Lf, x2);
                if (orc_kkt_sub(j->n, j->l, j->A, b, lam, x2) < orc_kkt_sub(j->n, j->l, j->A, b, lam, x))
                    memcpy(x, x2, sizeof(ocplx) * j->l);
                free(x2);
            }
            if (j->kkt_sub) j->kkt_sub[p] = orc_kkt_sub(j->n, j->l, j->A, b, lam, x);
            if (j->kkt_nat) j->kkt_nat[p] = orc_kkt_nat(j->n, j->l, j->A, b, lam, j->Lf, x);
            if (j->gap) j->gap[p] = orc_dual_gap(j->n, j->l, j->A, b, lam, x);
            if (j->objective) j->objective[p] = orc_objective(j->n, j->l, j->A, b, lam, x);
        }
    }
    return NULL;
}

static void run_jobs(job_t *proto, int64_t p, int nthreads)
{
    if (nthreads <= 0) nthreads = orc_default_threads();
    if (nthreads > p) nthreads = (int)(p > 0 ? p : 1);
    pthread_t *th = malloc(sizeof(pthread_t) * nthreads);
    job_t *jobs = malloc(sizeof(job_t) * nthreads);
    /* interleave contiguous chunks so that hard and easy pixels mix */
    int64_t chunk = (p + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *proto;
        jobs[t].p0 = (int64_t)t * chunk;
        jobs[t].p1 = jobs[t].p0 + chunk < p ? jobs[t].p0 + chunk : p;
        pthread_create(&th[t], NULL, worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
}

void orc_rbpg_batch(int n, int l, int64_t p, const ocplx *A, const ocplx *B,
                    const double *lambda, int64_t lambda_stride,
                    const orc_rbpg_opts *opt, int nthreads, ocplx *X,
                    int32_t *iters, double *kkt, int32_t *converged)
{
    job_t j;
    memset(&j, 0, sizeof j);
    j.kind = 0;
    j.n = n; j.l = l; j.A = A; j.B = B; j.lambda = lambda; j.lambda_stride = lambda_stride;
    j.opt = opt; j.Lf = orc_lipschitz(n, l, A); j.X = X;
    j.iters = iters; j.kkt = kkt; j.converged = converged;
    run_jobs(&j, p, nthreads);
}

void orc_rbpg_blocks_batch(int n, int l, int64_t p, const ocplx *A, const ocplx *B,
                           const double *lambda, int64_t lambda_stride, int J, const double *u,
                           const orc_rbpg_opts *opt, int nthreads, ocplx *X, int32_t *iters,
                           double *kkt, int32_t *converged)
{
    double *Lb = malloc(sizeof(double) * J);
    for (int jb = 0; jb < J; ++jb) Lb[jb] = orc_block_lipschitz(n, l, A, J, jb);
    job_t j;
    memset(&j, 0, sizeof j);
    j.kind = 3;
    j.n = n; j.l = l; j.A = A; j.B = B; j.lambda = lambda; j.lambda_stride = lambda_stride;
    j.opt = opt; j.Lf = orc_lipschitz(n, l, A); j.X = X;
    j.iters = iters; j.kkt = kkt; j.converged = converged;
    j.J = J; j.Lb = Lb; j.u = u;
    run_jobs(&j, p, nthreads);
    free(Lb);
}

void orc_exact_batch(int n, int l, int64_t p, const ocplx *A, const ocplx *B,
                     const double *lambda, int64_t lambda_stride, int nthreads,
                     ocplx *X, double *kkt_sub, double *kkt_nat, double *gap,
                     double *objective)
{
    job_t j;
    memset(&j, 0, sizeof j);
    j.kind = 1;
    j.n = n; j.l = l; j.A = A; j.B = B; j.lambda = lambda; j.lambda_stride = lambda_stride;
    j.Lf = orc_lipschitz(n, l, A); j.X = X;
    j.kkt_sub = kkt_sub; j.kkt_nat = kkt_nat; j.gap = gap; j.objective = objective;
    run_jobs(&j, p, nthreads);
}

void orc_unrolled_batch(int n, int l, int64_t p, const ocplx *A, const ocplx *B,
                        double lambda, double alpha, int K, int nthreads, ocplx *X)
{
    job_t j;
    memset(&j, 0, sizeof j);
    j.kind = 2;
    j.n = n; j.l = l; j.A = A; j.B = B; j.lam_scalar = lambda; j.alpha = alpha; j.K = K;
    j.X = X;
    run_jobs(&j, p, nthreads);
}
