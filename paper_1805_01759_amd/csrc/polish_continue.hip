// FP64 continuation of Algorithm 1 (J = 1; arXiv 1805.01759, Algorithm 1 with
// the prox of Eq. (10), the extrapolation of Eqs. (11)-(12) and the backtracking
// condition of Eq. (15)) for the pixels the FP64 refinement leaves above tol:
// minimisers with more nonzeros than its 32-slot working set holds, or an
// active-set walk that stalls.  Algorithm 1 has no limit on the support; in FP32
// it stalls above tol on such pixels, in FP64 it reaches it.
//
// One 64-lane workgroup per listed pixel (pixels from a shared counter), warm
// started from the best point the refinement wrote to X, with the step reset to
// alpha_0 (as Algorithm 1's Init from a given x^(0)), up to max_iter iterations
// in all (the FP32 stage's count included).  Lane j holds bins j + 64 c of x^k,
// G_k = 2 A^H r_k and the trial point x-bar in registers; x^{k-1}, G_{k-1}, the
// forward operand d and the residuals sit in LDS.  The gradient is affine, so
// G(y) = G_k + beta (G_k - G_{k-1}) and r(y) = r_k + beta (r_k - r_{k-1}) need no
// product; a trial costs one forward product A d (through the transposed copy
// of A, lanes over rows), an accepted step one adjoint (lanes over bins).
// Eq. (15) is tested as ||A d||^2 <= ||d||^2 / (2 alpha) (for quadratic f the
// two forms are the same), the monotone test of Algorithm 1 on F in FP64.
#include <algorithm>

#include "l1ls_internal.h"
#include "wave_reduce.h"

namespace l1ls {

using wr::wmax;
using wr::wsum;

struct ContinueArgs {
    int n, l, l_pad;
    const float2 *A;          // packed: rows_pad x l_pad
    const float2 *At;         // l_pad x n
    const float2 *B;
    const float *lambda;
    int64_t lambda_stride;
    float2 *X;
    const StackConsts *consts;
    const int32_t *list;      // pixels the 32-slot refinement left above tol
    const uint32_t *count;
    uint32_t *next;
    int32_t *iters;           // per-pixel iteration counts (the FP64 ones are added)
    unsigned long long *work; // [2]: FP64 flops
    int32_t budget;           // iterations left after the FP32 stage
    float tol, c_alpha;
    int32_t backtracking, monotone;
};

__host__ __device__ inline ContinueArgs continue_args_for(const StackDesc &d, const SolveOpts &o)
{
    const StackWorkspace lay = stack_workspace_layout(d.n, d.l, d.p);
    uint32_t *queue = (uint32_t *)(d.ws + lay.queue);
    ContinueArgs ca;
    ca.n = d.n;
    ca.l = d.l;
    ca.l_pad = lpad_for(d.l);
    ca.A = (const float2 *)(d.ws + lay.a_packed);
    ca.At = (const float2 *)(d.ws + lay.a_trans);
    ca.B = d.B;
    ca.lambda = d.lambda;
    ca.lambda_stride = d.lambda_stride;
    ca.X = d.X;
    ca.consts = (const StackConsts *)(d.ws + lay.consts);
    ca.list = (const int32_t *)(d.ws + lay.overflow);
    ca.count = queue + 7;
    ca.next = queue + 8;
    ca.iters = (int32_t *)(d.ws + lay.iters);
    ca.work = (unsigned long long *)(d.ws + lay.work);
    ca.budget = o.max_iter > o.fista_cap ? o.max_iter - o.fista_cap : 0;
    ca.tol = o.tol;
    ca.c_alpha = o.c_alpha;
    ca.backtracking = o.backtracking;
    ca.monotone = o.monotone;
    return ca;
}

// LDS: x^{k-1}, G_{k-1}, d (l_pad each) and r_k, r_{k-1}, A d, r(y) (n each)
static size_t continue_lds(int n, int l_pad) { return (size_t)(3 * l_pad + 4 * n) * sizeof(double2); }

template <int NC>
__device__ __forceinline__ void continue_stack(const ContinueArgs &a)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    const int lane = threadIdx.x;
    const int n = a.n, l = a.l, lp = a.l_pad;
    double2 *sxp = reinterpret_cast<double2 *>(dyn);
    double2 *sgp = sxp + lp;
    double2 *sd = sgp + lp;
    double2 *sr = sd + lp;
    double2 *srp = sr + n;
    double2 *sw = srp + n;
    double2 *sry = sw + n;
    const double lf = a.consts->lf, inv_lf = 1.0 / lf, afloor = inv_lf;
    const double alpha0 = a.consts->alpha0;
    const uint32_t count = *a.count;
    const unsigned long long prod = 8ull * (unsigned long long)n * (unsigned long long)l;
    unsigned long long fl = 0;

    // sw = A sd (lanes over rows, the transposed copy read contiguously; eight
    // bins' loads in flight)
    auto forward = [&]() {
        for (int nn = lane; nn < n; nn += 64) {
            double wr = 0.0, wi = 0.0;
            int m = 0;
            for (; m + 8 <= l; m += 8) {
                float2 av[8];
                double2 dv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    av[u] = a.At[(size_t)(m + u) * n + nn];
                    dv[u] = sd[m + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    wr += (double)av[u].x * dv[u].x - (double)av[u].y * dv[u].y;
                    wi += (double)av[u].x * dv[u].y + (double)av[u].y * dv[u].x;
                }
            }
            for (; m < l; ++m) {
                const float2 av = a.At[(size_t)m * n + nn];
                const double2 dv = sd[m];
                wr += (double)av.x * dv.x - (double)av.y * dv.y;
                wi += (double)av.x * dv.y + (double)av.y * dv.x;
            }
            sw[nn] = make_double2(wr, wi);
        }
        __syncthreads();
    };
    // G = 2 A^H sr for the lane's bins (four rows' loads in flight per chunk)
    auto adjoint = [&](double (&gr)[NC], double (&gi)[NC]) {
#pragma unroll
        for (int c = 0; c < NC; ++c) gr[c] = gi[c] = 0.0;
        for (int n0 = 0; n0 < n; n0 += 4) {
            double2 rv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) rv[u] = n0 + u < n ? sr[n0 + u] : make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int m = lane + 64 * c;
                if (m >= lp) continue;
                float2 av[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    av[u] = n0 + u < n ? a.A[(size_t)(n0 + u) * lp + m] : make_float2(0.0f, 0.0f);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    gr[c] += (double)av[u].x * rv[u].x + (double)av[u].y * rv[u].y;  // conj(a) r
                    gi[c] += (double)av[u].x * rv[u].y - (double)av[u].y * rv[u].x;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            gr[c] *= 2.0;
            gi[c] *= 2.0;
        }
    };
    // natural KKT residual L_f max |x - S_{lambda/L_f}(x - G/L_f)| / lambda
    auto kkt_of = [&](const double (&xr)[NC], const double (&xi)[NC], const double (&gr)[NC],
                      const double (&gi)[NC], double lam) {
        const double tau = lam * inv_lf, tau2 = tau * tau;
        double km = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double vr = xr[c] - gr[c] * inv_lf, vi = xi[c] - gi[c] * inv_lf;
            const double m2 = vr * vr + vi * vi;
            double er = xr[c], ei = xi[c];
            if (m2 > tau2) {
                const double sc = 1.0 - tau / sqrt(m2);
                er = xr[c] - vr * sc;
                ei = xi[c] - vi * sc;
            }
            km = fmax(km, er * er + ei * ei);
        }
        return lf * sqrt(wmax(km)) / lam;
    };

    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(a.next, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= count) break;
        const int64_t p = a.list[item];
        const float lam_f = a.lambda[p * a.lambda_stride];
        if (!(lam_f > 0.0f) || !isfinite(lam_f)) continue;
        const double lam = lam_f;
        float2 *xo = a.X + (size_t)p * l;
        const float2 *b = a.B + (size_t)p * n;
        double xr[NC], xi[NC], gr[NC], gi[NC], br[NC], bi[NC];
        double l1 = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int m = lane + 64 * c;
            const float2 v = m < l ? xo[m] : make_float2(0.0f, 0.0f);
            xr[c] = v.x;
            xi[c] = v.y;
            br[c] = bi[c] = 0.0;
            if (m < lp) {
                sd[m] = make_double2(xr[c], xi[c]);
                sxp[m] = sd[m];
            }
            l1 += sqrt(xr[c] * xr[c] + xi[c] * xi[c]);
        }
        __syncthreads();
        // Init from x^(0): r_1 = A x^(0) - b, F(x^(0)), G_1; x^(0) doubles as x^{k-1}
        forward();
        double rr = 0.0;
        for (int nn = lane; nn < n; nn += 64) {
            const float2 bb = b[nn];
            const double2 w = sw[nn];
            const double2 r = make_double2(w.x - bb.x, w.y - bb.y);
            sr[nn] = r;
            srp[nn] = r;
            rr += r.x * r.x + r.y * r.y;
        }
        __syncthreads();
        double F = wsum(rr) + lam * wsum(l1);
        const double F0 = F;
        adjoint(gr, gi);
        fl += 2 * prod;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int m = lane + 64 * c;
            if (m < lp) sgp[m] = make_double2(gr[c], gi[c]);
        }
        __syncthreads();
        double alpha = a.backtracking ? fmax(alpha0, afloor) : afloor;
        bool done = kkt_of(xr, xi, gr, gi, lam) <= (double)a.tol;
        int k = 1;
        for (; k <= a.budget && !done; ++k) {
            const double beta = fmax(0.0, (double)(k - 2) / (double)(k + 1));
            for (int nn = lane; nn < n; nn += 64) {
                const double2 r = sr[nn], rp = srp[nn];
                sry[nn] = make_double2(r.x + beta * (r.x - rp.x), r.y + beta * (r.y - rp.y));
            }
            double d2, w2, l1b;
            for (;;) {
                // x-bar = S_{alpha lambda}(y - alpha G(y)) (Eqs. (10), (12)); d = x-bar - y
                const double tau = alpha * lam;
                d2 = 0.0;
                l1b = 0.0;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const int m = lane + 64 * c;
                    if (m >= lp) continue;
                    const double2 xp = sxp[m], gp = sgp[m];
                    const double yr = xr[c] + beta * (xr[c] - xp.x), yi = xi[c] + beta * (xi[c] - xp.y);
                    const double gyr = gr[c] + beta * (gr[c] - gp.x), gyi = gi[c] + beta * (gi[c] - gp.y);
                    const double vr = yr - alpha * gyr, vi = yi - alpha * gyi;
                    const double mv = sqrt(vr * vr + vi * vi);
                    const double sc = mv > tau ? 1.0 - tau / mv : 0.0;
                    br[c] = m < l ? vr * sc : 0.0;
                    bi[c] = m < l ? vi * sc : 0.0;
                    const double dr = br[c] - (m < l ? yr : 0.0), di = bi[c] - (m < l ? yi : 0.0);
                    sd[m] = make_double2(dr, di);
                    d2 += dr * dr + di * di;
                    l1b += mv > tau && m < l ? mv - tau : 0.0;
                }
                __syncthreads();
                forward();
                fl += prod;
                double ww = 0.0;
                for (int nn = lane; nn < n; nn += 64) ww += sw[nn].x * sw[nn].x + sw[nn].y * sw[nn].y;
                w2 = wsum(ww);
                d2 = wsum(d2);
                // Eq. (15) in the form ||A d||^2 <= ||d||^2 / (2 alpha); it holds at 1/L_f
                if (!a.backtracking || w2 <= d2 / (2.0 * alpha) || alpha <= afloor) break;
                alpha = fmax((double)a.c_alpha * alpha, afloor);
                __syncthreads();
            }
            l1b = wsum(l1b);
            // r-bar = r(y) + A d, F(x-bar)
            double fb = 0.0;
            for (int nn = lane; nn < n; nn += 64) {
                const double2 ry = sry[nn], w = sw[nn];
                const double2 rb = make_double2(ry.x + w.x, ry.y + w.y);
                sw[nn] = rb;
                fb += rb.x * rb.x + rb.y * rb.y;
            }
            const double Fb = wsum(fb) + lam * l1b;
            const bool acc = !a.monotone || Fb <= F;  // monotone accept (ties accept)
            // x^{k-1} <- x^k (G, r alike), then x^{k+1} = x-bar on acceptance, else x^k
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int m = lane + 64 * c;
                if (m < lp) {
                    sxp[m] = make_double2(xr[c], xi[c]);
                    sgp[m] = make_double2(gr[c], gi[c]);
                }
                if (acc) {
                    xr[c] = br[c];
                    xi[c] = bi[c];
                }
            }
            for (int nn = lane; nn < n; nn += 64) {
                srp[nn] = sr[nn];
                if (acc) sr[nn] = sw[nn];
            }
            __syncthreads();
            if (acc) {
                F = Fb;
                adjoint(gr, gi);
                fl += prod;
            }
            done = kkt_of(xr, xi, gr, gi, lam) <= (double)a.tol;
        }
        // the result replaces the refinement's point only where it improved on it
        if (F < F0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int m = lane + 64 * c;
                if (m < l) xo[m] = make_float2((float)xr[c], (float)xi[c]);
            }
        }
        if (lane == 0 && a.iters) a.iters[p] += k - 1;
        __syncthreads();
    }
    if (lane == 0 && fl) atomicAdd(&a.work[2], fl);
}

// The same continuation for stacks beyond kContMaxL bins: the six L-vectors of a
// pixel (x^k, x^{k-1}, G_k, G_{k-1}, x-bar and d) live in the workgroup's
// workspace slot instead of registers and LDS, each bin's arithmetic and the
// order of its sums being those above; only the N-vectors stay in LDS.
__device__ __forceinline__ void continue_stack_g(const ContinueArgs &a, double2 *slot)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    const int lane = threadIdx.x;
    const int n = a.n, l = a.l, lp = a.l_pad;
    double2 *X = slot, *XP = X + lp, *G = XP + lp, *GP = G + lp, *XB = GP + lp, *D = XB + lp;
    double2 *sr = reinterpret_cast<double2 *>(dyn);
    double2 *srp = sr + n;
    double2 *sw = srp + n;
    double2 *sry = sw + n;
    const double lf = a.consts->lf, inv_lf = 1.0 / lf, afloor = inv_lf;
    const double alpha0 = a.consts->alpha0;
    const uint32_t count = *a.count;
    const unsigned long long prod = 8ull * (unsigned long long)n * (unsigned long long)l;
    unsigned long long fl = 0;

    // sw = A D (lanes over rows, the transposed copy read contiguously)
    auto forward = [&]() {
        for (int nn = lane; nn < n; nn += 64) {
            double wr = 0.0, wi = 0.0;
            int m = 0;
            for (; m + 8 <= l; m += 8) {
                float2 av[8];
                double2 dv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    av[u] = a.At[(size_t)(m + u) * n + nn];
                    dv[u] = D[m + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    wr += (double)av[u].x * dv[u].x - (double)av[u].y * dv[u].y;
                    wi += (double)av[u].x * dv[u].y + (double)av[u].y * dv[u].x;
                }
            }
            for (; m < l; ++m) {
                const float2 av = a.At[(size_t)m * n + nn];
                const double2 dv = D[m];
                wr += (double)av.x * dv.x - (double)av.y * dv.y;
                wi += (double)av.x * dv.y + (double)av.y * dv.x;
            }
            sw[nn] = make_double2(wr, wi);
        }
        __syncthreads();
    };
    // G = 2 A^H sr for the lane's bins (rows in order, four loads in flight)
    auto adjoint = [&]() {
        for (int m = lane; m < lp; m += 64) {
            double gr = 0.0, gi = 0.0;
            for (int n0 = 0; n0 < n; n0 += 4) {
                double2 rv[4];
                float2 av[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    rv[u] = n0 + u < n ? sr[n0 + u] : make_double2(0.0, 0.0);
                    av[u] = n0 + u < n ? a.A[(size_t)(n0 + u) * lp + m] : make_float2(0.0f, 0.0f);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    gr += (double)av[u].x * rv[u].x + (double)av[u].y * rv[u].y;  // conj(a) r
                    gi += (double)av[u].x * rv[u].y - (double)av[u].y * rv[u].x;
                }
            }
            G[m] = make_double2(2.0 * gr, 2.0 * gi);
        }
        __syncthreads();
    };
    auto kkt_of = [&](double lam) {
        const double tau = lam * inv_lf, tau2 = tau * tau;
        double km = 0.0;
        for (int m = lane; m < lp; m += 64) {
            const double2 x = X[m], g = G[m];
            const double vr = x.x - g.x * inv_lf, vi = x.y - g.y * inv_lf;
            const double m2 = vr * vr + vi * vi;
            double er = x.x, ei = x.y;
            if (m2 > tau2) {
                const double sc = 1.0 - tau / sqrt(m2);
                er = x.x - vr * sc;
                ei = x.y - vi * sc;
            }
            km = fmax(km, er * er + ei * ei);
        }
        return lf * sqrt(wmax(km)) / lam;
    };

    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(a.next, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= count) break;
        const int64_t p = a.list[item];
        const float lam_f = a.lambda[p * a.lambda_stride];
        if (!(lam_f > 0.0f) || !isfinite(lam_f)) continue;
        const double lam = lam_f;
        float2 *xo = a.X + (size_t)p * l;
        const float2 *b = a.B + (size_t)p * n;
        double l1 = 0.0;
        for (int m = lane; m < lp; m += 64) {
            const float2 v = m < l ? xo[m] : make_float2(0.0f, 0.0f);
            const double2 x = make_double2(v.x, v.y);
            X[m] = x;
            XP[m] = x;
            D[m] = x;
            l1 += sqrt(x.x * x.x + x.y * x.y);
        }
        __syncthreads();
        // Init from x^(0): r_1 = A x^(0) - b, F(x^(0)), G_1; x^(0) doubles as x^{k-1}
        forward();
        double rr = 0.0;
        for (int nn = lane; nn < n; nn += 64) {
            const float2 bb = b[nn];
            const double2 w = sw[nn];
            const double2 r = make_double2(w.x - bb.x, w.y - bb.y);
            sr[nn] = r;
            srp[nn] = r;
            rr += r.x * r.x + r.y * r.y;
        }
        __syncthreads();
        double F = wsum(rr) + lam * wsum(l1);
        const double F0 = F;
        adjoint();
        fl += 2 * prod;
        for (int m = lane; m < lp; m += 64) GP[m] = G[m];
        __syncthreads();
        double alpha = a.backtracking ? fmax(alpha0, afloor) : afloor;
        bool done = kkt_of(lam) <= (double)a.tol;
        int k = 1;
        for (; k <= a.budget && !done; ++k) {
            const double beta = fmax(0.0, (double)(k - 2) / (double)(k + 1));
            for (int nn = lane; nn < n; nn += 64) {
                const double2 r = sr[nn], rp = srp[nn];
                sry[nn] = make_double2(r.x + beta * (r.x - rp.x), r.y + beta * (r.y - rp.y));
            }
            double d2, w2, l1b;
            for (;;) {
                // x-bar = S_{alpha lambda}(y - alpha G(y)) (Eqs. (10), (12)); d = x-bar - y
                const double tau = alpha * lam;
                d2 = 0.0;
                l1b = 0.0;
                for (int m = lane; m < lp; m += 64) {
                    const double2 x = X[m], xp = XP[m], g = G[m], gp = GP[m];
                    const double yr = x.x + beta * (x.x - xp.x), yi = x.y + beta * (x.y - xp.y);
                    const double gyr = g.x + beta * (g.x - gp.x), gyi = g.y + beta * (g.y - gp.y);
                    const double vr = yr - alpha * gyr, vi = yi - alpha * gyi;
                    const double mv = sqrt(vr * vr + vi * vi);
                    const double sc = mv > tau ? 1.0 - tau / mv : 0.0;
                    const double bxr = m < l ? vr * sc : 0.0, bxi = m < l ? vi * sc : 0.0;
                    XB[m] = make_double2(bxr, bxi);
                    const double dr = bxr - (m < l ? yr : 0.0), di = bxi - (m < l ? yi : 0.0);
                    D[m] = make_double2(dr, di);
                    d2 += dr * dr + di * di;
                    l1b += mv > tau && m < l ? mv - tau : 0.0;
                }
                __syncthreads();
                forward();
                fl += prod;
                double ww = 0.0;
                for (int nn = lane; nn < n; nn += 64) ww += sw[nn].x * sw[nn].x + sw[nn].y * sw[nn].y;
                w2 = wsum(ww);
                d2 = wsum(d2);
                // Eq. (15) in the form ||A d||^2 <= ||d||^2 / (2 alpha); it holds at 1/L_f
                if (!a.backtracking || w2 <= d2 / (2.0 * alpha) || alpha <= afloor) break;
                alpha = fmax((double)a.c_alpha * alpha, afloor);
                __syncthreads();
            }
            l1b = wsum(l1b);
            // r-bar = r(y) + A d, F(x-bar)
            double fb = 0.0;
            for (int nn = lane; nn < n; nn += 64) {
                const double2 ry = sry[nn], w = sw[nn];
                const double2 rb = make_double2(ry.x + w.x, ry.y + w.y);
                sw[nn] = rb;
                fb += rb.x * rb.x + rb.y * rb.y;
            }
            const double Fb = wsum(fb) + lam * l1b;
            const bool acc = !a.monotone || Fb <= F;  // monotone accept (ties accept)
            // x^{k-1} <- x^k (G, r alike), then x^{k+1} = x-bar on acceptance, else x^k
            for (int m = lane; m < lp; m += 64) {
                const double2 x = X[m];
                XP[m] = x;
                GP[m] = G[m];
                if (acc) X[m] = XB[m];
            }
            for (int nn = lane; nn < n; nn += 64) {
                srp[nn] = sr[nn];
                if (acc) sr[nn] = sw[nn];
            }
            __syncthreads();
            if (acc) {
                F = Fb;
                adjoint();
                fl += prod;
            }
            done = kkt_of(lam) <= (double)a.tol;
        }
        // the result replaces the refinement's point only where it improved on it
        if (F < F0) {
            for (int m = lane; m < l; m += 64) {
                const double2 x = X[m];
                xo[m] = make_float2((float)x.x, (float)x.y);
            }
        }
        if (lane == 0 && a.iters) a.iters[p] += k - 1;
        __syncthreads();
    }
    if (lane == 0 && fl) atomicAdd(&a.work[2], fl);
}

// Stacks beyond kContMaxL bins of a table: workgroup g uses slot g of the stack's
// continuation region (cont_groups_for(p) slots; the workgroups beyond leave the
// stack to the others).
__global__ void __launch_bounds__(64) continue_kernel_g(const StackTable t)
{
    for (int i = 0; i < t.count; ++i) {
        const StackDesc &d = t.d[i];
        if (d.p <= 0 || lpad_for(d.l) <= kContMaxL) continue;
        if ((int64_t)blockIdx.x >= cont_groups_for(d.p)) continue;
        const ContinueArgs a = continue_args_for(d, t.o);
        const StackWorkspace lay = stack_workspace_layout(d.n, d.l, d.p);
        double2 *slot = reinterpret_cast<double2 *>(d.ws + lay.cstate) +
                        (size_t)blockIdx.x * (cont_slot_bytes(a.l_pad) / sizeof(double2));
        continue_stack_g(a, slot);
        __syncthreads();
    }
}

template <int NC>
__global__ void __launch_bounds__(64) continue_kernel(const StackTable t)
{
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0 || lpad_for(t.d[i].l) > kContMaxL) continue;
        const ContinueArgs a = continue_args_for(t.d[i], t.o);
        continue_stack<NC>(a);
        __syncthreads();
    }
}

template <int NC>
static hipError_t launch_continue_nc(const StackTable &t, size_t lds, int64_t want, hipStream_t s)
{
    auto kern = continue_kernel<NC>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t g = (int64_t)(per_cu > 0 ? per_cu : 1) * cus;
    if (g > want) g = want;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(64), lds, s, t);
    return hipGetLastError();
}

// One launch over the table's stacks of up to kContMaxL bins (lanes hold up to 4,
// 8 or 16 chunks of 64 bins), one over those beyond (the slot form); workgroups
// find the listed pixels through each stack's counter.
hipError_t launch_continue_table(const StackTable &t, hipStream_t s)
{
    if (!t.o.cont) return hipSuccess;
    size_t lds = 0, lds_g = 0;
    int lpmax = 0;
    int64_t want = 0, want_g = 0;
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        const int lp = lpad_for(t.d[i].l);
        if (lp > kContMaxL) {
            lds_g = std::max(lds_g, (size_t)4 * t.d[i].n * sizeof(double2));
            want_g = std::max<int64_t>(want_g, cont_groups_for(t.d[i].p));
            continue;
        }
        lds = std::max(lds, continue_lds(t.d[i].n, lp));
        lpmax = std::max(lpmax, lp);
        want = std::max<int64_t>(want, t.d[i].p);
    }
    hipError_t e = hipSuccess;
    if (want > 0) {
        if (lpmax <= 256) e = launch_continue_nc<4>(t, lds, want, s);
        else if (lpmax <= 512) e = launch_continue_nc<8>(t, lds, want, s);
        else e = launch_continue_nc<16>(t, lds, want, s);
    }
    if (e != hipSuccess || want_g == 0) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, continue_kernel_g, 64, lds_g);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t g = (int64_t)(per_cu > 0 ? per_cu : 1) * cus;
    if (g > want_g) g = want_g;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(continue_kernel_g, dim3((unsigned)g), dim3(64), lds_g, s, t);
    return hipGetLastError();
}

}  // namespace l1ls
