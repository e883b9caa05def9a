// FP64 evaluation of the optimality conditions of Eq. (1) at the returned
// x of every pixel (arXiv 1805.01759): residual r = A x - b, gradient
// g = 2 A^H r, natural KKT residual
//     KKT(x) = L_f max_l |x_l - S_{lambda/L_f}(x_l - g_l/L_f)| / lambda,
// objective F = ||r||^2 + lambda ||x||_1 and the number of nonzeros.  One
// 64-lane workgroup per tile of four pixels; each pixel's nonzero bins are
// listed in LDS (A x runs over those only), the columns of A are read two bins
// and eight rows at a time and serve the four residuals, and the wave
// reductions are DPP based.
#include "l1ls_internal.h"
#include "wave_reduce.h"

namespace l1ls {

// Pixels certified together by one 64-lane workgroup: every column of A read for
// the gradient serves all of them (one pixel a workgroup re-read A from L2 for
// each pixel, 205 KB a close pair).
constexpr int kCertPix = 4;

__device__ __forceinline__ void certify_tile(const CertifyArgs &a, int64_t p0, double2 *sr, int16_t *snz, int lp,
                                             int nm)
{
    const int lane = threadIdx.x;
    const int n = a.n, l = a.l, ld = a.l_pad;
    const double lf = a.consts->lf, inv_lf = 1.0 / lf;
    constexpr int PT = kCertPix;
    int nnz[PT];
    bool finite[PT], bad[PT], valid[PT];
    double lam[PT];
    const float2 *xs[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const int64_t p = p0 + k;
        valid[k] = p < a.p;
        const float lam_f = valid[k] ? a.lambda[p * a.lambda_stride] : 1.0f;
        bad[k] = !(lam_f > 0.0f) || !isfinite(lam_f);
        lam[k] = bad[k] ? 1.0 : (double)lam_f;
        xs[k] = a.X + (size_t)(valid[k] ? p : 0) * l;
        // list the nonzero bins of x (ballot per 64 bins)
        nnz[k] = 0;
        finite[k] = true;
        if (!valid[k]) continue;
        for (int m0 = 0; m0 < l; m0 += 64) {
            const int m = m0 + lane;
            const float2 xv = m < l ? xs[k][m] : make_float2(0.0f, 0.0f);
            finite[k] = finite[k] && isfinite(xv.x) && isfinite(xv.y);
            const bool nz = xv.x != 0.0f || xv.y != 0.0f;
            const uint64_t bal = __ballot(nz);
            if (nz) snz[k * lp + nnz[k] + __popcll(bal & ((1ull << lane) - 1ull))] = (int16_t)m;
            nnz[k] += __popcll(bal);
        }
    }
    __syncthreads();
    // r = A x - b over the nonzero bins (lanes over n); 0 for a pixel past the end
    double acc[PT];  // ||r||^2 + lambda ||x||_1
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        acc[k] = 0.0;
        const float2 *b = a.B + (size_t)(valid[k] ? p0 + k : 0) * n;
        for (int nn = lane; nn < n; nn += 64) {
            double ar = 0.0, ai = 0.0;
            const float2 *Arow = a.A + (size_t)nn * ld;
            for (int q = 0; q < nnz[k]; ++q) {
                const int m = snz[k * lp + q];
                const float2 xv = xs[k][m], av = Arow[m];
                ar += (double)av.x * xv.x - (double)av.y * xv.y;
                ai += (double)av.x * xv.y + (double)av.y * xv.x;
            }
            const float2 bv = valid[k] ? b[nn] : make_float2(0.0f, 0.0f);
            const double2 rv = make_double2(ar - (double)bv.x, ai - (double)bv.y);
            sr[k * nm + nn] = rv;
            acc[k] += rv.x * rv.x + rv.y * rv.y;
        }
        for (int q = lane; q < nnz[k]; q += 64) {
            const float2 xv = xs[k][snz[k * lp + q]];
            acc[k] += lam[k] * sqrt((double)xv.x * xv.x + (double)xv.y * xv.y);
        }
    }
    __syncthreads();
    // g_m = 2 sum_n conj(A_nm) r_n for the lane's bins m = lane + 64 c, two at a
    // time with eight rows of loads in flight, for every pixel of the tile;
    // magnitudes compared squared
    double kmax[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) kmax[k] = 0.0;
    const int nb = (l + 63) / 64;
    for (int c0 = 0; c0 < nb; c0 += 2) {
        const int m0 = lane + 64 * c0, m1 = m0 + 64;
        const int q0 = m0 < l ? m0 : 0, q1 = m1 < l ? m1 : 0;
        double gr0[PT], gi0[PT], gr1[PT], gi1[PT];
#pragma unroll
        for (int k = 0; k < PT; ++k) gr0[k] = gi0[k] = gr1[k] = gi1[k] = 0.0;
        int nn = 0;
        for (; nn + 2 <= n; nn += 2) {
            float2 a0[2], a1[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                a0[u] = a.A[(unsigned)((nn + u) * ld + q0)];
                a1[u] = a.A[(unsigned)((nn + u) * ld + q1)];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int k = 0; k < PT; ++k) {
                    const double2 rv = sr[k * nm + nn + u];
                    gr0[k] += a0[u].x * rv.x + a0[u].y * rv.y;
                    gi0[k] += a0[u].x * rv.y - a0[u].y * rv.x;
                    gr1[k] += a1[u].x * rv.x + a1[u].y * rv.y;
                    gi1[k] += a1[u].x * rv.y - a1[u].y * rv.x;
                }
        }
        for (; nn < n; ++nn) {
            const float2 a0 = a.A[(unsigned)(nn * ld + q0)], a1 = a.A[(unsigned)(nn * ld + q1)];
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                const double2 rv = sr[k * nm + nn];
                gr0[k] += a0.x * rv.x + a0.y * rv.y;
                gi0[k] += a0.x * rv.y - a0.y * rv.x;
                gr1[k] += a1.x * rv.x + a1.y * rv.y;
                gi1[k] += a1.x * rv.y - a1.y * rv.x;
            }
        }
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const double tau = lam[k] * inv_lf, tau2 = tau * tau;
            const double grs[2] = {gr0[k], gr1[k]}, gis[2] = {gi0[k], gi1[k]};
            const int ms[2] = {m0, m1};
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (ms[e] >= l || c0 + e >= nb) continue;
                const double gr = 2.0 * grs[e], gi = 2.0 * gis[e];
                const float2 xv = xs[k][ms[e]];
                const double xr = xv.x, xi = xv.y;
                const double vr = xr - gr * inv_lf, vi = xi - gi * inv_lf;
                const double m2 = vr * vr + vi * vi;
                double er = xr, ei = xi;  // x - prox(v), prox(v) = 0 when |v| <= tau
                if (m2 > tau2) {
                    const double sc = 1.0 - tau / sqrt(m2);
                    er = xr - vr * sc;
                    ei = xi - vi * sc;
                }
                kmax[k] = fmax(kmax[k], er * er + ei * ei);
                finite[k] = finite[k] && isfinite(gr) && isfinite(gi);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        if (!valid[k]) continue;
        const int64_t p = p0 + k;
        const double F = wr::wsum(acc[k]);
        const double km = sqrt(wr::wmax(kmax[k]));
        const bool all_finite = __ballot(!finite[k]) == 0 && isfinite(F);
        if (lane == 0) {
            const double kkt = lf * km / lam[k];
            uint32_t st = a.status_in ? a.status_in[p] : 0u;
            if (!all_finite) st |= L1LS_PX_NONFINITE;
            if (bad[k]) st |= L1LS_PX_BAD_LAMBDA;
            if (all_finite && !bad[k] && kkt <= (double)a.tol) st |= L1LS_PX_CONVERGED;
            if (nnz[k] == 0) st |= L1LS_PX_ZERO;
            if (a.status) a.status[p] = st;
            if (a.kkt) a.kkt[p] = bad[k] ? 0.0f : (float)kkt;
            if (a.objective) a.objective[p] = (float)F;
            if (a.nnz) a.nnz[p] = (int32_t)nnz[k];
            if (a.iters) a.iters[p] = a.iters_in ? a.iters_in[p] : 0;
        }
    }
}

// LDS of a workgroup for a table: the nonzero lists (l_pad entries) and the
// residuals (n entries) of kCertPix pixels, sized for the largest stack.
__host__ __device__ inline size_t certify_lds(int lp, int nm)
{
    return (size_t)kCertPix * ((size_t)nm * sizeof(double2) + (size_t)lp * sizeof(int16_t));
}

// One workgroup a tile of kCertPix pixels for up to 2^25 tiles a stack,
// grid-stride beyond (the grid stays within the dispatch limits at any pixel
// count); stacks in table order.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) certify_kernel(const StackTable t)
{
    extern __shared__ __align__(16) unsigned char cdyn[];
    int lp = 64, nm = 1;
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        lp = lp > lpad_for(t.d[i].l) ? lp : lpad_for(t.d[i].l);
        nm = nm > t.d[i].n ? nm : t.d[i].n;
    }
    double2 *sr = reinterpret_cast<double2 *>(cdyn);
    int16_t *snz = reinterpret_cast<int16_t *>(cdyn + (size_t)kCertPix * nm * sizeof(double2));
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        const CertifyArgs a = certify_args_for(t.d[i], t.o);
        const int64_t tiles = (a.p + kCertPix - 1) / kCertPix;
        for (int64_t tt = blockIdx.x; tt < tiles; tt += gridDim.x) {
            certify_tile(a, tt * kCertPix, sr, snz, lp, nm);
            __syncthreads();
        }
    }
}

hipError_t launch_certify_table(const StackTable &t, hipStream_t s)
{
    int64_t g = 0;
    int lp = 64, nm = 1;
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        g = t.d[i].p > g ? t.d[i].p : g;
        lp = lp > lpad_for(t.d[i].l) ? lp : lpad_for(t.d[i].l);
        nm = nm > t.d[i].n ? nm : t.d[i].n;
    }
    if (g == 0) return hipSuccess;
    g = (g + kCertPix - 1) / kCertPix;
    if (g > ((int64_t)1 << 25)) g = (int64_t)1 << 25;
    hipLaunchKernelGGL(certify_kernel, dim3((unsigned)g), dim3(64), certify_lds(lp, nm), s, t);
    return hipGetLastError();
}

}  // namespace l1ls
