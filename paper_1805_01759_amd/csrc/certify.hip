// FP64 evaluation of the optimality conditions of Eq. (1) at the returned
// x of every pixel (arXiv 1805.01759): residual r = A x - b, gradient
// g = 2 A^H r, natural KKT residual
//     KKT(x) = L_f max_l |x_l - S_{lambda/L_f}(x_l - g_l/L_f)| / lambda,
// objective F = ||r||^2 + lambda ||x||_1 and the number of nonzeros.  One
// 64-lane workgroup per pixel; x is staged in LDS with a list of its nonzero
// bins (A x runs over those only), the columns of A are read two bins and eight
// rows at a time, and the wave reductions are DPP based.
#include "l1ls_internal.h"
#include "wave_reduce.h"

namespace l1ls {

__device__ __forceinline__ void certify_pixel(const CertifyArgs &a, int64_t p, float2 *sx, double2 *sr,
                                              int16_t *snz)
{
    const int lane = threadIdx.x;
    const int n = a.n, l = a.l, ld = a.l_pad;
    const double lf = a.consts->lf, inv_lf = 1.0 / lf;
    const float lam_f = a.lambda[p * a.lambda_stride];
    const bool bad = !(lam_f > 0.0f) || !isfinite(lam_f);
    const double lam = bad ? 1.0 : (double)lam_f;
    const float2 *x = a.X + (size_t)p * l;
    // stage x and list its nonzero bins (ballot per 64 bins)
    int nnz = 0;
    bool finite = true;
    for (int m0 = 0; m0 < l; m0 += 64) {
        const int m = m0 + lane;
        const float2 xv = m < l ? x[m] : make_float2(0.0f, 0.0f);
        sx[m] = xv;
        finite = finite && isfinite(xv.x) && isfinite(xv.y);
        const bool nz = xv.x != 0.0f || xv.y != 0.0f;
        const uint64_t bal = __ballot(nz);
        if (nz) snz[nnz + __popcll(bal & ((1ull << lane) - 1ull))] = (int16_t)m;
        nnz += __popcll(bal);
    }
    __syncthreads();
    // r = A x - b over the nonzero bins (lanes over n)
    const float2 *b = a.B + (size_t)p * n;
    for (int nn = lane; nn < n; nn += 64) {
        double ar = 0.0, ai = 0.0;
        const float2 *Arow = a.A + (size_t)nn * ld;
        for (int q = 0; q < nnz; ++q) {
            const int m = snz[q];
            const float2 xv = sx[m], av = Arow[m];
            ar += (double)av.x * xv.x - (double)av.y * xv.y;
            ai += (double)av.x * xv.y + (double)av.y * xv.x;
        }
        const float2 bv = b[nn];
        sr[nn] = make_double2(ar - (double)bv.x, ai - (double)bv.y);
    }
    __syncthreads();
    double acc = 0.0;  // ||r||^2 + lambda ||x||_1
    for (int nn = lane; nn < n; nn += 64) acc += sr[nn].x * sr[nn].x + sr[nn].y * sr[nn].y;
    for (int q = lane; q < nnz; q += 64) {
        const float2 xv = sx[snz[q]];
        acc += lam * sqrt((double)xv.x * xv.x + (double)xv.y * xv.y);
    }
    // g_m = 2 sum_n conj(A_nm) r_n for the lane's bins m = lane + 64 c, two at a
    // time with eight rows of loads in flight; magnitudes compared squared
    const double tau = lam * inv_lf, tau2 = tau * tau;
    double kmax = 0.0;
    const int nb = (l + 63) / 64;
    for (int c0 = 0; c0 < nb; c0 += 2) {
        const int m0 = lane + 64 * c0, m1 = m0 + 64;
        const int q0 = m0 < l ? m0 : 0, q1 = m1 < l ? m1 : 0;
        double gr0 = 0.0, gi0 = 0.0, gr1 = 0.0, gi1 = 0.0;
        int nn = 0;
        for (; nn + 8 <= n; nn += 8) {
            float2 a0[8], a1[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                a0[u] = a.A[(unsigned)((nn + u) * ld + q0)];
                a1[u] = a.A[(unsigned)((nn + u) * ld + q1)];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double2 rv = sr[nn + u];
                gr0 += a0[u].x * rv.x + a0[u].y * rv.y;
                gi0 += a0[u].x * rv.y - a0[u].y * rv.x;
                gr1 += a1[u].x * rv.x + a1[u].y * rv.y;
                gi1 += a1[u].x * rv.y - a1[u].y * rv.x;
            }
        }
        for (; nn < n; ++nn) {
            const double2 rv = sr[nn];
            const float2 a0 = a.A[(unsigned)(nn * ld + q0)], a1 = a.A[(unsigned)(nn * ld + q1)];
            gr0 += a0.x * rv.x + a0.y * rv.y;
            gi0 += a0.x * rv.y - a0.y * rv.x;
            gr1 += a1.x * rv.x + a1.y * rv.y;
            gi1 += a1.x * rv.y - a1.y * rv.x;
        }
        const double grs[2] = {gr0, gr1}, gis[2] = {gi0, gi1};
        const int ms[2] = {m0, m1};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (ms[k] >= l || c0 + k >= nb) continue;
            const double gr = 2.0 * grs[k], gi = 2.0 * gis[k];
            const double xr = sx[ms[k]].x, xi = sx[ms[k]].y;
            const double vr = xr - gr * inv_lf, vi = xi - gi * inv_lf;
            const double m2 = vr * vr + vi * vi;
            double er = xr, ei = xi;  // x - prox(v), prox(v) = 0 when |v| <= tau
            if (m2 > tau2) {
                const double sc = 1.0 - tau / sqrt(m2);
                er = xr - vr * sc;
                ei = xi - vi * sc;
            }
            kmax = fmax(kmax, er * er + ei * ei);
            finite = finite && isfinite(gr) && isfinite(gi);
        }
    }
    const double F = wr::wsum(acc);
    kmax = sqrt(wr::wmax(kmax));
    const bool all_finite = __ballot(!finite) == 0 && isfinite(F);
    if (lane == 0) {
        const double kkt = lf * kmax / lam;
        uint32_t st = a.status_in ? a.status_in[p] : 0u;
        if (!all_finite) st |= L1LS_PX_NONFINITE;
        if (bad) st |= L1LS_PX_BAD_LAMBDA;
        if (all_finite && !bad && kkt <= (double)a.tol) st |= L1LS_PX_CONVERGED;
        if (nnz == 0) st |= L1LS_PX_ZERO;
        if (a.status) a.status[p] = st;
        if (a.kkt) a.kkt[p] = bad ? 0.0f : (float)kkt;
        if (a.objective) a.objective[p] = (float)F;
        if (a.nnz) a.nnz[p] = (int32_t)nnz;
        if (a.iters) a.iters[p] = a.iters_in ? a.iters_in[p] : 0;
    }
}

// LDS of a workgroup for a table: x and its nonzero list (l_pad entries each)
// and r (n entries), sized for the largest stack of the table.
__host__ __device__ inline size_t certify_lds(int lp, int nm)
{
    return (size_t)lp * sizeof(float2) + (size_t)nm * sizeof(double2) + (size_t)lp * sizeof(int16_t);
}

// One workgroup a pixel for up to 2^25 pixels a stack, grid-stride beyond (the
// grid stays within the dispatch limits at any pixel count); stacks in table order.
__global__ void __launch_bounds__(64) certify_kernel(const StackTable t)
{
    extern __shared__ __align__(16) unsigned char cdyn[];
    int lp = 64, nm = 1;
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        lp = lp > lpad_for(t.d[i].l) ? lp : lpad_for(t.d[i].l);
        nm = nm > t.d[i].n ? nm : t.d[i].n;
    }
    float2 *sx = reinterpret_cast<float2 *>(cdyn);
    double2 *sr = reinterpret_cast<double2 *>(cdyn + (size_t)lp * sizeof(float2));
    int16_t *snz = reinterpret_cast<int16_t *>(cdyn + (size_t)lp * sizeof(float2) + (size_t)nm * sizeof(double2));
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        const CertifyArgs a = certify_args_for(t.d[i], t.o);
        for (int64_t p = blockIdx.x; p < a.p; p += gridDim.x) {
            certify_pixel(a, p, sx, sr, snz);
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
    if (g > ((int64_t)1 << 25)) g = (int64_t)1 << 25;
    hipLaunchKernelGGL(certify_kernel, dim3((unsigned)g), dim3(64), certify_lds(lp, nm), s, t);
    return hipGetLastError();
}

}  // namespace l1ls
