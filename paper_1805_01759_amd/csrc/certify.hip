// FP64 evaluation of the optimality conditions of Eq. (1) at the returned
// x of every pixel (arXiv 1805.01759): residual r = A x - b, gradient
// g = 2 A^H r, natural KKT residual
//     KKT(x) = L_f max_l |x_l - S_{lambda/L_f}(x_l - g_l/L_f)| / lambda,
// objective F = ||r||^2 + lambda ||x||_1 and the number of nonzeros.  One
// 64-lane workgroup per pixel; x is staged in LDS and its zero entries are
// skipped (uniform branch) in A x.
#include "l1ls_internal.h"

namespace l1ls {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ void cprox64(double vr, double vi, double tau, double &o_r, double &o_i)
{
    const double m = sqrt(vr * vr + vi * vi);
    if (m > tau) {
        const double s = 1.0 - tau / m;
        o_r = vr * s;
        o_i = vi * s;
    } else {
        o_r = 0.0;
        o_i = 0.0;
    }
}

__global__ void __launch_bounds__(64) certify_kernel(const CertifyArgs a)
{
    __shared__ float2 sx[64 * kMaxWaves];
    __shared__ double2 sr[kMaxN];
    const int lane = threadIdx.x;
    const int64_t p = blockIdx.x;
    if (p >= a.p) return;
    const int n = a.n, l = a.l, ld = a.l_pad;
    const double lf = a.consts->lf;
    const float lam_f = a.lambda[p * a.lambda_stride];
    const bool bad = !(lam_f > 0.0f) || !isfinite(lam_f);
    const double lam = bad ? 1.0 : (double)lam_f;
    const float2 *x = a.X + (size_t)p * l;
    for (int m = lane; m < a.l_pad; m += 64) sx[m] = m < l ? x[m] : make_float2(0.0f, 0.0f);
    __syncthreads();
    // r = A x - b (lanes over n)
    const float2 *b = a.B + (size_t)p * n;
    for (int nn = lane; nn < n; nn += 64) {
        double ar = 0.0, ai = 0.0;
        const float2 *Arow = a.A + (size_t)nn * ld;
        for (int m = 0; m < l; ++m) {
            const float2 xv = sx[m];
            if (xv.x != 0.0f || xv.y != 0.0f) {
                const float2 av = Arow[m];
                ar += (double)av.x * xv.x - (double)av.y * xv.y;
                ai += (double)av.x * xv.y + (double)av.y * xv.x;
            }
        }
        const float2 bv = b[nn];
        sr[nn] = make_double2(ar - (double)bv.x, ai - (double)bv.y);
    }
    __syncthreads();
    double rr = 0.0;
    for (int nn = lane; nn < n; nn += 64) rr += sr[nn].x * sr[nn].x + sr[nn].y * sr[nn].y;
    // g_m = 2 sum_n conj(A_nm) r_n (lanes over m)
    double kmax = 0.0, l1 = 0.0, nz = 0.0;
    bool finite = true;
    for (int m = lane; m < l; m += 64) {
        double gr = 0.0, gi = 0.0;
        for (int nn = 0; nn < n; ++nn) {
            const float2 av = a.A[(size_t)nn * ld + m];
            const double2 rv = sr[nn];
            gr += (double)av.x * rv.x + (double)av.y * rv.y;
            gi += (double)av.x * rv.y - (double)av.y * rv.x;
        }
        gr *= 2.0;
        gi *= 2.0;
        const double xr = sx[m].x, xi = sx[m].y;
        double pr, pi;
        cprox64(xr - gr / lf, xi - gi / lf, lam / lf, pr, pi);
        const double er = xr - pr, ei = xi - pi;
        kmax = fmax(kmax, sqrt(er * er + ei * ei));
        l1 += sqrt(xr * xr + xi * xi);
        nz += (xr != 0.0 || xi != 0.0) ? 1.0 : 0.0;
        finite = finite && isfinite(gr) && isfinite(gi) && isfinite(xr) && isfinite(xi);
    }
    rr = wave_sum(rr);
    kmax = wave_max(kmax);
    l1 = wave_sum(l1);
    nz = wave_sum(nz);
    const bool all_finite = __ballot(!finite) == 0 && isfinite(rr);
    if (lane == 0) {
        const double kkt = lf * kmax / lam;
        uint32_t st = a.status_in ? a.status_in[p] : 0u;
        if (!all_finite) st |= L1LS_PX_NONFINITE;
        if (bad) st |= L1LS_PX_BAD_LAMBDA;
        if (all_finite && !bad && kkt <= (double)a.tol) st |= L1LS_PX_CONVERGED;
        if (nz == 0.0) st |= L1LS_PX_ZERO;
        if (a.status) a.status[p] = st;
        if (a.kkt) a.kkt[p] = bad ? 0.0f : (float)kkt;
        if (a.objective) a.objective[p] = (float)(rr + lam * l1);
        if (a.nnz) a.nnz[p] = (int32_t)nz;
        if (a.iters) a.iters[p] = a.iters_in ? a.iters_in[p] : 0;
    }
}

hipError_t launch_certify(const CertifyArgs &a, hipStream_t s)
{
    if (a.p <= 0) return hipSuccess;
    hipLaunchKernelGGL(certify_kernel, dim3((unsigned)a.p), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace l1ls
