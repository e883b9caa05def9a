// Algorithm 1 with J > 1 column blocks (randomized block prox-gradient,
// Eqs. (13)-(14) of arXiv 1805.01759) for the complex L1LS problem.
//
// Blocks: J contiguous groups of w = ceil(L/J) bins.  Iteration k updates the
// block i_k that the caller's uniform draw u_k selects with P_i = L_i / sum L,
// L_i = 2 lambda_max(A_i A_i^H) (the draws are shared by the pixels of a stack:
// pixel-local iteration k uses u_k).  Per block the pixel keeps its update
// count c (extrapolation weight max(0, (c-2)/(c+1))), its value before its last
// update, its own step (start 1/(2 max_{l in i} ||a_l||^2), shrunk by C_alpha
// while Eq. (15) fails on the block, floor 1/L_i), and the residual change of
// its last update Dr_i = A_i (x_i - x_i^prev), so that the residual at the
// extrapolated point is r + beta Dr_i without a product.  Per iteration:
//   g_i = 2 A_i^H r(y)                   (adjoint on the block)
//   x-bar_i = S_{alpha lambda}(y_i - alpha g_i),  d = x-bar_i - y_i,  w = A_i d
//   Eq. (15) on the block:  ||w||^2 <= ||d||^2 / (2 alpha)
//   accept iff F(x-bar) - F(x^k) = ||r(y) + w||^2 - ||r||^2 + lambda (||x-bar_i||_1 - ||x_i||_1) <= 0
// so a block update costs two products over N x w.  At a block's first update
// y_i = 0 and x-bar_i is linear in alpha: the shrink sequence is resolved from
// one product, as for one block.  The KKT residual (a full adjoint) is tested
// every J iterations.  One wave per pixel, pixels from the stack's queue; the
// pixel's x, x^prev, block scratch and residuals live in LDS.
#include "l1ls_internal.h"

namespace l1ls {

__device__ __forceinline__ float bsum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float bmax(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

#define BLOCK_WAVE_SYNC()                    \
    do {                                     \
        __builtin_amdgcn_wave_barrier();     \
        __builtin_amdgcn_s_waitcnt(0);       \
        __builtin_amdgcn_wave_barrier();     \
    } while (0)

__host__ __device__ inline int block_width(int l, int J) { return (l + J - 1) / J; }

size_t fista_blocks_lds(int n, int l_pad, int J)
{
    const int w = block_width(l_pad, J);
    return (size_t)(2 * l_pad + 3 * w + 2 * n + (size_t)J * n) * sizeof(float2) + (size_t)J * 2 * sizeof(float);
}

// Per-block constants: one workgroup per block.  L_i = 2 lambda_max(A_i A_i^H)
// by FP64 power iteration on v -> A_i (A_i^H v), alpha0_i = 1/(2 max ||a_l||^2).
__global__ void __launch_bounds__(256) setup_blocks_kernel(int n, int l, int J, const float2 *A,
                                                           BlockConsts *bc)
{
    __shared__ double red[3][256];
    __shared__ double2 v[kMaxN];
    __shared__ double2 t[1024];
    const int tid = threadIdx.x, bd = blockDim.x;
    const int jb = blockIdx.x;
    const int w = block_width(l, J);
    const int m0 = jb * w < l ? jb * w : l;
    const int m1 = (jb + 1) * w < l ? (jb + 1) * w : l;
    const int wb = m1 - m0;
    double cm = 0.0;
    for (int c = m0 + tid; c < m1; c += bd) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) {
            const float2 q = A[(size_t)r * l + c];
            s += (double)q.x * q.x + (double)q.y * q.y;
        }
        cm = fmax(cm, s);
    }
    red[0][tid] = cm;
    __syncthreads();
    for (int s = bd / 2; s > 0; s >>= 1) {
        if (tid < s) red[0][tid] = fmax(red[0][tid], red[0][tid + s]);
        __syncthreads();
    }
    const double colmax = red[0][0];
    __syncthreads();
    if (tid < n) v[tid] = make_double2(1.0 + 0.01 * tid, 0.001 * tid);
    __syncthreads();
    double lam_prev = -1.0;
    for (int it = 0; it < 4000 && wb > 0; ++it) {
        // t = A_i^H v (over the block's bins)
        for (int c = tid; c < wb; c += bd) {
            double sr = 0.0, si = 0.0;
            for (int r = 0; r < n; ++r) {
                const float2 q = A[(size_t)r * l + m0 + c];
                const double2 x = v[r];
                sr += q.x * x.x + q.y * x.y;  // conj(a) v
                si += q.x * x.y - q.y * x.x;
            }
            t[c] = make_double2(sr, si);
        }
        __syncthreads();
        // u = A_i t; Rayleigh quotient v^H u / v^H v; v = u / ||u||
        double pr = 0.0, nv = 0.0, nu = 0.0;
        double2 uu = make_double2(0.0, 0.0);
        if (tid < n) {
            double sr = 0.0, si = 0.0;
            for (int c = 0; c < wb; ++c) {
                const float2 q = A[(size_t)tid * l + m0 + c];
                const double2 x = t[c];
                sr += q.x * x.x - q.y * x.y;
                si += q.x * x.y + q.y * x.x;
            }
            uu = make_double2(sr, si);
            pr = v[tid].x * sr + v[tid].y * si;
            nv = v[tid].x * v[tid].x + v[tid].y * v[tid].y;
            nu = sr * sr + si * si;
        }
        red[0][tid] = pr;
        red[1][tid] = nv;
        red[2][tid] = nu;
        __syncthreads();
        for (int s = bd / 2; s > 0; s >>= 1) {
            if (tid < s) {
                red[0][tid] += red[0][tid + s];
                red[1][tid] += red[1][tid + s];
                red[2][tid] += red[2][tid + s];
            }
            __syncthreads();
        }
        const double lam_est = red[0][0] / red[1][0];
        const double inv = red[2][0] > 0.0 ? 1.0 / sqrt(red[2][0]) : 0.0;
        __syncthreads();
        if (tid < n) v[tid] = make_double2(uu.x * inv, uu.y * inv);
        __syncthreads();
        const bool stop = it > 20 && fabs(lam_est - lam_prev) <= 1e-15 * fabs(lam_est);
        lam_prev = lam_est;
        if (stop) break;
    }
    if (tid == 0) {
        const double L = wb > 0 ? 2.0 * lam_prev : 0.0;
        bc[jb].L = L;
        bc[jb].alpha0 = colmax > 0.0 ? 1.0 / (2.0 * colmax) : 1.0;
        bc[jb].afloor = L > 0.0 ? 1.0 / L : bc[jb].alpha0;
        bc[jb].pad = 0.0;
    }
}

__global__ void __launch_bounds__(64) fista_blocks_kernel(const BlocksArgs ba)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const FistaArgs &a = ba.f;
    const int lane = threadIdx.x;
    const int n = a.n, l = a.l, ld = a.l_pad, J = ba.J;
    const int w = block_width(l, J);
    float2 *sx = reinterpret_cast<float2 *>(smem);  // x^k (ld)
    float2 *sxp = sx + ld;                          // each block's value before its last update
    float2 *sy = sxp + ld;                          // y on the block (w)
    float2 *sg = sy + w;                            // g on the block
    float2 *sd = sg + w;                            // d = x-bar - y on the block
    float2 *sr = sd + w;                            // r = A x - b (n)
    float2 *sry = sr + n;                           // r(y)
    float2 *sdr = sry + n;                          // Dr per block (J n)
    float *sal = reinterpret_cast<float *>(sdr + (size_t)J * n);  // step per block (J)
    int *scnt = reinterpret_cast<int *>(sal + J);                  // updates per block (J)

    const double lf_d = a.consts->lf;
    const float lf = (float)lf_d, inv_lf = (float)(1.0 / lf_d);
    double ltot = 0.0;
    for (int j = 0; j < J; ++j) ltot += ba.bc[j].L;
    unsigned long long fl = 0;  // FP32 flops of the products (8 per complex multiply-add)
    const unsigned long long f8n = 8ull * (unsigned long long)n;

    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(a.queue, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= (uint32_t)a.p) break;
        const int64_t pix = item;
        float lam = a.lambda[pix * a.lambda_stride];
        const bool bad = !(lam > 0.0f) || !isfinite(lam);
        if (bad) lam = 1.0f;
        const float2 *Bp = a.B + (size_t)pix * n;
        for (int m = lane; m < ld; m += 64) sx[m] = sxp[m] = make_float2(0.0f, 0.0f);
        float bb = 0.0f;
        if (lane < n) {
            const float2 v = Bp[lane];
            sr[lane] = make_float2(-v.x, -v.y);
            bb = v.x * v.x + v.y * v.y;
        }
        for (int e = lane; e < J * n; e += 64) sdr[e] = make_float2(0.0f, 0.0f);
        for (int j = lane; j < J; j += 64) {
            float a0 = (float)ba.bc[j].alpha0;
            const float fl = (float)ba.bc[j].afloor;
            if (a.backtracking && a0 < fl) a0 = fl;
            sal[j] = a0;
            scnt[j] = 0;
        }
        float Fk = bsum(bb);
        BLOCK_WAVE_SYNC();

        // natural KKT residual of x (full adjoint of r); lanes over bins
        auto kkt_of_x = [&]() -> float {
            const float tk = lam * inv_lf;
            float km = 0.0f;
            for (int m = lane; m < l; m += 64) {
                float gr = 0.0f, gi = 0.0f;
                for (int r = 0; r < n; ++r) {
                    const float2 q = a.A[(size_t)r * ld + m], rv = sr[r];
                    gr = fmaf(q.x, rv.x, fmaf(q.y, rv.y, gr));
                    gi = fmaf(q.x, rv.y, fmaf(-q.y, rv.x, gi));
                }
                const float2 xv = sx[m];
                const float vr = xv.x - 2.0f * gr * inv_lf, vi = xv.y - 2.0f * gi * inv_lf;
                const float mm = sqrtf(vr * vr + vi * vi);
                const float sc = mm > tk ? 1.0f - tk / mm : 0.0f;
                const float er = xv.x - vr * sc, ei = xv.y - vi * sc;
                km = fmaxf(km, er * er + ei * ei);
            }
            return lf * sqrtf(bmax(km)) / lam;
        };

        int k = 0;
        float kkt = kkt_of_x();
        fl += f8n * (unsigned long long)l;
        bool conv = kkt <= a.tol, nonfinite = !isfinite(kkt);
        while (!conv && !nonfinite && !bad && k < a.fista_cap) {
            ++k;
            // the block of this iteration (FP64, the draw against the cumulative L)
            const double uk = ba.u[k - 1] * ltot;
            int ib = J - 1;
            double acc = 0.0;
            for (int j = 0; j < J; ++j) {
                acc += ba.bc[j].L;
                if (uk < acc) { ib = j; break; }
            }
            const int m0 = ib * w < l ? ib * w : l;
            const int m1 = (ib + 1) * w < l ? (ib + 1) * w : l;
            const int wb = m1 - m0;
            const int c = scnt[ib] + 1;
            const float beta = fmaxf(0.0f, (float)(c - 2) / (float)(c + 1));
            float alpha = sal[ib];
            const float afloor = (float)ba.bc[ib].afloor;
            // r(y) = r + beta Dr_i
            if (lane < n) {
                const float2 rv = sr[lane], dv = sdr[(size_t)ib * n + lane];
                sry[lane] = make_float2(fmaf(beta, dv.x, rv.x), fmaf(beta, dv.y, rv.y));
            }
            BLOCK_WAVE_SYNC();
            // y and g = 2 A_i^H r(y) on the block
            for (int mm = lane; mm < wb; mm += 64) {
                const int m = m0 + mm;
                const float2 xv = sx[m], xpv = sxp[m];
                sy[mm] = make_float2(fmaf(beta, xv.x - xpv.x, xv.x), fmaf(beta, xv.y - xpv.y, xv.y));
                float gr = 0.0f, gi = 0.0f;
                for (int r = 0; r < n; ++r) {
                    const float2 q = a.A[(size_t)r * ld + m], rv = sry[r];
                    gr = fmaf(q.x, rv.x, fmaf(q.y, rv.y, gr));
                    gi = fmaf(q.x, rv.y, fmaf(-q.y, rv.x, gi));
                }
                sg[mm] = make_float2(2.0f * gr, 2.0f * gi);
            }
            fl += f8n * (unsigned long long)wb;
            BLOCK_WAVE_SYNC();
            float w2 = 0.0f, d2 = 0.0f, l1d = 0.0f;
            float2 wv = make_float2(0.0f, 0.0f);
            for (int trial = 0; trial < 64; ++trial) {
                const float tau = alpha * lam;
                float d2l = 0.0f, l1l = 0.0f;
                for (int mm = lane; mm < wb; mm += 64) {
                    const float2 yv = sy[mm], gv = sg[mm], xv = sx[m0 + mm];
                    const float vr = fmaf(-alpha, gv.x, yv.x), vi = fmaf(-alpha, gv.y, yv.y);
                    const float mag = sqrtf(vr * vr + vi * vi);
                    const float sc = mag > tau ? 1.0f - tau / mag : 0.0f;
                    const float br = vr * sc, bi = vi * sc;
                    const float dr = br - yv.x, di = bi - yv.y;
                    sd[mm] = make_float2(dr, di);
                    d2l = fmaf(dr, dr, fmaf(di, di, d2l));
                    l1l += (mag > tau ? mag - tau : 0.0f) - sqrtf(xv.x * xv.x + xv.y * xv.y);
                }
                BLOCK_WAVE_SYNC();
                wv = make_float2(0.0f, 0.0f);
                if (lane < n) {
                    for (int mm = 0; mm < wb; ++mm) {
                        const float2 q = a.A[(size_t)lane * ld + m0 + mm], dv = sd[mm];
                        wv.x = fmaf(q.x, dv.x, fmaf(-q.y, dv.y, wv.x));
                        wv.y = fmaf(q.x, dv.y, fmaf(q.y, dv.x, wv.y));
                    }
                }
                fl += f8n * (unsigned long long)wb;
                w2 = bsum(wv.x * wv.x + wv.y * wv.y);
                d2 = bsum(d2l);
                l1d = bsum(l1l);
                bool jumped = false;
                if (c == 1 && a.backtracking && w2 > d2 / (2.0f * alpha) && alpha > afloor) {
                    // the block's first update: y_i = 0, so x-bar_i = alpha S_lambda(-g_i) is
                    // linear in alpha and Eq. (15) reads alpha <= ||d||^2 / (2 ||A d||^2)
                    const float rho = d2 / (2.0f * w2);
                    float an = alpha;
                    while (an > rho && an > afloor) an = fmaxf(a.c_alpha * an, afloor);
                    const float cc = an / alpha;
                    for (int mm = lane; mm < wb; mm += 64) {
                        const float2 dv = sd[mm];
                        sd[mm] = make_float2(dv.x * cc, dv.y * cc);
                    }
                    wv.x *= cc;
                    wv.y *= cc;
                    w2 *= cc * cc;
                    d2 *= cc * cc;
                    l1d *= cc;
                    alpha = an;
                    jumped = true;
                    BLOCK_WAVE_SYNC();
                }
                const bool fail = a.backtracking && !jumped && (w2 > d2 / (2.0f * alpha)) && alpha > afloor;
                if (!fail) break;
                alpha = fmaxf(a.c_alpha * alpha, afloor);
            }
            // monotone acceptance: F(x-bar) - F(x^k) from the residuals and the block's l1 change
            float dfr = 0.0f;
            float2 rb = make_float2(0.0f, 0.0f), rv = make_float2(0.0f, 0.0f);
            if (lane < n) {
                const float2 ry = sry[lane];
                rv = sr[lane];
                rb = make_float2(ry.x + wv.x, ry.y + wv.y);
                dfr = (rb.x - rv.x) * (rb.x + rv.x) + (rb.y - rv.y) * (rb.y + rv.y);
            }
            dfr = bsum(dfr);
            const float dF = fmaf(lam, l1d, dfr);
            const bool accept = !a.monotone || dF <= 0.0f;
            for (int mm = lane; mm < wb; mm += 64) {
                const int m = m0 + mm;
                const float2 xv = sx[m];
                sxp[m] = xv;
                if (accept) {
                    const float2 yv = sy[mm], dv = sd[mm];
                    sx[m] = make_float2(yv.x + dv.x, yv.y + dv.y);
                }
            }
            if (lane < n) {
                sdr[(size_t)ib * n + lane] = accept ? make_float2(rb.x - rv.x, rb.y - rv.y) : make_float2(0.0f, 0.0f);
                if (accept) sr[lane] = rb;
            }
            if (lane == 0) {
                sal[ib] = alpha;
                scnt[ib] = c;
            }
            if (accept) Fk += dF;
            BLOCK_WAVE_SYNC();
            if (k % J == 0 || k >= a.fista_cap) {
                kkt = kkt_of_x();
                fl += f8n * (unsigned long long)l;
                conv = kkt <= a.tol;
                nonfinite = !isfinite(kkt) || !isfinite(Fk);
            }
        }
        // retire: x, status, iterations; unsolved finite pixels go to the FP64 stage
        float2 *Xo = a.X + (size_t)pix * l;
        for (int m = lane; m < l; m += 64) Xo[m] = sx[m];
        if (lane == 0) {
            uint32_t st = 0;
            if (bad) st |= L1LS_PX_BAD_LAMBDA;
            else if (nonfinite) st |= L1LS_PX_NONFINITE;
            else if (!conv) st |= L1LS_PX_MAX_ITER;
            a.status[pix] = st;
            a.iters[pix] = k;
            a.kkt32[pix] = bad ? 0.0f : kkt;
            if (a.polish && !bad && !nonfinite) {
                const uint32_t slot = atomicAdd(a.polish_count, 1u);
                a.polish_list[slot] = (int32_t)pix;
            }
        }
        BLOCK_WAVE_SYNC();
    }
    if (lane == 0) atomicAdd(&a.work[0], fl);
}

hipError_t launch_setup_blocks(int n, int l, int J, const float2 *A, BlockConsts *bc, hipStream_t s)
{
    hipLaunchKernelGGL(setup_blocks_kernel, dim3(J), dim3(256), 0, s, n, l, J, A, bc);
    return hipGetLastError();
}

hipError_t launch_fista_blocks(const BlocksArgs &ba, hipStream_t s)
{
    const size_t lds = fista_blocks_lds(ba.f.n, ba.f.l_pad, ba.J);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fista_blocks_kernel, 64, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t groups = (int64_t)per_cu * cus;
    if (groups > ba.f.p) groups = ba.f.p;
    if (groups < 1) groups = 1;
    hipLaunchKernelGGL(fista_blocks_kernel, dim3((unsigned)groups), dim3(64), lds, s, ba);
    return hipGetLastError();
}

}  // namespace l1ls
