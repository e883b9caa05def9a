// Wave-per-pixel form of the accelerated proximal-gradient iteration (complex
// L1LS of arXiv 1805.01759, Algorithm 1 with one block), for shapes outside
// the register-resident MFMA kernel (N up to 128, L up to 1024).  It follows
// the same reading of the algorithm as that kernel:
//   beta_k = max(0, (k-2)/(k+1));  y = x^k + beta (x^k - x^{k-1});
//   grad f(y) = G_k + beta (G_k - G_{k-1})       (grad f is affine)
//   x-bar = S_{alpha lambda}(y - alpha grad f(y));  d = x-bar - y;  w = A d
//   Eq. (15) for quadratic f:  ||A d||^2 <= ||d||^2 / (2 alpha), else alpha *= C_alpha
//   accept iff F(x-bar) - F(x^k) <= 0, formed from differences
//   r_{k+1} = r(y) + w,  G_{k+1} = 2 A^H r_{k+1}
// One wave per pixel; A is read from the packed workspace copies (L2-resident:
// it is shared by every pixel).
#include <algorithm>

#include "l1ls_internal.h"

namespace l1ls {

__device__ __forceinline__ float wsumf(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wmaxf(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ void cprox_w(float vr, float vi, float tau, float &o_r, float &o_i)
{
    const float m = sqrtf(vr * vr + vi * vi);
    const float sc = m > tau ? 1.0f - tau / m : 0.0f;
    o_r = vr * sc;
    o_i = vi * sc;
}

#define WAVE_SYNC()                          \
    do {                                     \
        __builtin_amdgcn_wave_barrier();     \
        __builtin_amdgcn_s_waitcnt(0);       \
        __builtin_amdgcn_wave_barrier();     \
    } while (0)

// The pixel's x^k, x^{k-1}, G_k, G_{k-1} live in registers: lane `lane` holds
// bins m = lane + 64 c, c < NC (NC = 64-bin chunks, rounded up to an
// instantiated count); d, the residuals and A d sit in LDS for the row-wise
// forward product, so a pixel needs (l_pad + 3 N) x 8 bytes of LDS.
template <int NC>
__device__ __forceinline__ void fista_wave_stack(const FistaArgs &a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int n = a.n, l = a.l, ld = a.l_pad;
    float2 *D = reinterpret_cast<float2 *>(smem);  // d = x-bar - y of the current trial (64 NC)
    float2 *R = D + 64 * NC;                        // r_k (n)
    float2 *Rp = R + n;                             // r_{k-1}
    float2 *W = Rp + n;                             // A d
    // lanes per row of the forward product: 64 / (rows handled per pass)
    const int rows_per_pass = n <= 16 ? 16 : (n <= 32 ? 32 : 64);
    const int rpl = 64 / rows_per_pass;
    const float lf = (float)a.consts->lf;
    const float inv_lf = (float)(1.0 / a.consts->lf);
    const float alpha0 = (float)a.consts->alpha0;
    const float afloor = inv_lf;
    unsigned long long n_fwd = 0, n_adj = 0;
    float2 X[NC], Xp[NC], G[NC], Gp[NC];

    // G = 2 A^H r for the lane's bins (bins >= l give 0: A is zero padded to l_pad)
    auto adjoint = [&]() {
        float gr[NC], gi[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) gr[c] = gi[c] = 0.0f;
        for (int i = 0; i < n; ++i) {
            const float2 rv = R[i];
            const float2 *row = a.A + (size_t)i * ld;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int j = lane + 64 * c;
                const float2 av = j < ld ? row[j] : make_float2(0.0f, 0.0f);
                gr[c] = fmaf(av.x, rv.x, fmaf(av.y, rv.y, gr[c]));
                gi[c] = fmaf(av.x, rv.y, fmaf(-av.y, rv.x, gi[c]));
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) G[c] = make_float2(2.0f * gr[c], 2.0f * gi[c]);
    };

    // W = A D (D in LDS): lanes over rows (rpl lanes per row when N is small,
    // each taking every rpl-th column), A read through its transposed copy so
    // that the lanes' loads are contiguous; returns ||W||^2
    auto forward = [&]() {
        float w2 = 0.0f;
        for (int i0 = 0; i0 < n; i0 += rows_per_pass) {
            const int i = i0 + lane % rows_per_pass, part = lane / rows_per_pass;
            float wr = 0.0f, wi = 0.0f;
            if (i < n) {
                for (int j = part; j < l; j += rpl) {
                    const float2 av = a.At[(size_t)j * n + i], dv = D[j];
                    wr = fmaf(av.x, dv.x, fmaf(-av.y, dv.y, wr));
                    wi = fmaf(av.x, dv.y, fmaf(av.y, dv.x, wi));
                }
            }
            for (int o = rows_per_pass; o < 64; o <<= 1) {
                wr += __shfl_xor(wr, o, 64);
                wi += __shfl_xor(wi, o, 64);
            }
            if (i < n && part == 0) {
                W[i] = make_float2(wr, wi);
                w2 += wr * wr + wi * wi;
            }
        }
        return wsumf(w2);
    };

    for (;;) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(a.queue, 1u);
        base = __shfl(base, 0, 64);
        if ((int64_t)base >= a.p) break;
        const int64_t pix = base;
        float lam = a.lambda[pix * a.lambda_stride];
        const bool bad = !(lam > 0.0f) || !isfinite(lam);
        if (bad) lam = 1.0f;
        const float2 *b = a.B + (size_t)pix * n;
        float Fk;
        if (a.warm) {
            // Init of Algorithm 1 from the given x^(0) (in X): x^1 = x^0,
            // r_1 = A x^0 - b and F(x^0) = ||r_1||^2 + lambda ||x^0||_1
            const float2 *xi0 = a.X + (size_t)pix * l;
            float l1 = 0.0f;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int m = lane + 64 * c;
                X[c] = Xp[c] = m < l ? xi0[m] : make_float2(0.0f, 0.0f);
                Gp[c] = make_float2(0.0f, 0.0f);
                D[m] = X[c];
                l1 += sqrtf(X[c].x * X[c].x + X[c].y * X[c].y);
            }
            WAVE_SYNC();
            forward();
            ++n_fwd;
            WAVE_SYNC();
            float rr = 0.0f;
            for (int i = lane; i < n; i += 64) {
                const float2 v = b[i], w = W[i];
                R[i] = Rp[i] = make_float2(w.x - v.x, w.y - v.y);
                rr += (w.x - v.x) * (w.x - v.x) + (w.y - v.y) * (w.y - v.y);
            }
            Fk = wsumf(rr) + lam * wsumf(l1);
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) X[c] = Xp[c] = Gp[c] = make_float2(0.0f, 0.0f);
            float bb = 0.0f;
            for (int i = lane; i < n; i += 64) {
                const float2 v = b[i];
                R[i] = Rp[i] = make_float2(-v.x, -v.y);
                bb += v.x * v.x + v.y * v.y;
            }
            Fk = wsumf(bb);
        }
        WAVE_SYNC();
        adjoint();
        ++n_adj;
        float alpha = alpha0;
        int k = 1;
        float kkt = 0.0f;
        bool conv = false, nonfinite = false;
        for (;;) {
            // natural KKT residual at x^k with G_k
            float kmax = 0.0f;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const float2 x = X[c], g = G[c];
                float p_r, p_i;
                cprox_w(x.x - g.x * inv_lf, x.y - g.y * inv_lf, lam * inv_lf, p_r, p_i);
                const float e_r = x.x - p_r, e_i = x.y - p_i;
                kmax = fmaxf(kmax, e_r * e_r + e_i * e_i);
            }
            kkt = lf * sqrtf(wmaxf(kmax)) / lam;
            nonfinite = !isfinite(kkt) || !isfinite(Fk);
            conv = kkt <= a.tol;
            if (bad || nonfinite || conv || (k - 1) >= a.fista_cap) break;
            const float beta = fmaxf(0.0f, (float)(k - 2) / (float)(k + 1));
            float d2 = 0.0f, dl1 = 0.0f;
            for (int trial = 0; trial < 64; ++trial) {
                const float tau = alpha * lam;
                d2 = 0.0f;
                dl1 = 0.0f;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const float2 x = X[c], xp = Xp[c], g = G[c], gp = Gp[c];
                    const float y_r = x.x + beta * (x.x - xp.x), y_i = x.y + beta * (x.y - xp.y);
                    const float gy_r = g.x + beta * (g.x - gp.x), gy_i = g.y + beta * (g.y - gp.y);
                    float xb_r, xb_i;
                    cprox_w(y_r - alpha * gy_r, y_i - alpha * gy_i, tau, xb_r, xb_i);
                    const float d_r = xb_r - y_r, d_i = xb_i - y_i;
                    D[lane + 64 * c] = make_float2(d_r, d_i);
                    d2 += d_r * d_r + d_i * d_i;
                    const float den = sqrtf(xb_r * xb_r + xb_i * xb_i) + sqrtf(x.x * x.x + x.y * x.y);
                    const float num = (xb_r - x.x) * (xb_r + x.x) + (xb_i - x.y) * (xb_i + x.y);
                    dl1 += den > 0.0f ? num / den : 0.0f;
                }
                d2 = wsumf(d2);
                dl1 = wsumf(dl1);
                WAVE_SYNC();
                const float w2 = forward();
                ++n_fwd;
                WAVE_SYNC();
                if (!(a.backtracking && w2 > d2 / (2.0f * alpha) && alpha > afloor)) break;
                if (k == 1 && trial == 0 && !a.warm) {
                    // First iteration: y = 0, so x-bar(alpha) = alpha S_lambda(-G_0) is linear in
                    // alpha and Eq. (15) reads alpha <= ||d||^2 / (2 ||A d||^2) at every alpha:
                    // jump to where the shrink sequence ends and scale d, A d, ||x-bar||_1.
                    const float rho = d2 / (2.0f * w2);
                    float an = alpha;
                    while (an > rho && an > afloor) an = fmaxf(a.c_alpha * an, afloor);
                    const float cs = an / alpha;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const float2 dv = D[lane + 64 * c];
                        D[lane + 64 * c] = make_float2(dv.x * cs, dv.y * cs);
                    }
                    for (int i = lane; i < n; i += 64) W[i] = make_float2(W[i].x * cs, W[i].y * cs);
                    dl1 *= cs;
                    alpha = an;
                    WAVE_SYNC();
                    break;
                }
                alpha = fmaxf(a.c_alpha * alpha, afloor);
            }
            // monotone acceptance from differences
            float dfr = 0.0f;
            for (int i = lane; i < n; i += 64) {
                const float2 r = R[i], rp = Rp[i], w = W[i];
                const float dr_r = beta * (r.x - rp.x) + w.x, dr_i = beta * (r.y - rp.y) + w.y;
                dfr += dr_r * (2.0f * r.x + dr_r) + dr_i * (2.0f * r.y + dr_i);
            }
            const float dF = wsumf(dfr) + lam * dl1;
            const bool accept = !a.monotone || dF <= 0.0f;
            for (int i = lane; i < n; i += 64) {
                const float2 r = R[i], rp = Rp[i], w = W[i];
                Rp[i] = r;
                if (accept)
                    R[i] = make_float2(r.x + beta * (r.x - rp.x) + w.x, r.y + beta * (r.y - rp.y) + w.y);
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const float2 x = X[c], xp = Xp[c], d = D[lane + 64 * c];
                Xp[c] = x;
                Gp[c] = G[c];
                if (accept)
                    X[c] = make_float2(x.x + beta * (x.x - xp.x) + d.x, x.y + beta * (x.y - xp.y) + d.y);
            }
            if (accept) Fk += dF;
            ++k;
            WAVE_SYNC();
            adjoint();
            ++n_adj;
        }
        // retire
        float2 *xo = a.X + (size_t)pix * l;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (lane + 64 * c < l) xo[lane + 64 * c] = X[c];
        if (lane == 0) {
            uint32_t st = 0;
            if (bad) st |= L1LS_PX_BAD_LAMBDA;
            else if (nonfinite) st |= L1LS_PX_NONFINITE;
            else if (!conv) st |= L1LS_PX_MAX_ITER;
            a.status[pix] = st;
            a.iters[pix] = k - 1;
            a.kkt32[pix] = bad ? 0.0f : kkt;
            if (a.polish && !bad && !nonfinite) {
                const uint32_t slot = atomicAdd(a.polish_count, 1u);
                a.polish_list[slot] = (int32_t)pix;
            }
        }
        WAVE_SYNC();
    }
    if (lane == 0) {
        atomicAdd(&a.work[0], n_fwd);
        atomicAdd(&a.work[1], n_adj);
    }
}

// The stacks of a table one after another (pixels from each stack's queue).
template <int NC>
__global__ void __launch_bounds__(64) fista_wave_kernel(const StackTable t)
{
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        fista_wave_stack<NC>(fista_args_for(t.d[i], t.o));
    }
}

// instantiated chunk counts (64 bins each) and the one used for l
int wave_chunks(int l)
{
    const int c = (l + 63) / 64;
    const int opts[] = {1, 2, 3, 4, 6, 8, 12, 16};
    for (int o : opts)
        if (c <= o) return o;
    return -1;
}

size_t fista_wave_lds(int n, int l) { return (size_t)(64 * wave_chunks(l) + 3 * n) * sizeof(float2); }

template <int NC>
static hipError_t launch_wave_nc(const StackTable &t, hipStream_t s)
{
    size_t lds = 0;
    int64_t need = 0;
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        if (wave_chunks(t.d[i].l) != NC) return hipErrorInvalidConfiguration;
        lds = std::max(lds, fista_wave_lds(t.d[i].n, t.d[i].l));
        need += t.d[i].p;
    }
    if (need == 0) return hipSuccess;
    auto kern = fista_wave_kernel<NC>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t groups = (int64_t)per_cu * cus;
    if (groups > need) groups = need;
    if (groups < 1) groups = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(64), lds, s, t);
    return hipGetLastError();
}

hipError_t launch_wave_table(const StackTable &t, int nc, hipStream_t s)
{
    switch (nc) {
    case 1: return launch_wave_nc<1>(t, s);
    case 2: return launch_wave_nc<2>(t, s);
    case 3: return launch_wave_nc<3>(t, s);
    case 4: return launch_wave_nc<4>(t, s);
    case 6: return launch_wave_nc<6>(t, s);
    case 8: return launch_wave_nc<8>(t, s);
    case 12: return launch_wave_nc<12>(t, s);
    case 16: return launch_wave_nc<16>(t, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace l1ls
