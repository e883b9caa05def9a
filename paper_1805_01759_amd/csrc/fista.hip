// Persistent accelerated proximal-gradient kernel for the complex L1LS
// problem of Shi, Zhu, Yin, Bamler (arXiv 1805.01759), gfx950.
//
// One workgroup owns a tile of 16 pixel slots and W waves; wave w owns the
// complex unknowns [64 w, 64 w + 64) of every slot.  Per slot it runs
// Algorithm 1 with one block (J = 1):
//   y      = x^k + beta_k (x^k - x^{k-1}),  beta_k = max(0, (k-2)/(k+1))   Eqs. (11)-(12)
//   x-bar  = S_{alpha lambda}(y - alpha grad f(y))                          Eqs. (10), (12)
//   shrink alpha by C_alpha until Eq. (15) holds                            Eq. (15)
//   accept x-bar only if F(x-bar) <= F(x^k)                                  Algorithm 1
// with f(x) = ||Ax - b||^2, grad f = 2 A^H (A x - b).
//
// Data layout and the two contractions.  The tile's unknowns are real-embedded
// (row 2m = Re x_m, row 2m+1 = Im x_m) and kept in registers in the output
// layout of v_mfma_f32_16x16x4f32: lane (j = lane%16, h = lane/16) holds, for
// each 16-row block b of its wave's slice, rows 16 b + 4 h + r (r = 0..3) of
// pixel slot j, i.e. complex unknowns m = 8 b + 2 h and 8 b + 2 h + 1.  The
// same four registers are the B operand of the forward product (its four
// k-slots are the four lane groups h), so the prox output feeds the matrix
// core with no data movement; A supplies the A operand, permuted to match.
//   forward  W = A d      (d = x-bar - y)  : MFMA over K = 2 x slice, split
//                                            over waves, reduced through LDS
//   adjoint  G = 2 A^H r  (r = A x - b)    : MFMA over K = 2 N, per wave
// grad f is affine in x, so grad f(y) = G_k + beta (G_k - G_{k-1}) needs no
// product; one adjoint per accepted step gives G_{k+1} and with it the exact
// KKT residual of x^{k+1}.  For quadratic f the condition of Eq. (15) at
// (y, x-bar) is identical to ||A d||^2 <= ||d||^2 / (2 alpha) (the linear terms
// cancel), which is evaluated from the forward product of d and is free of
// the cancellation of the literal form.
//
// Pixels retire when the FP32 KKT residual passes tol, or after fista_cap
// iterations; a retired slot is refilled at once from a global atomic queue.
#include "l1ls_internal.h"

namespace l1ls {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Sum / max over the four lanes (h = 0..3) that hold one pixel slot.
__device__ __forceinline__ float sum_h(float v)
{
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}
__device__ __forceinline__ float max_h(float v)
{
    v = fmaxf(v, __shfl_xor(v, 16, 64));
    v = fmaxf(v, __shfl_xor(v, 32, 64));
    return v;
}

// Complex soft threshold S_tau(v) = v max(0, 1 - tau/|v|); |v| <= tau -> 0.
__device__ __forceinline__ void cprox(float vr, float vi, float tau, float &orr, float &oi)
{
    const float m2 = vr * vr + vi * vi;
    const float s = 1.0f - tau * __builtin_amdgcn_rsqf(m2);
    const float sc = m2 > tau * tau ? s : 0.0f;  // select: no branch, 0/0 discarded
    orr = vr * sc;
    oi = vi * sc;
}

// One complex unknown: extrapolate, gradient step, prox.  Shared by the trial
// and the acceptance so that both produce bit-identical x-bar.
__device__ __forceinline__ void step_one(float x_r, float x_i, float xp_r, float xp_i, float g_r,
                                         float g_i, float gp_r, float gp_i, float beta,
                                         float alpha, float tau, float &y_r, float &y_i,
                                         float &xb_r, float &xb_i)
{
    y_r = x_r + beta * (x_r - xp_r);
    y_i = x_i + beta * (x_i - xp_i);
    float gy_r = g_r + beta * (g_r - gp_r);
    float gy_i = g_i + beta * (g_i - gp_i);
    cprox(y_r - alpha * gy_r, y_i - alpha * gy_i, tau, xb_r, xb_i);
}

template <bool ALDS>
struct AView {
    const float2 *p;
    int ld;
    __device__ __forceinline__ f4 load4(int n, int m) const
    {
        return *reinterpret_cast<const f4 *>(p + (size_t)n * ld + m);
    }
    __device__ __forceinline__ float2 load2(int n, int m) const { return p[(size_t)n * ld + m]; }
};

template <int NZB, int KB, bool ALDS>
__global__ void __launch_bounds__(256) fista_kernel(const FistaArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int W = a.waves;
    const int j = lane & 15;
    const int h = lane >> 4;
    const int n = a.n;
    const int l = a.l;
    const int lds_ld = a.l_pad + 4;  // padded row stride in LDS (bank spread)

    size_t off = 0;
    float2 *sA = reinterpret_cast<float2 *>(smem);
    if (ALDS) off = ((size_t)n * lds_ld * sizeof(float2) + 15) & ~(size_t)15;
    f4 *sPW = reinterpret_cast<f4 *>(smem + off);
    off += (size_t)W * NZB * 64 * sizeof(f4);
    f4 *sPS = reinterpret_cast<f4 *>(smem + off);
    off += (size_t)W * 16 * sizeof(f4);
    uint32_t *sQ = reinterpret_cast<uint32_t *>(smem + off);

    AView<ALDS> Av;
    if (ALDS) {
        for (int idx = tid; idx < n * (a.l_pad / 2); idx += blockDim.x) {
            int row = idx / (a.l_pad / 2), c2 = idx % (a.l_pad / 2);
            *reinterpret_cast<f4 *>(sA + (size_t)row * lds_ld + 2 * c2) =
                *reinterpret_cast<const f4 *>(a.A + (size_t)row * a.l_pad + 2 * c2);
        }
        Av.p = sA;
        Av.ld = lds_ld;
    } else {
        Av.p = a.A;
        Av.ld = a.l_pad;
    }

    const double lf_d = a.consts->lf;
    const float lf = (float)lf_d;
    const float inv_lf = (float)(1.0 / lf_d);
    const float alpha0 = (float)a.consts->alpha0;
    const float afloor = inv_lf;
    const int m_base = w * 8 * KB;

    float X[KB][4], Xp[KB][4], G[KB][4], Gp[KB][4];
    float R[NZB][4], Rp[NZB][4];  // residual A x - b of x^k and x^{k-1}
#pragma unroll
    for (int b = 0; b < KB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) X[b][r] = Xp[b][r] = G[b][r] = Gp[b][r] = 0.0f;
#pragma unroll
    for (int ob = 0; ob < NZB; ++ob)
#pragma unroll
        for (int r = 0; r < 4; ++r) R[ob][r] = Rp[ob][r] = 0.0f;

    int64_t pix = -1;
    int k = 1;
    float alpha = alpha0, lam = 1.0f, Fk = 0.0f;
    bool active = false, bad = false, qdone = false;

    // ---- refill the slots in `mask` from the global queue (workgroup-uniform)
    auto refill = [&](uint32_t mask) {
        if (mask == 0) return;
        if (qdone) {
            if ((mask >> j) & 1u) { active = false; pix = -1; }
            return;
        }
        const uint32_t nfree = __popc(mask);
        __syncthreads();
        if (tid == 0) sQ[0] = atomicAdd(a.queue, nfree);
        __syncthreads();
        const uint64_t base = sQ[0];
        if (base + nfree >= (uint64_t)a.p) qdone = true;
        if ((mask >> j) & 1u) {
            const uint64_t np = base + (uint64_t)__popc(mask & ((1u << j) - 1u));
            if (np < (uint64_t)a.p) {
                pix = (int64_t)np;
                active = true;
                k = 1;
                alpha = alpha0;
                lam = a.lambda[pix * a.lambda_stride];
                bad = !(lam > 0.0f) || !isfinite(lam);
                if (bad) lam = 1.0f;
#pragma unroll
                for (int b = 0; b < KB; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) X[b][r] = Xp[b][r] = G[b][r] = Gp[b][r] = 0.0f;
                float bb = 0.0f;
                const float2 *Bp = a.B + (size_t)pix * n;
#pragma unroll
                for (int ob = 0; ob < NZB; ++ob)
#pragma unroll
                    for (int rp = 0; rp < 2; ++rp) {
                        const int nn = 8 * ob + 2 * h + rp;
                        float2 v = nn < n ? Bp[nn] : make_float2(0.0f, 0.0f);
                        R[ob][2 * rp] = Rp[ob][2 * rp] = -v.x;
                        R[ob][2 * rp + 1] = Rp[ob][2 * rp + 1] = -v.y;
                        bb += v.x * v.x + v.y * v.y;
                    }
                Fk = sum_h(bb);
            } else {
                active = false;
                pix = -1;
            }
        }
    };

    // ---- G = 2 A^H r for the wave's slice (all slots)
    auto adjoint = [&]() {
        float R2[NZB][4];
#pragma unroll
        for (int ob = 0; ob < NZB; ++ob)
#pragma unroll
            for (int r = 0; r < 4; ++r) R2[ob][r] = 2.0f * R[ob][r];
        f4 acc[KB];
#pragma unroll
        for (int b = 0; b < KB; ++b) acc[b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        const bool gim = (j & 1) != 0;
#pragma unroll
        for (int kb = 0; kb < NZB; ++kb) {
            // rows n >= N carry r = 0; their (clamped, in-bounds) A values are masked
            const int n0 = 8 * kb + 2 * h;
            const float k0 = n0 < n ? 1.0f : 0.0f, k1 = n0 + 1 < n ? 1.0f : 0.0f;
            const int r0 = n0 < n ? n0 : n - 1, r1 = n0 + 1 < n ? n0 + 1 : n - 1;
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                const int m = m_base + 8 * b + (j >> 1);
                const float2 a0 = Av.load2(r0, m), a1 = Av.load2(r1, m);
                // Re G_m = sum Re(a) Re(r') + Im(a) Im(r');  Im G_m = sum Re(a) Im(r') - Im(a) Re(r')
                acc[b] = mfma4(k0 * (gim ? -a0.y : a0.x), R2[kb][0], acc[b]);
                acc[b] = mfma4(k0 * (gim ? a0.x : a0.y), R2[kb][1], acc[b]);
                acc[b] = mfma4(k1 * (gim ? -a1.y : a1.x), R2[kb][2], acc[b]);
                acc[b] = mfma4(k1 * (gim ? a1.x : a1.y), R2[kb][3], acc[b]);
                if ((b & 1) == 1) __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) G[b][r] = acc[b][r];
    };

    unsigned long long n_fwd = 0, n_adj = 0;  // pixel products (wave 0, lane 0 counts)
    refill(0xFFFFu);
    if (__ballot(active) == 0) return;
    adjoint();
    n_adj += __popcll(__ballot(active && h == 0));

    for (;;) {
        const float beta = fmaxf(0.0f, (float)(k - 2) / (float)(k + 1));
        bool first = true, retire = false, conv = false, nonfinite = false, capped = false;
        float kkt = 0.0f, l1 = 0.0f;
        f4 Wt[NZB];
        // natural KKT residual of x^k with its exact gradient G_k, and nnz(x^k)
        float kmax = 0.0f, nz = 0.0f;
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                float p_r, p_i;
                const float x_r = X[b][2 * c], x_i = X[b][2 * c + 1];
                cprox(x_r - G[b][2 * c] * inv_lf, x_i - G[b][2 * c + 1] * inv_lf, lam * inv_lf,
                      p_r, p_i);
                const float e_r = x_r - p_r, e_i = x_i - p_i;
                kmax = fmaxf(kmax, e_r * e_r + e_i * e_i);
                nz += (x_r != 0.0f || x_i != 0.0f) ? 1.0f : 0.0f;
            }
        kmax = max_h(kmax);
        nz = sum_h(nz);
        for (int trial = 0; trial < 64; ++trial) {
            n_fwd += __popcll(__ballot(active && h == 0));
            const float tau = alpha * lam;
            f4 acc[NZB];
#pragma unroll
            for (int ob = 0; ob < NZB; ++ob) acc[ob] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            float d2 = 0.0f, s1 = 0.0f;
            const bool zim = (j & 1) != 0;
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                float d[4];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    float y_r, y_i, xb_r, xb_i;
                    step_one(X[b][2 * c], X[b][2 * c + 1], Xp[b][2 * c], Xp[b][2 * c + 1],
                             G[b][2 * c], G[b][2 * c + 1], Gp[b][2 * c], Gp[b][2 * c + 1], beta,
                             alpha, tau, y_r, y_i, xb_r, xb_i);
                    d[2 * c] = xb_r - y_r;
                    d[2 * c + 1] = xb_i - y_i;
                    d2 += d[2 * c] * d[2 * c] + d[2 * c + 1] * d[2 * c + 1];
                    // |x-bar| - |x^k| without cancellation:
                    //   (|x-bar|^2 - |x^k|^2) / (|x-bar| + |x^k|)
                    const float x_r = X[b][2 * c], x_i = X[b][2 * c + 1];
                    const float den = sqrtf(xb_r * xb_r + xb_i * xb_i) + sqrtf(x_r * x_r + x_i * x_i);
                    const float num = (xb_r - x_r) * (xb_r + x_r) + (xb_i - x_i) * (xb_i + x_i);
                    s1 += den > 0.0f ? num * __builtin_amdgcn_rcpf(den) : 0.0f;
                }
                const int m0 = m_base + 8 * b + 2 * h;
#pragma unroll
                for (int ob = 0; ob < NZB; ++ob) {
                    const int nn = 8 * ob + (j >> 1);
                    const float kz = nn < n ? 1.0f : 0.0f;
                    f4 av = Av.load4(nn < n ? nn : n - 1, m0) * kz;
                    // Re Z_n = sum Re(a) Re(x) - Im(a) Im(x);  Im Z_n = sum Im(a) Re(x) + Re(a) Im(x)
                    acc[ob] = mfma4(zim ? av[1] : av[0], d[0], acc[ob]);
                    acc[ob] = mfma4(zim ? av[0] : -av[1], d[1], acc[ob]);
                    acc[ob] = mfma4(zim ? av[3] : av[2], d[2], acc[ob]);
                    acc[ob] = mfma4(zim ? av[2] : -av[3], d[3], acc[ob]);
                }
                // keep each block's operand loads next to their MFMAs (register pressure)
                __builtin_amdgcn_sched_barrier(0);
            }
            // cross-wave reduction of the forward partial products and scalars
            d2 = sum_h(d2);
            s1 = sum_h(s1);
#pragma unroll
            for (int ob = 0; ob < NZB; ++ob) sPW[((size_t)w * NZB + ob) * 64 + lane] = acc[ob];
            if (h == 0) sPS[w * 16 + j] = f4{d2, s1, kmax, nz};
            __syncthreads();
#pragma unroll
            for (int ob = 0; ob < NZB; ++ob) Wt[ob] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            f4 S = f4{0.0f, 0.0f, 0.0f, 0.0f};
            for (int ww = 0; ww < W; ++ww) {
#pragma unroll
                for (int ob = 0; ob < NZB; ++ob) Wt[ob] += sPW[((size_t)ww * NZB + ob) * 64 + lane];
                f4 ps = sPS[ww * 16 + j];
                S[0] += ps[0];
                S[1] += ps[1];
                S[2] = fmaxf(S[2], ps[2]);
                S[3] += ps[3];
            }
            __syncthreads();
            float w2 = 0.0f;
#pragma unroll
            for (int ob = 0; ob < NZB; ++ob)
#pragma unroll
                for (int r = 0; r < 4; ++r) w2 += Wt[ob][r] * Wt[ob][r];
            w2 = sum_h(w2);
            if (first) {
                kkt = lf * sqrtf(S[2]) / lam;
                nonfinite = !isfinite(kkt) || !isfinite(Fk);
                conv = kkt <= a.tol;
                capped = (k - 1) >= a.fista_cap;
                retire = active && (bad || nonfinite || conv || capped);
                // diag of a retiring slot: nnz of x^k
                if (retire && w == 0 && h == 0) {
                    uint32_t st = 0;
                    if (bad) st |= L1LS_PX_BAD_LAMBDA;
                    else if (nonfinite) st |= L1LS_PX_NONFINITE;
                    else if (!conv) st |= L1LS_PX_MAX_ITER;
                    a.status[pix] = st;
                    a.iters[pix] = k - 1;
                    a.kkt32[pix] = bad ? 0.0f : kkt;
                    // every finite pixel is offered to the FP64 stage, which first checks
                    // the FP64 KKT residual (the FP32 one carries rounding and drift)
                    if (a.polish && !bad && !nonfinite) {
                        uint32_t slot = atomicAdd(a.polish_count, 1u);
                        a.polish_list[slot] = (int32_t)pix;
                    }
                }
                first = false;
            }
            l1 = S[1];
            const bool fail = active && !retire && a.backtracking && (w2 > S[0] / (2.0f * alpha)) &&
                              alpha > afloor;
            if (__ballot(fail) == 0) break;
            if (fail) alpha = fmaxf(a.c_alpha * alpha, afloor);
        }

        // ---- retire: write x^k of the wave's slice
        if (retire) {
            float2 *Xo = a.X + (size_t)pix * l;
#pragma unroll
            for (int b = 0; b < KB; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int m = m_base + 8 * b + 2 * h + c;
                    if (m < l) Xo[m] = make_float2(X[b][2 * c], X[b][2 * c + 1]);
                }
        }

        // ---- monotone acceptance and state rotation (live slots)
        {
            // residual of x-bar: r(y) + A d, with r(y) = r_k + beta (r_k - r_{k-1}).
            // Monotone test of Algorithm 1 as the sign of F(x-bar) - F(x^k), formed
            // from differences so that it is not swamped by the rounding of F:
            //   ||r-bar||^2 - ||r_k||^2 = <r-bar - r_k, r-bar + r_k>,
            //   ||x-bar||_1 - ||x^k||_1 = sum (|x-bar| - |x^k|)  (accumulated above).
            float dfr = 0.0f;
            float Rb[NZB][4];
#pragma unroll
            for (int ob = 0; ob < NZB; ++ob)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float dr = beta * (R[ob][r] - Rp[ob][r]) + Wt[ob][r];
                    Rb[ob][r] = R[ob][r] + dr;
                    dfr += dr * (Rb[ob][r] + R[ob][r]);
                }
            dfr = sum_h(dfr);
            const float dF = dfr + lam * l1;
            const bool live = active && !retire;
            const bool accept = live && (!a.monotone || dF <= 0.0f);
            const float tau = alpha * lam;
#pragma unroll
            for (int b = 0; b < KB; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    float y_r, y_i, xb_r, xb_i;
                    step_one(X[b][2 * c], X[b][2 * c + 1], Xp[b][2 * c], Xp[b][2 * c + 1],
                             G[b][2 * c], G[b][2 * c + 1], Gp[b][2 * c], Gp[b][2 * c + 1], beta,
                             alpha, tau, y_r, y_i, xb_r, xb_i);
                    if (live) {
                        Xp[b][2 * c] = X[b][2 * c];
                        Xp[b][2 * c + 1] = X[b][2 * c + 1];
                        Gp[b][2 * c] = G[b][2 * c];
                        Gp[b][2 * c + 1] = G[b][2 * c + 1];
                    }
                    if (accept) {
                        X[b][2 * c] = xb_r;
                        X[b][2 * c + 1] = xb_i;
                    }
                }
#pragma unroll
            for (int ob = 0; ob < NZB; ++ob)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (live) Rp[ob][r] = R[ob][r];
                    if (accept) R[ob][r] = Rb[ob][r];
                }
            if (accept) Fk += dF;
            if (live) ++k;
        }

        // ---- refill retired slots, stop when the tile is empty
        const uint32_t rmask = (uint32_t)(__ballot(retire && h == 0) & 0xFFFFull);
        if (retire) active = false;
        refill(rmask);
        if (__ballot(active) == 0) break;
        adjoint();
        n_adj += __popcll(__ballot(active && h == 0));
    }
    if (tid == 0) {
        atomicAdd(&a.work[0], n_fwd);
        atomicAdd(&a.work[1], n_adj);
    }
}

// ---------------------------------------------------------------------------
// Setup: pack A (zero-padded columns), alpha0 = 1/(2 max_l ||a_l||^2),
// L_f = 2 lambda_max(A A^H) by FP64 power iteration on the Gram matrix, and
// reset the work queue.  One workgroup of 256 threads.
__global__ void __launch_bounds__(256) setup_kernel(int n, int l, int l_pad, const float2 *A,
                                                    float2 *Ap, double2 *M, StackConsts *consts,
                                                    uint32_t *queue, unsigned long long *work)
{
    __shared__ double red[256];
    __shared__ double2 v[kMaxN];
    __shared__ double2 wv[kMaxN];
    __shared__ double ctl[4];
    const int tid = threadIdx.x, bd = blockDim.x;
    if (tid < 4) queue[tid] = 0u;
    if (tid < 2) work[tid] = 0ull;
    for (int idx = tid; idx < n * l_pad; idx += bd) {
        const int r = idx / l_pad, c = idx % l_pad;
        Ap[idx] = c < l ? A[(size_t)r * l + c] : make_float2(0.0f, 0.0f);
    }
    double cm = 0.0;
    for (int c = tid; c < l; c += bd) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) {
            const float2 q = A[(size_t)r * l + c];
            s += (double)q.x * q.x + (double)q.y * q.y;
        }
        cm = fmax(cm, s);
    }
    red[tid] = cm;
    __syncthreads();
    for (int s = bd / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    const double colmax = red[0];
    __syncthreads();
    // Gram M = A A^H (FP64), row-major n x n
    for (int e = tid; e < n * n; e += bd) {
        const int i = e / n, kk = e % n;
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < l; ++c) {
            const float2 p = A[(size_t)i * l + c], q = A[(size_t)kk * l + c];
            sr += (double)p.x * q.x + (double)p.y * q.y;  // p conj(q)
            si += (double)p.y * q.x - (double)p.x * q.y;
        }
        M[e] = make_double2(sr, si);
    }
    __threadfence_block();
    __syncthreads();
    if (tid < n) v[tid] = make_double2(1.0 + 0.01 * tid, 0.001 * tid);
    if (tid == 0) { ctl[0] = 0.0; ctl[1] = 0.0; }
    __syncthreads();
    int it;
    double lam_prev = -1.0;
    for (it = 0; it < 4000; ++it) {
        // w = M v ; rayleigh = v^H M v / v^H v ; v = w / ||w||
        double pr = 0.0, nv = 0.0, nw = 0.0;
        if (tid < n) {
            double sr = 0.0, si = 0.0;
            for (int kk = 0; kk < n; ++kk) {
                const double2 m = M[tid * n + kk], x = v[kk];
                sr += m.x * x.x - m.y * x.y;
                si += m.x * x.y + m.y * x.x;
            }
            wv[tid] = make_double2(sr, si);
            pr = v[tid].x * sr + v[tid].y * si;  // Re(conj(v) w)
            nv = v[tid].x * v[tid].x + v[tid].y * v[tid].y;
            nw = sr * sr + si * si;
        }
        // three block sums
        red[tid] = pr;
        __syncthreads();
        for (int s = bd / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        const double rq_num = red[0];
        __syncthreads();
        red[tid] = nv;
        __syncthreads();
        for (int s = bd / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        const double vv = red[0];
        __syncthreads();
        red[tid] = nw;
        __syncthreads();
        for (int s = bd / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        const double ww = red[0];
        __syncthreads();
        const double lam_est = rq_num / vv;
        const double inv = ww > 0.0 ? 1.0 / sqrt(ww) : 0.0;
        if (tid < n) v[tid] = make_double2(wv[tid].x * inv, wv[tid].y * inv);
        __syncthreads();
        if (it > 20 && fabs(lam_est - lam_prev) <= 1e-15 * fabs(lam_est)) {
            lam_prev = lam_est;
            break;
        }
        lam_prev = lam_est;
    }
    if (tid == 0) {
        consts->lf = 2.0 * lam_prev;
        consts->alpha0 = colmax > 0.0 ? 1.0 / (2.0 * colmax) : 1.0;
        consts->lmax_it = (double)it;
        consts->pad = 0.0;
    }
}

// ---------------------------------------------------------------------------

size_t fista_lds_bytes(int n, int l_pad, int waves, int zb, bool a_lds)
{
    size_t off = a_lds ? (((size_t)n * (l_pad + 4) * sizeof(float2) + 15) & ~(size_t)15) : 0;
    off += (size_t)waves * zb * 64 * 16;
    off += (size_t)waves * 16 * 16;
    off += 16;
    return off;
}

bool fista_a_fits_lds(int n, int l_pad, int waves, int zb)
{
    // one wave per SIMD: a workgroup of W waves may use W/4 of the CU's 160 KB
    return fista_lds_bytes(n, l_pad, waves, zb, true) <= (size_t)160 * 1024 * waves / 4;
}

hipError_t launch_setup(int n, int l, int l_pad, const float2 *A, float2 *Ap, double2 *gram,
                        StackConsts *consts, uint32_t *queue, unsigned long long *work,
                        hipStream_t s)
{
    hipLaunchKernelGGL(setup_kernel, dim3(1), dim3(256), 0, s, n, l, l_pad, A, Ap, gram, consts,
                       queue, work);
    return hipGetLastError();
}

template <int NZB, int KB, bool ALDS>
static hipError_t launch_one(const FistaArgs &a, int max_groups, hipStream_t s)
{
    const size_t lds = fista_lds_bytes(a.n, a.l_pad, a.waves, NZB, ALDS);
    auto kern = fista_kernel<NZB, KB, ALDS>;
    static bool attr_done = false;  // per instantiation
    if (!attr_done) {
        hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
        attr_done = true;
    }
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * a.waves, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t groups = (int64_t)per_cu * cus;
    const int64_t need = (a.p + kTile - 1) / kTile;
    if (groups > need) groups = need;
    if (max_groups > 0 && groups > max_groups) groups = max_groups;
    if (groups < 1) groups = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(64 * a.waves), lds, s, a);
    return hipGetLastError();
}

template <int NZB>
static hipError_t launch_zb(const FistaArgs &a, int max_groups, hipStream_t s)
{
    const bool lds = fista_a_fits_lds(a.n, a.l_pad, a.waves, NZB);
    if (slice_blocks_for(a.l) == 8)
        return lds ? launch_one<NZB, 8, true>(a, max_groups, s) : launch_one<NZB, 8, false>(a, max_groups, s);
    return lds ? launch_one<NZB, 16, true>(a, max_groups, s) : launch_one<NZB, 16, false>(a, max_groups, s);
}

hipError_t launch_fista(const FistaArgs &a, int precision, int max_groups, hipStream_t s)
{
    (void)precision;
    switch (zblocks_for(a.n)) {
    case 1: return launch_zb<1>(a, max_groups, s);
    case 2: return launch_zb<2>(a, max_groups, s);
    case 3: return launch_zb<3>(a, max_groups, s);
    case 4: return launch_zb<4>(a, max_groups, s);
    case 5: return launch_zb<5>(a, max_groups, s);
    case 6: return launch_zb<6>(a, max_groups, s);
    case 7: return launch_zb<7>(a, max_groups, s);
    case 8: return launch_zb<8>(a, max_groups, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace l1ls
