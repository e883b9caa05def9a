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
#pragma once
#include "l1ls_internal.h"

namespace l1ls {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

typedef short s4 __attribute__((ext_vector_type(4)));

// bfloat16 round-to-nearest-even of an FP32 value (finite inputs), as bits
__device__ __forceinline__ uint32_t bf16_rne_bits(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// x = hi + lo with hi = bf16_rne(x), lo = bf16_rne(x - hi): ~16 significand bits
__device__ __forceinline__ void split_bf16(const float (&v)[4], s4 &hi, s4 &lo)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t h = bf16_rne_bits(v[q]);
        const float rem = v[q] - __uint_as_float(h << 16);
        hi[q] = (short)h;
        lo[q] = (short)bf16_rne_bits(rem);
    }
}

// One 16x16 tile times one 16-row block of the K dimension: the four FP32 MFMA
// k-steps r = 0..3 (k-slot h of lane group h holds row 16 b + 4 h + r) are the
// four k values 4 h + r of a 16x16x16 bf16 MFMA, so the split-BF16 form is three
// such MFMAs (hi*hi + hi*lo + lo*hi) with FP32 accumulation.
template <int PREC>
__device__ __forceinline__ f4 mma_block(const float (&av)[4], const float (&bv)[4], f4 acc)
{
    if constexpr (PREC == L1LS_FP32) {
        acc = mfma4(av[0], bv[0], acc);
        acc = mfma4(av[1], bv[1], acc);
        acc = mfma4(av[2], bv[2], acc);
        acc = mfma4(av[3], bv[3], acc);
    } else {
        s4 ah, al, bh, bl;
        split_bf16(av, ah, al);
        split_bf16(bv, bh, bl);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    }
    return acc;
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

// Operand loads of A.  `off` is an opaque zero (see opaque_zero) so that the
// compiler re-loads A at every use instead of hoisting the loop-invariant
// values into registers (which would cost 64 NZB registers per lane).
template <bool ALDS>
struct AView {
    const float2 *p;
    int ld;
    __device__ __forceinline__ f4 load4(int n, int m, int off) const
    {
        return *reinterpret_cast<const f4 *>(p + off + n * ld + m);
    }
    __device__ __forceinline__ float2 load2(int n, int m, int off) const { return p[off + n * ld + m]; }
};

__device__ __forceinline__ int opaque_zero()
{
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

template <int NZB, int KB, bool ALDS, int PREC>
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
        const int aoff = opaque_zero();
#pragma unroll
        for (int kb = 0; kb < NZB; ++kb) {
            // rows n >= N carry r = 0; their (clamped, in-bounds) A values are masked
            const int n0 = 8 * kb + 2 * h;
            const float k0 = n0 < n ? 1.0f : 0.0f, k1 = n0 + 1 < n ? 1.0f : 0.0f;
            const int r0 = n0 < n ? n0 : n - 1, r1 = n0 + 1 < n ? n0 + 1 : n - 1;
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                const int m = m_base + 8 * b + (j >> 1);
                const float2 a0 = Av.load2(r0, m, aoff), a1 = Av.load2(r1, m, aoff);
                // Re G_m = sum Re(a) Re(r') + Im(a) Im(r');  Im G_m = sum Re(a) Im(r') - Im(a) Re(r')
                const float ao[4] = {k0 * (gim ? -a0.y : a0.x), k0 * (gim ? a0.x : a0.y),
                                     k1 * (gim ? -a1.y : a1.x), k1 * (gim ? a1.x : a1.y)};
                acc[b] = mma_block<PREC>(ao, R2[kb], acc[b]);
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
            const int aoff = opaque_zero();
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
                    f4 av = Av.load4(nn < n ? nn : n - 1, m0, aoff) * kz;
                    // Re Z_n = sum Re(a) Re(x) - Im(a) Im(x);  Im Z_n = sum Im(a) Re(x) + Re(a) Im(x)
                    const float ao[4] = {zim ? av[1] : av[0], zim ? av[0] : -av[1],
                                         zim ? av[3] : av[2], zim ? av[2] : -av[3]};
                    acc[ob] = mma_block<PREC>(ao, d, acc[ob]);
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
            float d2s = S[0];
            bool jumped = false;
            if (k == 1 && trial == 0 && active && !retire && a.backtracking && w2 > d2s / (2.0f * alpha) &&
                alpha > afloor) {
                // First iteration: y = x^0 = 0, so x-bar(alpha) = alpha S_lambda(-G_0) is linear
                // in alpha and Eq. (15) reads alpha <= ||d||^2 / (2 ||A d||^2) at every alpha:
                // the shrink sequence ends where this one product says, and A d and
                // ||x-bar||_1 scale with alpha.
                const float rho = d2s / (2.0f * w2);
                float an = alpha;
                while (an > rho && an > afloor) an = fmaxf(a.c_alpha * an, afloor);
                const float c = an / alpha;
#pragma unroll
                for (int ob = 0; ob < NZB; ++ob) Wt[ob] *= c;
                w2 *= c * c;
                d2s *= c * c;
                l1 *= c;
                alpha = an;
                jumped = true;
            }
            const bool fail = active && !retire && !jumped && a.backtracking &&
                              (w2 > d2s / (2.0f * alpha)) && alpha > afloor;
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

template <int NZB, int KB, bool ALDS, int PREC>
hipError_t launch_one(const FistaArgs &a, int max_groups, hipStream_t s)
{
    const size_t lds = fista_lds_bytes(a.n, a.l_pad, a.waves, NZB, ALDS);
    auto kern = fista_kernel<NZB, KB, ALDS, PREC>;
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


}  // namespace l1ls
