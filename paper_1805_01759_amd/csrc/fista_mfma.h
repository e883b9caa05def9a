// Persistent accelerated proximal-gradient kernel (FP32 contractions) for the
// complex L1LS problem of Shi, Zhu, Yin, Bamler (arXiv 1805.01759), gfx950.
//
// One workgroup owns a tile of 16 pixel slots and W <= 4 waves (one per SIMD);
// wave w owns the complex unknowns [16 KB w, 16 KB (w + 1)) of every slot.  Per
// slot it runs Algorithm 1 with one block (J = 1):
//   y      = x^k + beta_k (x^k - x^{k-1}),  beta_k = max(0, (k-2)/(k+1))   Eqs. (11)-(12)
//   x-bar  = S_{alpha lambda}(y - alpha grad f(y))                          Eqs. (10), (12)
//   shrink alpha by C_alpha until Eq. (15) holds                            Eq. (15)
//   accept x-bar only if F(x-bar) <= F(x^k)                                  Algorithm 1
// with f(x) = ||Ax - b||^2, grad f = 2 A^H (A x - b).
//
// Register layout (the output layout of v_mfma_f32_16x16x4f32: lane l holds
// rows 4 (l/16) + q, q = 0..3, of column l%16).  Lane (j = lane%16, h = lane/16):
//   unknowns  block b, q:  m = 16 KB w + 16 b + 4 h + q of pixel slot j,
//             real and imaginary parts in separate vectors (X_re[b][q], X_im[b][q]);
//   residual  block t, q:  n = 16 t + 4 h + q of pixel slot j (R_re[t][q], R_im[t][q]).
// Both contractions take A directly as the MFMA A operand (a plain load, no
// per-element selects or masks: A is zero padded to 16 T rows), and the complex
// arithmetic is spread over separate real and imaginary accumulators:
//   forward  W = A d:     W_re += A_re d_re + A_im (-d_im),  W_im += A_im d_re + A_re d_im
//            (A operand: row n = 16 t + j, k-slot h <-> m = 16 b + 4 h + q; the k-slots
//            are exactly the unknowns the lane holds, so d feeds the B operand as is)
//   adjoint  G = 2 A^H r: G_re += A_re (2 r_re) + A_im (2 r_im),
//                         G_im += A_re (2 r_im) + A_im (-2 r_re)
//            (A operand: row m = 16 b + j, k-slot h <-> n = 16 t + 4 h + q)
// so each wave issues 16 T KB MFMAs per product and almost no VALU for operands.
//
// grad f is affine in x, so grad f(y) = G_k + beta (G_k - G_{k-1}) needs no
// product; one adjoint per accepted step gives G_{k+1} and with it the exact
// KKT residual of x^{k+1}.  For quadratic f the condition of Eq. (15) at
// (y, x-bar) is identical to ||A d||^2 <= ||d||^2 / (2 alpha) (the linear terms
// cancel), which is evaluated from the forward product of d.  The monotone
// test is the sign of F(x-bar) - F(x^k) formed from differences:
//   ||r-bar||^2 - ||r_k||^2 = <r-bar - r_k, r-bar + r_k>,
//   ||x-bar||_1 - ||x^k||_1 = sum_m (|x-bar_m| - |x^k_m|), |x-bar_m| from the prox.
// The last trial's x-bar stays in registers for the acceptance.
//
// Split-BF16 (PREC = L1LS_SPLIT_BF16): every real product a.b is formed as
// hi(a)hi(b) + hi(a)lo(b) + lo(a)hi(b) with x = hi(x) + lo(x), hi = RNE bf16 of x,
// lo = RNE bf16 of the remainder, accumulated in FP32 by v_mfma_f32_16x16x16bf16_1k,
// whose four k values per lane are the q = 0..3 of the FP32 form.  A is split
// once into four bf16 planes (re/im x hi/lo), each held twice: row-major for the
// forward product (four consecutive m per lane read) and transposed for the
// adjoint (four consecutive n per lane read), so the A operands are plain 8-byte
// loads; the planes are staged in LDS where they fit (ALDS) and otherwise read
// from the copy the setup writes to the workspace, which stays in L2.  d and r
// are split per product with the hardware bf16 conversion.
//
// Pixels retire when the FP32 KKT residual passes tol, or after fista_cap
// iterations; a retired slot is refilled at once from a global atomic queue.
#pragma once
#include "l1ls_internal.h"

namespace l1ls {

namespace fm {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f4 mfma_bf(s4 a, s4 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// v = hi + lo with hi = RNE bf16(v), lo = RNE bf16(v - hi), four at a time
__device__ __forceinline__ void split4(float v0, float v1, float v2, float v3, s4 &hi, s4 &lo)
{
    const bf2 h01 = {(__bf16)v0, (__bf16)v1}, h23 = {(__bf16)v2, (__bf16)v3};
    const bf2 l01 = {(__bf16)(v0 - (float)h01[0]), (__bf16)(v1 - (float)h01[1])};
    const bf2 l23 = {(__bf16)(v2 - (float)h23[0]), (__bf16)(v3 - (float)h23[1])};
    const uint2 hu = make_uint2(__builtin_bit_cast(uint32_t, h01), __builtin_bit_cast(uint32_t, h23));
    const uint2 lu = make_uint2(__builtin_bit_cast(uint32_t, l01), __builtin_bit_cast(uint32_t, l23));
    hi = __builtin_bit_cast(s4, hu);
    lo = __builtin_bit_cast(s4, lu);
}
// -x for four packed bf16 values (sign bits)
__device__ __forceinline__ s4 neg4(s4 v)
{
    uint2 u = __builtin_bit_cast(uint2, v);
    u.x ^= 0x80008000u;
    u.y ^= 0x80008000u;
    return __builtin_bit_cast(s4, u);
}
__device__ __forceinline__ s4 ld4(const uint16_t *p) { return *reinterpret_cast<const s4 *>(p); }

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

// One complex unknown of the trial: extrapolate, gradient step, prox
// S_tau(v) = v max(0, 1 - tau/|v|).  Returns x-bar and |x-bar|; shared by the
// trial and the acceptance so that both produce bit-identical values.
__device__ __forceinline__ void trial_one(float x_r, float x_i, float xp_r, float xp_i, float g_r,
                                          float g_i, float gp_r, float gp_i, float beta,
                                          float alpha, float tau, float &y_r, float &y_i,
                                          float &xb_r, float &xb_i, float &axb)
{
    y_r = fmaf(beta, x_r - xp_r, x_r);
    y_i = fmaf(beta, x_i - xp_i, x_i);
    const float gy_r = fmaf(beta, g_r - gp_r, g_r);
    const float gy_i = fmaf(beta, g_i - gp_i, g_i);
    const float v_r = fmaf(-alpha, gy_r, y_r);
    const float v_i = fmaf(-alpha, gy_i, y_i);
    const float m2 = fmaf(v_r, v_r, v_i * v_i);
    const float rs = __builtin_amdgcn_rsqf(m2);
    const bool keep = m2 > tau * tau;          // |v| > tau; 0/0 of the rsq is discarded
    const float sc = keep ? fmaf(-tau, rs, 1.0f) : 0.0f;
    xb_r = v_r * sc;
    xb_i = v_i * sc;
    axb = keep ? fmaf(m2, rs, -tau) : 0.0f;    // |v| - tau
}

// A as the MFMA A operand: LDS copy (row stride ld) or the packed global copy.
struct AView {
    const float2 *p;
    int ld;
    __device__ __forceinline__ f4 load4(int row, int m) const
    {
        return *reinterpret_cast<const f4 *>(p + row * ld + m);
    }
    __device__ __forceinline__ float2 load2(int row, int m) const { return p[row * ld + m]; }
};

}  // namespace fm

// LDS row stride of the staged A (float2 units): l_pad + 2 spreads the rows of
// one load over distinct banks.  Split-BF16 planes: row-major stride l_pad + 4,
// transposed stride 16 T + 4 (bf16 units).
__host__ __device__ inline int fm_lds_ld(int l_pad) { return l_pad + 2; }
__host__ __device__ inline int fm_bf_ldf(int l_pad) { return l_pad + 4; }
__host__ __device__ inline int fm_bf_lda(int rows) { return rows + 4; }
__host__ __device__ inline size_t fm_bf_planes_bytes(int rows, int l_pad)
{
    return ((size_t)4 * rows * fm_bf_ldf(l_pad) + (size_t)4 * l_pad * fm_bf_lda(rows)) * sizeof(uint16_t);
}

template <int T, int KB, bool ALDS, int PREC, int WMAX>
__device__ __forceinline__ void fista_mfma_stack(const FistaArgs &a)
{
    constexpr bool BF = PREC == L1LS_SPLIT_BF16;
    using fm::f4;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int W = a.waves;
    const int j = lane & 15;
    const int h = lane >> 4;
    const int n = a.n;
    const int l = a.l;
    const int rows = 16 * T;

    size_t off = 0;
    float2 *sA = reinterpret_cast<float2 *>(smem);
    // split-BF16 planes [4][rows][ldf] and transposed [4][l_pad][lda]: staged in LDS
    // (ALDS) or read from the workspace copy the setup wrote (L2)
    uint16_t *sF = reinterpret_cast<uint16_t *>(smem);
    uint16_t *sT = sF + (size_t)4 * rows * fm_bf_ldf(a.l_pad);
    const uint16_t *pF = ALDS ? sF : a.Abf, *pT = ALDS ? sT : a.Abf + (size_t)4 * rows * a.l_pad;
    const int ldf = ALDS ? fm_bf_ldf(a.l_pad) : a.l_pad, lda = ALDS ? fm_bf_lda(rows) : rows;
    if (BF && ALDS) off = (fm_bf_planes_bytes(rows, a.l_pad) + 15) & ~(size_t)15;
    else if (ALDS) off = ((size_t)rows * fm_lds_ld(a.l_pad) * sizeof(float2) + 15) & ~(size_t)15;
    f4 *sPW = reinterpret_cast<f4 *>(smem + off);   // [W][2T][64] forward partials
    off += (size_t)W * 2 * T * 64 * sizeof(f4);
    f4 *sPS = reinterpret_cast<f4 *>(smem + off);   // [W][16] per-slot partial scalars
    off += (size_t)W * 16 * sizeof(f4);
    uint32_t *sQ = reinterpret_cast<uint32_t *>(smem + off);
    off += 16;
    // LEAN (128 unknowns a wave): G_{k-1} lives in LDS, one float2 per lane and
    // (block, q) of each wave, and x-bar is recomputed at the acceptance instead
    // of kept; the state then fits the registers of one wave per SIMD
    constexpr bool LEAN = KB >= 8;
    float2 *sGp = reinterpret_cast<float2 *>(smem + off) + (size_t)w * KB * 4 * 64 + lane;
    // ... and each wave's copy of r_{k-1} (every wave holds the whole residual)
    float2 *sRp = reinterpret_cast<float2 *>(smem + off) + (size_t)W * KB * 4 * 64 + (size_t)w * T * 4 * 64 + lane;

    fm::AView Av;
    if constexpr (BF && ALDS) {
        // planes c = 0 re hi, 1 im hi, 2 re lo, 3 im lo
        for (int idx = tid; idx < rows * a.l_pad; idx += blockDim.x) {
            const int row = idx / a.l_pad, m = idx % a.l_pad;
            const float2 v = a.A[(size_t)row * a.l_pad + m];
            const __bf16 rh = (__bf16)v.x, ih = (__bf16)v.y;
            const __bf16 rl = (__bf16)(v.x - (float)rh), il = (__bf16)(v.y - (float)ih);
            const uint16_t pv[4] = {__builtin_bit_cast(uint16_t, rh), __builtin_bit_cast(uint16_t, ih),
                                    __builtin_bit_cast(uint16_t, rl), __builtin_bit_cast(uint16_t, il)};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                sF[((size_t)c * rows + row) * ldf + m] = pv[c];
                sT[((size_t)c * a.l_pad + m) * lda + row] = pv[c];
            }
        }
        __syncthreads();
    } else if (ALDS) {
        const int ld = fm_lds_ld(a.l_pad), half = a.l_pad / 2;
        for (int idx = tid; idx < rows * half; idx += blockDim.x) {
            const int row = idx / half, c2 = idx % half;
            *reinterpret_cast<f4 *>(sA + (size_t)row * ld + 2 * c2) =
                *reinterpret_cast<const f4 *>(a.A + (size_t)row * a.l_pad + 2 * c2);
        }
        Av.p = sA;
        Av.ld = ld;
    } else {
        Av.p = a.A;
        Av.ld = a.l_pad;
    }

    const double lf_d = a.consts->lf;
    const float lf = (float)lf_d;
    const float inv_lf = (float)(1.0 / lf_d);
    const float alpha0 = (float)a.consts->alpha0;
    const float afloor = inv_lf;
    const int m_base = w * 16 * KB;

    float Xr[KB][4], Xi[KB][4], Xpr[KB][4], Xpi[KB][4];
    float Gr[KB][4], Gi[KB][4], Gpr[KB][4], Gpi[KB][4];
    float XBr[KB][4], XBi[KB][4];                      // x-bar of the last trial
    float Rr[T][4], Ri[T][4], Rpr[T][4], Rpi[T][4];    // residual A x - b of x^k, x^{k-1}
#pragma unroll
    for (int b = 0; b < KB; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Xr[b][q] = Xi[b][q] = Xpr[b][q] = Xpi[b][q] = Gr[b][q] = Gi[b][q] = 0.0f;
            if constexpr (LEAN) {
                sGp[(b * 4 + q) * 64] = make_float2(0.0f, 0.0f);
            } else {
                Gpr[b][q] = Gpi[b][q] = XBr[b][q] = XBi[b][q] = 0.0f;
            }
        }
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Rr[t][q] = Ri[t][q] = 0.0f;
            if constexpr (LEAN) sRp[(t * 4 + q) * 64] = make_float2(0.0f, 0.0f);
            else Rpr[t][q] = Rpi[t][q] = 0.0f;
        }

    int64_t pix = -1;
    int k = 1;
    float alpha = alpha0, lam = 1.0f, Fk = 0.0f;
    bool active = false, bad = false, qdone = false;

    // ---- refill the slots in `mask` from the global queue (workgroup-uniform).
    // A fresh slot's state is reset with per-lane selects rather than under a
    // branch, so that the register state is not copied around a divergent join.
    // G needs no reset (the next adjoint overwrites it); everything that enters
    // an extrapolation, even with beta = 0, is cleared so that nothing non-finite
    // of the previous pixel survives.
    // `got`: thread 0's result of the queue atomic for this mask, issued as soon as
    // the retiring slots are known so that its latency hides under the acceptance
    // (the barrier that publishes it is the only one here: the next write of sQ
    // comes after the next trial's barriers).
    unsigned long long n_fwd = 0, n_adj = 0;  // pixel products (thread 0 counts)
    auto refill = [&](uint32_t mask, uint32_t got) {
        if (mask == 0) return;
        const bool mine = (mask >> j) & 1u;
        bool fresh = false;
        bool any_fresh = false;  // workgroup-uniform
        if (!qdone) {
            const uint32_t nfree = __popc(mask);
            if (tid == 0) sQ[0] = got;
            __syncthreads();
            const uint64_t base = sQ[0];
            any_fresh = base < (uint64_t)a.p;
            if (base + nfree >= (uint64_t)a.p) qdone = true;
            const uint64_t np = base + (uint64_t)__popc(mask & ((1u << j) - 1u));
            fresh = mine && np < (uint64_t)a.p;
            if (fresh) pix = (int64_t)np;
        }
        if (mine && !fresh) {
            active = false;
            pix = -1;
        }
        if (fresh) {
            active = true;
            k = 1;
            alpha = alpha0;
            lam = a.lambda[pix * a.lambda_stride];
            bad = !(lam > 0.0f) || !isfinite(lam);
            if (bad) lam = 1.0f;
        }
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Xr[b][q] = fresh ? 0.0f : Xr[b][q];
                Xi[b][q] = fresh ? 0.0f : Xi[b][q];
                Xpr[b][q] = fresh ? 0.0f : Xpr[b][q];
                Xpi[b][q] = fresh ? 0.0f : Xpi[b][q];
                if constexpr (LEAN) {
                    if (fresh) sGp[(b * 4 + q) * 64] = make_float2(0.0f, 0.0f);
                } else {
                    Gpr[b][q] = fresh ? 0.0f : Gpr[b][q];
                    Gpi[b][q] = fresh ? 0.0f : Gpi[b][q];
                }
            }
        float bb = 0.0f;
        const float2 *Bp = a.B + (size_t)(fresh ? pix : 0) * n;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int nn = 16 * t + 4 * h + q;
                const float2 v = fresh && nn < n ? Bp[nn] : make_float2(0.0f, 0.0f);
                Rr[t][q] = fresh ? -v.x : Rr[t][q];
                Ri[t][q] = fresh ? -v.y : Ri[t][q];
                if constexpr (LEAN) {
                    if (fresh) sRp[(t * 4 + q) * 64] = make_float2(-v.x, -v.y);
                } else {
                    Rpr[t][q] = fresh ? -v.x : Rpr[t][q];
                    Rpi[t][q] = fresh ? -v.y : Rpi[t][q];
                }
                bb = fmaf(v.x, v.x, fmaf(v.y, v.y, bb));
            }
        bb = fm::sum_h(bb);
        if (fresh) Fk = bb;
        if (a.warm && any_fresh) {
            // Init of Algorithm 1 from the given x^(0) (in X) for the fresh slots:
            // x^1 = x^0, r_1 = A x^0 - b (one FP32 product from the packed A in
            // global memory, for either precision) and F(x^0) = ||r_1||^2 + lambda ||x^0||_1
            const float2 *Xi0 = a.X + (size_t)(fresh ? pix : 0) * l;
            float l1p = 0.0f;
#pragma unroll
            for (int b = 0; b < KB; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int m = m_base + 16 * b + 4 * h + q;
                    const float2 v = fresh && m < l ? Xi0[m] : make_float2(0.0f, 0.0f);
                    Xr[b][q] = fresh ? v.x : Xr[b][q];
                    Xi[b][q] = fresh ? v.y : Xi[b][q];
                    Xpr[b][q] = Xr[b][q];
                    Xpi[b][q] = Xi[b][q];
                    l1p += fresh ? __builtin_amdgcn_sqrtf(fmaf(v.x, v.x, v.y * v.y)) : 0.0f;
                }
            const fm::AView Ag{a.A, a.l_pad};
            f4 Vr[T], Vi[T];
#pragma unroll
            for (int t = 0; t < T; ++t) Vr[t] = Vi[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                const int m0 = m_base + 16 * b + 4 * h;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const f4 a01 = Ag.load4(16 * t + j, m0), a23 = Ag.load4(16 * t + j, m0 + 2);
                    // W_re += A_re x_re - A_im x_im;  W_im += A_im x_re + A_re x_im
                    Vr[t] = fm::mfma(a01[0], Xr[b][0], Vr[t]);
                    Vr[t] = fm::mfma(a01[1], -Xi[b][0], Vr[t]);
                    Vi[t] = fm::mfma(a01[1], Xr[b][0], Vi[t]);
                    Vi[t] = fm::mfma(a01[0], Xi[b][0], Vi[t]);
                    Vr[t] = fm::mfma(a01[2], Xr[b][1], Vr[t]);
                    Vr[t] = fm::mfma(a01[3], -Xi[b][1], Vr[t]);
                    Vi[t] = fm::mfma(a01[3], Xr[b][1], Vi[t]);
                    Vi[t] = fm::mfma(a01[2], Xi[b][1], Vi[t]);
                    Vr[t] = fm::mfma(a23[0], Xr[b][2], Vr[t]);
                    Vr[t] = fm::mfma(a23[1], -Xi[b][2], Vr[t]);
                    Vi[t] = fm::mfma(a23[1], Xr[b][2], Vi[t]);
                    Vi[t] = fm::mfma(a23[0], Xi[b][2], Vi[t]);
                    Vr[t] = fm::mfma(a23[2], Xr[b][3], Vr[t]);
                    Vr[t] = fm::mfma(a23[3], -Xi[b][3], Vr[t]);
                    Vi[t] = fm::mfma(a23[3], Xr[b][3], Vi[t]);
                    Vi[t] = fm::mfma(a23[2], Xi[b][3], Vi[t]);
                }
            }
            l1p = fm::sum_h(l1p);
            // the same two-stage cross-wave sum as the trial's forward product
#pragma unroll
            for (int t = 0; t < T; ++t) {
                sPW[((size_t)w * 2 * T + 2 * t) * 64 + lane] = Vr[t];
                sPW[((size_t)w * 2 * T + 2 * t + 1) * 64 + lane] = Vi[t];
            }
            if (h == 0) sPS[w * 16 + j] = f4{l1p, 0.0f, 0.0f, 0.0f};
            __syncthreads();
            {
                const int EW = 2 * T * 64, E = EW + 16;
                for (int e = tid; e < E; e += blockDim.x) {
                    if (e < EW) {
                        f4 acc = sPW[e];
                        for (int ww = 1; ww < W; ++ww) acc += sPW[(size_t)ww * EW + e];
                        sPW[e] = acc;
                    } else {
                        f4 acc = sPS[e - EW];
                        for (int ww = 1; ww < W; ++ww) acc[0] += sPS[ww * 16 + e - EW][0];
                        sPS[e - EW] = acc;
                    }
                }
            }
            __syncthreads();
            float rr = 0.0f;
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const f4 wr = sPW[(size_t)(2 * t) * 64 + lane], wi = sPW[(size_t)(2 * t + 1) * 64 + lane];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // rows n >= N: A is zero there, and so is -b
                    const float r_r = wr[q] + Rr[t][q], r_i = wi[q] + Ri[t][q];  // A x0 - b
                    Rr[t][q] = fresh ? r_r : Rr[t][q];
                    Ri[t][q] = fresh ? r_i : Ri[t][q];
                    if constexpr (LEAN) {
                        if (fresh) sRp[(t * 4 + q) * 64] = make_float2(r_r, r_i);
                    } else {
                        Rpr[t][q] = fresh ? r_r : Rpr[t][q];
                        Rpi[t][q] = fresh ? r_i : Rpi[t][q];
                    }
                    rr = fmaf(r_r, r_r, fmaf(r_i, r_i, rr));
                }
            }
            rr = fm::sum_h(rr);
            const float l1 = sPS[j][0];
            __syncthreads();
            if (fresh) Fk = fmaf(lam, l1, rr);
            n_fwd += __popcll(__ballot(fresh && h == 0));
        }
    };

    // ---- G = 2 A^H r for the wave's unknowns (all slots)
    auto adjoint = [&]() {
        if constexpr (BF) {
            fm::s4 rrh[T], rrl[T], rih[T], ril[T];
#pragma unroll
            for (int t = 0; t < T; ++t) {
                fm::split4(2.0f * Rr[t][0], 2.0f * Rr[t][1], 2.0f * Rr[t][2], 2.0f * Rr[t][3], rrh[t], rrl[t]);
                fm::split4(2.0f * Ri[t][0], 2.0f * Ri[t][1], 2.0f * Ri[t][2], 2.0f * Ri[t][3], rih[t], ril[t]);
            }
#pragma unroll
            for (int b = 0; b < KB; ++b) {
                f4 gr = f4{0.0f, 0.0f, 0.0f, 0.0f}, gi = f4{0.0f, 0.0f, 0.0f, 0.0f};
                const int m = m_base + 16 * b + j;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const int n0 = 16 * t + 4 * h;
                    const fm::s4 arh = fm::ld4(pT + ((size_t)0 * a.l_pad + m) * lda + n0);
                    const fm::s4 aih = fm::ld4(pT + ((size_t)1 * a.l_pad + m) * lda + n0);
                    const fm::s4 arl = fm::ld4(pT + ((size_t)2 * a.l_pad + m) * lda + n0);
                    const fm::s4 ail = fm::ld4(pT + ((size_t)3 * a.l_pad + m) * lda + n0);
                    // G_re += A_re (2 r_re) + A_im (2 r_im);  G_im += A_re (2 r_im) - A_im (2 r_re)
                    gr = fm::mfma_bf(arh, rrh[t], gr);
                    gr = fm::mfma_bf(arh, rrl[t], gr);
                    gr = fm::mfma_bf(arl, rrh[t], gr);
                    gr = fm::mfma_bf(aih, rih[t], gr);
                    gr = fm::mfma_bf(aih, ril[t], gr);
                    gr = fm::mfma_bf(ail, rih[t], gr);
                    gi = fm::mfma_bf(arh, rih[t], gi);
                    gi = fm::mfma_bf(arh, ril[t], gi);
                    gi = fm::mfma_bf(arl, rih[t], gi);
                    gi = fm::mfma_bf(aih, fm::neg4(rrh[t]), gi);
                    gi = fm::mfma_bf(aih, fm::neg4(rrl[t]), gi);
                    gi = fm::mfma_bf(ail, fm::neg4(rrh[t]), gi);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    Gr[b][q] = gr[q];
                    Gi[b][q] = gi[q];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            return;
        }
        float r2r[T][4], r2i[T][4], nr2r[T][4];
        if constexpr (!LEAN) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    r2r[t][q] = 2.0f * Rr[t][q];
                    r2i[t][q] = 2.0f * Ri[t][q];
                    nr2r[t][q] = -2.0f * Rr[t][q];
                }
        }
#pragma unroll
        for (int b = 0; b < KB; ++b) {
            f4 gr = f4{0.0f, 0.0f, 0.0f, 0.0f}, gi = f4{0.0f, 0.0f, 0.0f, 0.0f};
            const int m = m_base + 16 * b + j;
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float2 av = Av.load2(16 * t + 4 * h + q, m);
                    // LEAN forms 2 r on the fly (three registers fewer per residual entry)
                    const float pr = LEAN ? 2.0f * Rr[t][q] : r2r[t][q];
                    const float pi = LEAN ? 2.0f * Ri[t][q] : r2i[t][q];
                    const float npr = LEAN ? -2.0f * Rr[t][q] : nr2r[t][q];
                    gr = fm::mfma(av.x, pr, gr);
                    gr = fm::mfma(av.y, pi, gr);
                    gi = fm::mfma(av.x, pi, gi);
                    gi = fm::mfma(av.y, npr, gi);
                }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Gr[b][q] = gr[q];
                Gi[b][q] = gi[q];
            }
        }
    };

    uint32_t qgot = 0;                        // thread 0: queue position for the retiring slots
    refill(0xFFFFu, tid == 0 ? atomicAdd(a.queue, 16u) : 0u);
    if (__ballot(active) == 0) return;
    adjoint();
    n_adj += __popcll(__ballot(active && h == 0));

    for (;;) {
        const float beta = fmaxf(0.0f, (float)(k - 2) / (float)(k + 1));
        bool first = true, retire = false, conv = false, nonfinite = false;
        float kkt = 0.0f, l1 = 0.0f;
        f4 Wr[T], Wi[T];
        // natural KKT residual of x^k with its exact gradient G_k
        float kmax = 0.0f;
        {
            const float tk = lam * inv_lf;
#pragma unroll
            for (int b = 0; b < KB; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float x_r = Xr[b][q], x_i = Xi[b][q];
                    const float v_r = fmaf(-inv_lf, Gr[b][q], x_r);
                    const float v_i = fmaf(-inv_lf, Gi[b][q], x_i);
                    const float m2 = fmaf(v_r, v_r, v_i * v_i);
                    const float sc = m2 > tk * tk ? fmaf(-tk, __builtin_amdgcn_rsqf(m2), 1.0f) : 0.0f;
                    const float e_r = fmaf(-v_r, sc, x_r), e_i = fmaf(-v_i, sc, x_i);
                    kmax = fmaxf(kmax, fmaf(e_r, e_r, e_i * e_i));
                }
            kmax = fm::max_h(kmax);
        }
        for (int trial = 0; trial < 64; ++trial) {
            n_fwd += __popcll(__ballot(active && h == 0));
            const float tau = alpha * lam;
#pragma unroll
            for (int t = 0; t < T; ++t) Wr[t] = Wi[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            float d2 = 0.0f, s1 = 0.0f;
            // element work of block b: extrapolate, gradient step, prox, d = x-bar - y
            float dr[KB][4], di[KB][4];
            auto element_block = [&](int b) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float y_r, y_i, xb_r, xb_i, axb;
                    float gp_r, gp_i;
                    if constexpr (LEAN) {
                        const float2 g2 = sGp[(b * 4 + q) * 64];
                        gp_r = g2.x;
                        gp_i = g2.y;
                    } else {
                        gp_r = Gpr[b][q];
                        gp_i = Gpi[b][q];
                    }
                    fm::trial_one(Xr[b][q], Xi[b][q], Xpr[b][q], Xpi[b][q], Gr[b][q], Gi[b][q],
                                  gp_r, gp_i, beta, alpha, tau, y_r, y_i, xb_r, xb_i, axb);
                    dr[b][q] = xb_r - y_r;
                    di[b][q] = xb_i - y_i;
                    if constexpr (!LEAN) {
                        XBr[b][q] = xb_r;
                        XBi[b][q] = xb_i;
                    }
                    d2 = fmaf(dr[b][q], dr[b][q], fmaf(di[b][q], di[b][q], d2));
                    s1 += axb - __builtin_amdgcn_sqrtf(fmaf(Xr[b][q], Xr[b][q], Xi[b][q] * Xi[b][q]));
                }
            };
            if constexpr (!BF) {
                // software pipeline: block b + 1's element work is interleaved with
                // block b's MFMAs (one wave per SIMD: the VALU work hides under the
                // matrix-core passes instead of following them)
                element_block(0);
#pragma unroll
                for (int b = 0; b < KB; ++b) {
                    const int m0 = m_base + 16 * b + 4 * h;
                    f4 a01[T], a23[T];
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        a01[t] = Av.load4(16 * t + j, m0);      // (re, im) of m0, m0 + 1
                        a23[t] = Av.load4(16 * t + j, m0 + 2);  // (re, im) of m0 + 2, m0 + 3
                    }
                    if (b + 1 < KB) element_block(b + 1);
                    float ndi[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) ndi[q] = -di[b][q];
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        Wr[t] = fm::mfma(a01[t][0], dr[b][0], Wr[t]);
                        Wr[t] = fm::mfma(a01[t][1], ndi[0], Wr[t]);
                        Wi[t] = fm::mfma(a01[t][1], dr[b][0], Wi[t]);
                        Wi[t] = fm::mfma(a01[t][0], di[b][0], Wi[t]);
                        Wr[t] = fm::mfma(a01[t][2], dr[b][1], Wr[t]);
                        Wr[t] = fm::mfma(a01[t][3], ndi[1], Wr[t]);
                        Wi[t] = fm::mfma(a01[t][3], dr[b][1], Wi[t]);
                        Wi[t] = fm::mfma(a01[t][2], di[b][1], Wi[t]);
                        Wr[t] = fm::mfma(a23[t][0], dr[b][2], Wr[t]);
                        Wr[t] = fm::mfma(a23[t][1], ndi[2], Wr[t]);
                        Wi[t] = fm::mfma(a23[t][1], dr[b][2], Wi[t]);
                        Wi[t] = fm::mfma(a23[t][0], di[b][2], Wi[t]);
                        Wr[t] = fm::mfma(a23[t][2], dr[b][3], Wr[t]);
                        Wr[t] = fm::mfma(a23[t][3], ndi[3], Wr[t]);
                        Wi[t] = fm::mfma(a23[t][3], dr[b][3], Wi[t]);
                        Wi[t] = fm::mfma(a23[t][2], di[b][3], Wi[t]);
                    }
                    if (b + 1 < KB) {
                        // 16 T MFMAs with the next block's element work between them
#pragma unroll
                        for (int u = 0; u < 16 * T; ++u) {
                            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                            __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);  // then up to 6 VALU
                        }
                    }
                }
            } else {
#pragma unroll
                for (int b = 0; b < KB; ++b) {
                    element_block(b);
                    const int m0 = m_base + 16 * b + 4 * h;
                    fm::s4 drh, drl, dih, dil;
                    fm::split4(dr[b][0], dr[b][1], dr[b][2], dr[b][3], drh, drl);
                    fm::split4(di[b][0], di[b][1], di[b][2], di[b][3], dih, dil);
                    const fm::s4 ndih = fm::neg4(dih), ndil = fm::neg4(dil);
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        const int row = 16 * t + j;
                        const fm::s4 arh = fm::ld4(pF + ((size_t)0 * rows + row) * ldf + m0);
                        const fm::s4 aih = fm::ld4(pF + ((size_t)1 * rows + row) * ldf + m0);
                        const fm::s4 arl = fm::ld4(pF + ((size_t)2 * rows + row) * ldf + m0);
                        const fm::s4 ail = fm::ld4(pF + ((size_t)3 * rows + row) * ldf + m0);
                        // W_re += A_re d_re + A_im (-d_im);  W_im += A_im d_re + A_re d_im
                        Wr[t] = fm::mfma_bf(arh, drh, Wr[t]);
                        Wr[t] = fm::mfma_bf(arh, drl, Wr[t]);
                        Wr[t] = fm::mfma_bf(arl, drh, Wr[t]);
                        Wr[t] = fm::mfma_bf(aih, ndih, Wr[t]);
                        Wr[t] = fm::mfma_bf(aih, ndil, Wr[t]);
                        Wr[t] = fm::mfma_bf(ail, ndih, Wr[t]);
                        Wi[t] = fm::mfma_bf(aih, drh, Wi[t]);
                        Wi[t] = fm::mfma_bf(aih, drl, Wi[t]);
                        Wi[t] = fm::mfma_bf(ail, drh, Wi[t]);
                        Wi[t] = fm::mfma_bf(arh, dih, Wi[t]);
                        Wi[t] = fm::mfma_bf(arh, dil, Wi[t]);
                        Wi[t] = fm::mfma_bf(arl, dih, Wi[t]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // cross-wave reduction of the forward partial products and scalars
            d2 = fm::sum_h(d2);
            s1 = fm::sum_h(s1);
#pragma unroll
            for (int t = 0; t < T; ++t) {
                sPW[((size_t)w * 2 * T + 2 * t) * 64 + lane] = Wr[t];
                sPW[((size_t)w * 2 * T + 2 * t + 1) * 64 + lane] = Wi[t];
            }
            if (h == 0) sPS[w * 16 + j] = f4{d2, s1, kmax, 0.0f};
            __syncthreads();
            // two stages: each thread sums one entry over the waves (in wave order,
            // into wave 0's slot), then every wave reads the sums
            {
                const int EW = 2 * T * 64, E = EW + 16;
                for (int e = tid; e < E; e += blockDim.x) {
                    if (e < EW) {
                        f4 acc = sPW[e];
                        for (int ww = 1; ww < W; ++ww) acc += sPW[(size_t)ww * EW + e];
                        sPW[e] = acc;
                    } else {
                        f4 acc = sPS[e - EW];
                        for (int ww = 1; ww < W; ++ww) {
                            const f4 ps = sPS[ww * 16 + e - EW];
                            acc[0] += ps[0];
                            acc[1] += ps[1];
                            acc[2] = fmaxf(acc[2], ps[2]);
                        }
                        sPS[e - EW] = acc;
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < T; ++t) {
                Wr[t] = sPW[(size_t)(2 * t) * 64 + lane];
                Wi[t] = sPW[(size_t)(2 * t + 1) * 64 + lane];
            }
            const f4 S = sPS[j];
            __syncthreads();
            float w2 = 0.0f;
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) w2 = fmaf(Wr[t][q], Wr[t][q], fmaf(Wi[t][q], Wi[t][q], w2));
            w2 = fm::sum_h(w2);
            if (first) {
                kkt = lf * sqrtf(S[2]) / lam;
                nonfinite = !isfinite(kkt) || !isfinite(Fk);
                conv = kkt <= a.tol;
                const bool capped = (k - 1) >= a.fista_cap;
                retire = active && (bad || nonfinite || conv || capped);
                {
                    const uint32_t rm = (uint32_t)(__ballot(retire && h == 0) & 0xFFFFull);
                    if (tid == 0 && rm != 0u && !qdone) qgot = atomicAdd(a.queue, (uint32_t)__popc(rm));
                }
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
                        const uint32_t slot = atomicAdd(a.polish_count, 1u);
                        a.polish_list[slot] = (int32_t)pix;
                    }
                }
                first = false;
            }
            l1 = S[1];
            float d2s = S[0];
            bool jumped = false;
            if (k == 1 && trial == 0 && !a.warm && active && !retire && a.backtracking &&
                w2 > d2s / (2.0f * alpha) && alpha > afloor) {
                // First iteration: y = x^0 = 0, so x-bar(alpha) = alpha S_lambda(-G_0) is linear
                // in alpha and Eq. (15) reads alpha <= ||d||^2 / (2 ||A d||^2) at every alpha.
                // The shrink sequence alpha0 C^i therefore ends where this one product
                // says, and d, A d, ||x-bar||_1 scale with alpha: no further products.
                const float rho = d2s / (2.0f * w2);
                float an = alpha;
                while (an > rho && an > afloor) an = fmaxf(a.c_alpha * an, afloor);
                const float c = an / alpha;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    Wr[t] *= c;
                    Wi[t] *= c;
                }
                if constexpr (!LEAN) {
                    // (LEAN recomputes x-bar at the acceptance with the final step)
#pragma unroll
                    for (int b = 0; b < KB; ++b)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            XBr[b][q] *= c;
                            XBi[b][q] *= c;
                        }
                }
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

        // ---- retire: write x^k of the wave's unknowns (and, from wave 0, its residual)
        if (retire && a.R && w == 0) {
            float2 *Ro = a.R + (size_t)pix * n;
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int nn = 16 * t + 4 * h + q;
                    if (nn < n) Ro[nn] = make_float2(Rr[t][q], Ri[t][q]);
                }
        }
        if (retire) {
            float2 *Xo = a.X + (size_t)pix * l;
#pragma unroll
            for (int b = 0; b < KB; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int m = m_base + 16 * b + 4 * h + q;
                    if (m < l) Xo[m] = make_float2(Xr[b][q], Xi[b][q]);
                }
        }

        // ---- monotone acceptance and state rotation (live slots)
        {
            // residual of x-bar: r(y) + A d, with r(y) = r_k + beta (r_k - r_{k-1})
            float dfr = 0.0f;
            float Rbr[T][4], Rbi[T][4];
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float rp_r, rp_i;
                    if constexpr (LEAN) {
                        const float2 r2 = sRp[(t * 4 + q) * 64];
                        rp_r = r2.x;
                        rp_i = r2.y;
                    } else {
                        rp_r = Rpr[t][q];
                        rp_i = Rpi[t][q];
                    }
                    const float dr_r = fmaf(beta, Rr[t][q] - rp_r, Wr[t][q]);
                    const float dr_i = fmaf(beta, Ri[t][q] - rp_i, Wi[t][q]);
                    Rbr[t][q] = Rr[t][q] + dr_r;
                    Rbi[t][q] = Ri[t][q] + dr_i;
                    dfr = fmaf(dr_r, Rbr[t][q] + Rr[t][q], fmaf(dr_i, Rbi[t][q] + Ri[t][q], dfr));
                }
            dfr = fm::sum_h(dfr);
            const float dF = fmaf(lam, l1, dfr);
            const bool live = active && !retire;
            const bool accept = live && (!a.monotone || dF <= 0.0f);
#pragma unroll
            for (int b = 0; b < KB; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if constexpr (LEAN) {
                        // x-bar of the last trial, recomputed from the same inputs (the
                        // jump of the first iteration: at its final step)
                        const float2 g2 = sGp[(b * 4 + q) * 64];
                        float y_r, y_i, xb_r, xb_i, axb;
                        fm::trial_one(Xr[b][q], Xi[b][q], Xpr[b][q], Xpi[b][q], Gr[b][q], Gi[b][q], g2.x,
                                      g2.y, beta, alpha, alpha * lam, y_r, y_i, xb_r, xb_i, axb);
                        if (live) {
                            Xpr[b][q] = Xr[b][q];
                            Xpi[b][q] = Xi[b][q];
                            sGp[(b * 4 + q) * 64] = make_float2(Gr[b][q], Gi[b][q]);
                        }
                        if (accept) {
                            Xr[b][q] = xb_r;
                            Xi[b][q] = xb_i;
                        }
                    } else {
                        if (live) {
                            Xpr[b][q] = Xr[b][q];
                            Xpi[b][q] = Xi[b][q];
                            Gpr[b][q] = Gr[b][q];
                            Gpi[b][q] = Gi[b][q];
                        }
                        if (accept) {
                            Xr[b][q] = XBr[b][q];
                            Xi[b][q] = XBi[b][q];
                        }
                    }
                }
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (live) {
                        if constexpr (LEAN) {
                            sRp[(t * 4 + q) * 64] = make_float2(Rr[t][q], Ri[t][q]);
                        } else {
                            Rpr[t][q] = Rr[t][q];
                            Rpi[t][q] = Ri[t][q];
                        }
                    }
                    if (accept) {
                        Rr[t][q] = Rbr[t][q];
                        Ri[t][q] = Rbi[t][q];
                    }
                }
            if (accept) Fk += dF;
            if (live) ++k;
        }

        // ---- refill retired slots, stop when the tile is empty
        const uint32_t rmask = (uint32_t)(__ballot(retire && h == 0) & 0xFFFFull);
        if (retire) active = false;
        refill(rmask, qgot);
        if (__ballot(active) == 0) break;
        adjoint();
        n_adj += __popcll(__ballot(active && h == 0));
    }
    if (tid == 0) {
        atomicAdd(&a.work[0], n_fwd);
        atomicAdd(&a.work[1], n_adj);
    }
}



// The stacks of a table one after another: a workgroup takes 16-pixel tiles of a
// stack from that stack's queue until it is empty and its own tile has drained,
// then stages the next stack's A.  Every stack of the table has this tiling
// (same T, KB and waves, hence the same padded L and LDS size).
template <int T, int KB, bool ALDS, int PREC, int WMAX>
__global__ void __launch_bounds__(64 * WMAX) fista_mfma_kernel(const StackTable t)
{
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        FistaArgs a = fista_args_for(t.d[i], t.o);
        a.waves = blockDim.x / 64;
        fista_mfma_stack<T, KB, ALDS, PREC, WMAX>(a);
        __syncthreads();
    }
}

template <int T, int KB, bool ALDS, int PREC, int WMAX>
hipError_t launch_mfma_one(const StackTable &t, int waves, hipStream_t s)
{
    if (waves < 1 || waves > WMAX) return hipErrorInvalidConfiguration;
    int64_t need = 0;
    for (int i = 0; i < t.count; ++i) {
        const StackDesc &d = t.d[i];
        if (d.p <= 0) continue;
        if (waves * 16 * KB != lpad_for(d.l) || rows_pad_for(d.n) != 16 * T) return hipErrorInvalidConfiguration;
        need += (d.p + kTile - 1) / kTile;
    }
    if (need == 0) return hipSuccess;
    const size_t lds = fista_mfma_lds_bytes(16 * T, waves * 16 * KB, waves, ALDS, PREC);
    auto kern = fista_mfma_kernel<T, KB, ALDS, PREC, WMAX>;
    static bool attr_done = false;  // per instantiation
    if (!attr_done) {
        hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
        attr_done = true;
    }
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * waves, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t groups = (int64_t)per_cu * cus;
    if (groups > need) groups = need;
    if (groups < 1) groups = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(64 * waves), lds, s, t);
    return hipGetLastError();
}

}  // namespace l1ls
