// Streamed MFMA form of the accelerated proximal-gradient iteration (complex
// L1LS of arXiv 1805.01759, Algorithm 1 with one block, J = 1): up to 128 rows
// (T <= 8 blocks of 16) and up to 1,024 bins, FP32 or split-BF16 contractions.
//
// The arithmetic is that of the register tile (fista_mfma.h), operation for
// operation: the split re/im v_mfma_f32_16x16x4f32 contractions with A as the A
// operand (split-BF16: the three-pass v_mfma_f32_16x16x16bf16_1k forms on the
// bf16 planes of A the setup writes, read from L2), the element step of one
// unknown (fm::trial_one), the Eq. (15) test
// on ||A d||^2 <= ||d||^2 / (2 alpha), the monotone acceptance formed from
// differences, the one-product step jump of the first iteration and the warm
// start.  The four waves of a workgroup take contiguous runs of 16-unknown
// blocks, as the register tile's waves do, so that where both tiles exist they
// give bit-identical results.
//
// What differs is where the iterate lives.  A tile of 16 pixel slots keeps its
// iterates and gradients in a workspace slot of its own (two x arrays and three
// G arrays, l_pad x 640 bytes: 640 KB at 1,024 bins, more than a CU's registers
// and LDS together), streamed one block (16 unknowns x 16 slots, 2 KB an array)
// at a time.  The acceptance of iteration k only decides (from the residuals,
// which stay on chip); x^{k+1} is formed in the first trial pass of iteration
// k + 1, which recomputes x-bar of iteration k from the same inputs:
//   trial       reads x^k, x^{k-1}, G_{k+1}, G_k, G_{k-1}; writes x^{k+1} over
//               x^{k-1}; forms d = x-bar - y and A d for iteration k + 1
//   adjoint     writes G_{k+1} = 2 A^H r_{k+1} over G_{k-2}
// (five reads and two writes an iteration; a repeated trial of Eq. (15) reads
// the four arrays of its own iteration).  The x arrays are a pair and the G
// arrays a ring of three, addressed per slot, so no rotation moves data.  Within a block, lane
// (j = lane % 16, h = lane / 16) holds unknowns 16 b + 4 h + q, q = 0..3, of
// slot j, the output layout of the MFMA; the lane's four complex values are
// 32 contiguous bytes, so a wave reads or writes one array's block as 2 KB.
// The residual r_k (N complex a slot) stays in every wave's registers and
// r_{k-1} in LDS; A is read from the packed copy (L2).
#pragma once
#include "fista_mfma.h"

namespace l1ls {

constexpr int kStreamWaves = 4;

// LDS of the streamed tile: forward partials [W][2T][64] f4, per-slot scalars
// [W][16] f4, the queue word, and each wave's r_{k-1} ([W][T][4][64] float2).
__host__ __device__ inline size_t fista_stream_lds_bytes_t(int T)
{
    return (size_t)kStreamWaves * 2 * T * 64 * 16 + (size_t)kStreamWaves * 16 * 16 + 16 +
           (size_t)kStreamWaves * T * 4 * 64 * 8;
}

namespace fs {

// Block b of array `arr` (0, 1: the x pair; 2, 3: the G pair) in a tile's state:
// the lane's four complex values (32 bytes).
__device__ __forceinline__ fm::f4 *blk(float2 *st, int NB, int arr, int b, int lane)
{
    return reinterpret_cast<fm::f4 *>(st + ((size_t)(arr * NB + b) * 64 + lane) * 4);
}
__device__ __forceinline__ void ld_blk(const fm::f4 *p, float (&re)[4], float (&im)[4])
{
    const fm::f4 v0 = p[0], v1 = p[1];
    re[0] = v0[0];
    im[0] = v0[1];
    re[1] = v0[2];
    im[1] = v0[3];
    re[2] = v1[0];
    im[2] = v1[1];
    re[3] = v1[2];
    im[3] = v1[3];
}
__device__ __forceinline__ void st_blk(fm::f4 *p, const float (&re)[4], const float (&im)[4])
{
    p[0] = fm::f4{re[0], im[0], re[1], im[1]};
    p[1] = fm::f4{re[2], im[2], re[3], im[3]};
}

}  // namespace fs

template <int T, int PREC>
__device__ __forceinline__ void fista_stream_stack(const FistaArgs &a, float2 *st)
{
    constexpr bool BF = PREC == L1LS_SPLIT_BF16;
    using fm::f4;
    constexpr int W = kStreamWaves;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int j = lane & 15;
    const int h = lane >> 4;
    const int n = a.n;
    const int l = a.l;
    const int NB = a.l_pad / 16;
    // wave w's blocks: a contiguous run, as the register tile splits the unknowns
    const int NBW = (NB + W - 1) / W;
    const int b_lo = w * NBW, b_hi = b_lo + NBW < NB ? b_lo + NBW : NB;

    size_t off = 0;
    f4 *sPW = reinterpret_cast<f4 *>(smem);  // [W][2T][64] forward partials
    off += (size_t)W * 2 * T * 64 * sizeof(f4);
    f4 *sPS = reinterpret_cast<f4 *>(smem + off);  // [W][16] per-slot partial scalars
    off += (size_t)W * 16 * sizeof(f4);
    uint32_t *sQ = reinterpret_cast<uint32_t *>(smem + off);
    off += 16;
    float2 *sRp = reinterpret_cast<float2 *>(smem + off) + (size_t)w * T * 4 * 64 + lane;  // r_{k-1}

    const fm::AView Av{a.A, a.l_pad};
    // split-BF16 planes of A (re hi, im hi, re lo, im lo): row-major [4][rows][l_pad]
    // for the forward product, transposed [4][l_pad][rows] for the adjoint
    const int rows = 16 * T;
    const uint16_t *pF = a.Abf, *pT = a.Abf + (size_t)4 * rows * a.l_pad;
    const double lf_d = a.consts->lf;
    const float lf = (float)lf_d;
    const float inv_lf = (float)(1.0 / lf_d);
    const float alpha0 = (float)a.consts->alpha0;
    const float afloor = inv_lf;

    float Rr[T][4], Ri[T][4];  // residual A x^k - b
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Rr[t][q] = Ri[t][q] = 0.0f;
            sRp[(t * 4 + q) * 64] = make_float2(0.0f, 0.0f);
        }

    int64_t pix = -1;
    // per slot: iteration k; xs, the x array holding the stored iterate (x^k, or
    // x^{k-1} while the acceptance of iteration k-1 is pending), the other holding
    // the one before; rot, the G array (of 2 + 0..2) holding G_k, (rot + 2) % 3
    // G_{k-1} and (rot + 1) % 3 G_{k-2}; pend, acc, beta_p: the pending acceptance
    int k = 1, xs = 0, rot = 0;
    bool pend = false, acc = false;
    float beta_p = 0.0f;
    float alpha = alpha0, lam = 1.0f, Fk = 0.0f;
    bool active = false, bad = false, qdone = false;
    unsigned long long n_fwd = 0, n_adj = 0;

    // Cross-wave sum of the forward partials (into Wr, Wi) and of the per-slot
    // scalars (components 0, 1 summed, 2 the maximum), in wave order.
    auto reduce = [&](f4 (&Wr)[T], f4 (&Wi)[T], f4 sc) -> f4 {
#pragma unroll
        for (int t = 0; t < T; ++t) {
            sPW[((size_t)w * 2 * T + 2 * t) * 64 + lane] = Wr[t];
            sPW[((size_t)w * 2 * T + 2 * t + 1) * 64 + lane] = Wi[t];
        }
        if (h == 0) sPS[w * 16 + j] = sc;
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
        return S;
    };

    // A operands of block b for the forward product (issued ahead of the element
    // work that forms d, so that their L2 latency hides under it)
    auto fwd_load = [&](int b, f4 (&a01)[T], f4 (&a23)[T]) {
        const int m0 = 16 * b + 4 * h;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            a01[t] = Av.load4(16 * t + j, m0);      // (re, im) of m0, m0 + 1
            a23[t] = Av.load4(16 * t + j, m0 + 2);  // (re, im) of m0 + 2, m0 + 3
        }
    };
    // W += A d for one block of complex d (the register tile's order of products)
    auto fwd_mfma = [&](const f4 (&a01)[T], const f4 (&a23)[T], const float (&dr)[4], const float (&di)[4],
                        f4 (&Wr)[T], f4 (&Wi)[T]) {
        float ndi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) ndi[q] = -di[q];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            Wr[t] = fm::mfma(a01[t][0], dr[0], Wr[t]);
            Wr[t] = fm::mfma(a01[t][1], ndi[0], Wr[t]);
            Wi[t] = fm::mfma(a01[t][1], dr[0], Wi[t]);
            Wi[t] = fm::mfma(a01[t][0], di[0], Wi[t]);
            Wr[t] = fm::mfma(a01[t][2], dr[1], Wr[t]);
            Wr[t] = fm::mfma(a01[t][3], ndi[1], Wr[t]);
            Wi[t] = fm::mfma(a01[t][3], dr[1], Wi[t]);
            Wi[t] = fm::mfma(a01[t][2], di[1], Wi[t]);
            Wr[t] = fm::mfma(a23[t][0], dr[2], Wr[t]);
            Wr[t] = fm::mfma(a23[t][1], ndi[2], Wr[t]);
            Wi[t] = fm::mfma(a23[t][1], dr[2], Wi[t]);
            Wi[t] = fm::mfma(a23[t][0], di[2], Wi[t]);
            Wr[t] = fm::mfma(a23[t][2], dr[3], Wr[t]);
            Wr[t] = fm::mfma(a23[t][3], ndi[3], Wr[t]);
            Wi[t] = fm::mfma(a23[t][3], dr[3], Wi[t]);
            Wi[t] = fm::mfma(a23[t][2], di[3], Wi[t]);
        }
    };
    // split-BF16: the four bf16 planes of A for block b (row 16 t + j, bins m0..m0+3)
    auto bf_load = [&](int b, fm::s4 (&af)[T][4]) {
        const int m0 = 16 * b + 4 * h;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c) af[t][c] = fm::ld4(pF + ((size_t)c * rows + 16 * t + j) * a.l_pad + m0);
    };
    // W += A d in three bf16 passes (hi hi + hi lo + lo hi), the register tile's order
    auto bf_mfma = [&](const fm::s4 (&af)[T][4], const float (&dr)[4], const float (&di)[4], f4 (&Wr)[T],
                       f4 (&Wi)[T]) {
        fm::s4 drh, drl, dih, dil;
        fm::split4(dr[0], dr[1], dr[2], dr[3], drh, drl);
        fm::split4(di[0], di[1], di[2], di[3], dih, dil);
        const fm::s4 ndih = fm::neg4(dih), ndil = fm::neg4(dil);
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const fm::s4 arh = af[t][0], aih = af[t][1], arl = af[t][2], ail = af[t][3];
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
    };

    // ---- refill the slots in `mask` from the global queue (workgroup-uniform);
    // `got` is thread 0's queue atomic for this mask.  A fresh slot starts at
    // x^1 = x^0 (0, or the given point), with x^0 and G_0 = 0 in the other arrays
    // of the pairs (beta is 0 for k = 1, 2, but nothing non-finite of the previous
    // pixel may survive into the extrapolation).
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
            xs = 0;
            rot = 0;
            pend = false;
            alpha = alpha0;
            lam = a.lambda[pix * a.lambda_stride];
            bad = !(lam > 0.0f) || !isfinite(lam);
            if (bad) lam = 1.0f;
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
                if (fresh) sRp[(t * 4 + q) * 64] = make_float2(-v.x, -v.y);
                bb = fmaf(v.x, v.x, fmaf(v.y, v.y, bb));
            }
        bb = fm::sum_h(bb);
        if (fresh) Fk = bb;
        if (!any_fresh) return;
        const float zero[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (!a.warm) {
            if (fresh) {
                for (int b = b_lo; b < b_hi; ++b) {
                    fs::st_blk(fs::blk(st, NB, 0, b, lane), zero, zero);
                    fs::st_blk(fs::blk(st, NB, 1, b, lane), zero, zero);
                    fs::st_blk(fs::blk(st, NB, 4, b, lane), zero, zero);
                }
            }
            return;
        }
        // Init of Algorithm 1 from the given x^(0) (in X) for the fresh slots:
        // x^1 = x^0, r_1 = A x^0 - b, F(x^0) = ||r_1||^2 + lambda ||x^0||_1
        const float2 *Xi0 = a.X + (size_t)(fresh ? pix : 0) * l;
        float l1p = 0.0f;
        f4 Vr[T], Vi[T];
#pragma unroll
        for (int t = 0; t < T; ++t) Vr[t] = Vi[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int b = b_lo; b < b_hi; ++b) {
            float xr[4], xi[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = 16 * b + 4 * h + q;
                const float2 v = fresh && m < l ? Xi0[m] : make_float2(0.0f, 0.0f);
                xr[q] = fresh ? v.x : 0.0f;
                xi[q] = fresh ? v.y : 0.0f;
                l1p += fresh ? __builtin_amdgcn_sqrtf(fmaf(v.x, v.x, v.y * v.y)) : 0.0f;
            }
            if (fresh) {
                fs::st_blk(fs::blk(st, NB, 0, b, lane), xr, xi);
                fs::st_blk(fs::blk(st, NB, 1, b, lane), xr, xi);
                fs::st_blk(fs::blk(st, NB, 4, b, lane), zero, zero);
            }
            // W_re += A_re x_re - A_im x_im;  W_im += A_im x_re + A_re x_im
            f4 a01[T], a23[T];
            fwd_load(b, a01, a23);
            fwd_mfma(a01, a23, xr, xi, Vr, Vi);
        }
        l1p = fm::sum_h(l1p);
        const f4 S = reduce(Vr, Vi, f4{l1p, 0.0f, 0.0f, 0.0f});
        float rr = 0.0f;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // rows n >= N: A is zero there, and so is -b
                const float r_r = Vr[t][q] + Rr[t][q], r_i = Vi[t][q] + Ri[t][q];  // A x0 - b
                Rr[t][q] = fresh ? r_r : Rr[t][q];
                Ri[t][q] = fresh ? r_i : Ri[t][q];
                if (fresh) sRp[(t * 4 + q) * 64] = make_float2(r_r, r_i);
                rr = fmaf(r_r, r_r, fmaf(r_i, r_i, rr));
            }
        rr = fm::sum_h(rr);
        if (fresh) Fk = fmaf(lam, S[0], rr);
        n_fwd += __popcll(__ballot(fresh && h == 0));
    };

    // ---- G_k = 2 A^H r_k for the wave's blocks (all slots), into G array `rot`
    // (a block's A operands are all issued before its products)
    auto adj_load = [&](int b, float2 (&av)[T][4]) {
        const int m = 16 * b + j;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) av[t][q] = Av.load2(16 * t + 4 * h + q, m);
    };
    auto adjoint = [&]() {
        if constexpr (BF) {
            // 2 r split once into bf16 hi and lo parts, then per block the transposed
            // planes of A (bins 16 b + j, rows 16 t + 4 h .. + 3)
            fm::s4 rrh[T], rrl[T], rih[T], ril[T];
#pragma unroll
            for (int t = 0; t < T; ++t) {
                fm::split4(2.0f * Rr[t][0], 2.0f * Rr[t][1], 2.0f * Rr[t][2], 2.0f * Rr[t][3], rrh[t], rrl[t]);
                fm::split4(2.0f * Ri[t][0], 2.0f * Ri[t][1], 2.0f * Ri[t][2], 2.0f * Ri[t][3], rih[t], ril[t]);
            }
            for (int b = b_lo; b < b_hi; ++b) {
                const int m = 16 * b + j;
                fm::s4 ap[T][4];
#pragma unroll
                for (int t = 0; t < T; ++t)
#pragma unroll
                    for (int c = 0; c < 4; ++c) ap[t][c] = fm::ld4(pT + ((size_t)c * a.l_pad + m) * rows + 16 * t + 4 * h);
                __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
                f4 gr = f4{0.0f, 0.0f, 0.0f, 0.0f}, gi = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const fm::s4 arh = ap[t][0], aih = ap[t][1], arl = ap[t][2], ail = ap[t][3];
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
                const float g_r[4] = {gr[0], gr[1], gr[2], gr[3]}, g_i[4] = {gi[0], gi[1], gi[2], gi[3]};
                fs::st_blk(fs::blk(st, NB, 2 + rot, b, lane), g_r, g_i);
            }
            return;
        }
        for (int b = b_lo; b < b_hi; ++b) {
            float2 av[T][4];
            adj_load(b, av);
            __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
            f4 gr = f4{0.0f, 0.0f, 0.0f, 0.0f}, gi = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // G_re += A_re (2 r_re) + A_im (2 r_im);  G_im += A_re (2 r_im) - A_im (2 r_re)
                    const float pr = 2.0f * Rr[t][q], pi = 2.0f * Ri[t][q], npr = -2.0f * Rr[t][q];
                    gr = fm::mfma(av[t][q].x, pr, gr);
                    gr = fm::mfma(av[t][q].y, pi, gr);
                    gi = fm::mfma(av[t][q].x, pi, gi);
                    gi = fm::mfma(av[t][q].y, npr, gi);
                }
            const float g_r[4] = {gr[0], gr[1], gr[2], gr[3]}, g_i[4] = {gi[0], gi[1], gi[2], gi[3]};
            fs::st_blk(fs::blk(st, NB, 2 + rot, b, lane), g_r, g_i);
        }
    };

    uint32_t qgot = 0;  // thread 0: queue position for the retiring slots
    refill(0xFFFFu, tid == 0 ? atomicAdd(a.queue, 16u) : 0u);
    if (__ballot(active) == 0) return;
    adjoint();
    n_adj += __popcll(__ballot(active && h == 0));

    for (;;) {
        const float beta = fmaxf(0.0f, (float)(k - 2) / (float)(k + 1));
        bool first = true, retire = false, conv = false, nonfinite = false;
        float kkt = 0.0f, l1 = 0.0f;
        f4 Wr[T], Wi[T];
        const int gs = 2 + rot, gps = 2 + (rot == 0 ? 2 : rot - 1), gqs = 2 + (rot == 2 ? 0 : rot + 1);
        for (int trial = 0; trial < 64; ++trial) {
            const bool anyp = __ballot(pend) != 0;  // wave-uniform: a slot's lanes agree
            n_fwd += __popcll(__ballot(active && h == 0));
            const float tau = alpha * lam;
            const float tk = lam * inv_lf;
#pragma unroll
            for (int t = 0; t < T; ++t) Wr[t] = Wi[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            float d2 = 0.0f, s1 = 0.0f, kmax = 0.0f;
            for (int b = b_lo; b < b_hi; ++b) {
                f4 a01[T], a23[T];
                fm::s4 af[T][4];
                if constexpr (BF) bf_load(b, af);
                else fwd_load(b, a01, a23);
                float x_r[4], x_i[4], xp_r[4], xp_i[4], g_r[4], g_i[4], gp_r[4], gp_i[4];
                fs::ld_blk(fs::blk(st, NB, xs, b, lane), x_r, x_i);
                fs::ld_blk(fs::blk(st, NB, 1 - xs, b, lane), xp_r, xp_i);
                fs::ld_blk(fs::blk(st, NB, gs, b, lane), g_r, g_i);
                fs::ld_blk(fs::blk(st, NB, gps, b, lane), gp_r, gp_i);
                if (anyp) {
                    // the pending acceptance of iteration k - 1: its x-bar recomputed from
                    // x^{k-1}, x^{k-2}, G_{k-1}, G_{k-2} with its step, and x^k (x-bar if
                    // accepted, else x^{k-1}) stored over x^{k-2}
                    float gq_r[4] = {0.0f, 0.0f, 0.0f, 0.0f}, gq_i[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    if (pend) fs::ld_blk(fs::blk(st, NB, gqs, b, lane), gq_r, gq_i);
                    float o_r[4], o_i[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float y_r, y_i, xb_r, xb_i, axb;
                        fm::trial_one(x_r[q], x_i[q], xp_r[q], xp_i[q], gp_r[q], gp_i[q], gq_r[q], gq_i[q],
                                      beta_p, alpha, alpha * lam, y_r, y_i, xb_r, xb_i, axb);
                        o_r[q] = acc ? xb_r : x_r[q];
                        o_i[q] = acc ? xb_i : x_i[q];
                    }
                    if (pend) {
                        fs::st_blk(fs::blk(st, NB, 1 - xs, b, lane), o_r, o_i);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            xp_r[q] = x_r[q];
                            xp_i[q] = x_i[q];
                            x_r[q] = o_r[q];
                            x_i[q] = o_i[q];
                        }
                    }
                }
                if (trial == 0) {
                    // natural KKT residual of x^k with its exact gradient G_k
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float v_r = fmaf(-inv_lf, g_r[q], x_r[q]);
                        const float v_i = fmaf(-inv_lf, g_i[q], x_i[q]);
                        const float m2 = fmaf(v_r, v_r, v_i * v_i);
                        const float sc = m2 > tk * tk ? fmaf(-tk, __builtin_amdgcn_rsqf(m2), 1.0f) : 0.0f;
                        const float e_r = fmaf(-v_r, sc, x_r[q]), e_i = fmaf(-v_i, sc, x_i[q]);
                        kmax = fmaxf(kmax, fmaf(e_r, e_r, e_i * e_i));
                    }
                }
                // extrapolate, gradient step, prox, d = x-bar - y
                float dr[4], di[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float y_r, y_i, xb_r, xb_i, axb;
                    fm::trial_one(x_r[q], x_i[q], xp_r[q], xp_i[q], g_r[q], g_i[q], gp_r[q], gp_i[q], beta,
                                  alpha, tau, y_r, y_i, xb_r, xb_i, axb);
                    dr[q] = xb_r - y_r;
                    di[q] = xb_i - y_i;
                    d2 = fmaf(dr[q], dr[q], fmaf(di[q], di[q], d2));
                    s1 += axb - __builtin_amdgcn_sqrtf(fmaf(x_r[q], x_r[q], x_i[q] * x_i[q]));
                }
                if constexpr (BF) bf_mfma(af, dr, di, Wr, Wi);
                else fwd_mfma(a01, a23, dr, di, Wr, Wi);
            }
            if (pend) {  // x^k is stored now
                xs ^= 1;
                pend = false;
            }
            d2 = fm::sum_h(d2);
            s1 = fm::sum_h(s1);
            if (trial == 0) kmax = fm::max_h(kmax);
            const f4 S = reduce(Wr, Wi, f4{d2, s1, kmax, 0.0f});
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
                    uint32_t stt = 0;
                    if (bad) stt |= L1LS_PX_BAD_LAMBDA;
                    else if (nonfinite) stt |= L1LS_PX_NONFINITE;
                    else if (!conv) stt |= L1LS_PX_MAX_ITER;
                    a.status[pix] = stt;
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
                // in alpha and Eq. (15) reads alpha <= ||d||^2 / (2 ||A d||^2) at every alpha:
                // the shrink sequence alpha0 C^i ends where this one product says.
                const float rho = d2s / (2.0f * w2);
                float an = alpha;
                while (an > rho && an > afloor) an = fmaxf(a.c_alpha * an, afloor);
                const float c = an / alpha;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    Wr[t] *= c;
                    Wi[t] *= c;
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

        // ---- retire: write x^k (and, from wave 0, its residual)
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
        if (__ballot(retire) != 0) {
            float2 *Xo = a.X + (size_t)(retire ? pix : 0) * l;
            for (int b = b_lo; b < b_hi; ++b) {
                if (!retire) continue;
                float x_r[4], x_i[4];
                fs::ld_blk(fs::blk(st, NB, xs, b, lane), x_r, x_i);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int m = 16 * b + 4 * h + q;
                    if (m < l) Xo[m] = make_float2(x_r[q], x_i[q]);
                }
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
                    const float2 r2 = sRp[(t * 4 + q) * 64];
                    const float dr_r = fmaf(beta, Rr[t][q] - r2.x, Wr[t][q]);
                    const float dr_i = fmaf(beta, Ri[t][q] - r2.y, Wi[t][q]);
                    Rbr[t][q] = Rr[t][q] + dr_r;
                    Rbi[t][q] = Ri[t][q] + dr_i;
                    dfr = fmaf(dr_r, Rbr[t][q] + Rr[t][q], fmaf(dr_i, Rbi[t][q] + Ri[t][q], dfr));
                }
            dfr = fm::sum_h(dfr);
            const float dF = fmaf(lam, l1, dfr);
            const bool live = active && !retire;
            const bool accept = live && (!a.monotone || dF <= 0.0f);
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (live) sRp[(t * 4 + q) * 64] = make_float2(Rr[t][q], Ri[t][q]);
                    if (accept) {
                        Rr[t][q] = Rbr[t][q];
                        Ri[t][q] = Rbi[t][q];
                    }
                }
            if (accept) Fk += dF;
            if (live) {
                // x^{k+1} is formed in the next trial pass (the step and the decision
                // are kept); G_{k+1} goes over G_{k-2}
                pend = true;
                acc = accept;
                beta_p = beta;
                ++k;
                rot = rot == 2 ? 0 : rot + 1;
            }
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

// The stacks of a table one after another (every stack of the table has T row
// blocks).  Workgroup g uses state slot g of the stack's region, which holds
// stream_groups_for(p) slots: the workgroups beyond that (more than the stack
// has tiles) leave the stack to the others.
template <int T, int PREC>
__global__ void __launch_bounds__(64 * kStreamWaves) __attribute__((amdgpu_waves_per_eu(T <= 4 ? 2 : 1)))
fista_stream_kernel(const StackTable t)
{
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        if ((int64_t)blockIdx.x >= stream_groups_for(t.d[i].p)) continue;
        const FistaArgs a = fista_args_for(t.d[i], t.o);
        float2 *st = a.fstate + (size_t)blockIdx.x * (stream_tile_bytes(a.l_pad) / sizeof(float2));
        fista_stream_stack<T, PREC>(a, st);
        __syncthreads();
    }
}

template <int T, int PREC>
hipError_t launch_stream_t(const StackTable &t, hipStream_t s)
{
    int64_t need = 0;
    for (int i = 0; i < t.count; ++i) {
        const StackDesc &d = t.d[i];
        if (d.p <= 0) continue;
        if (rows_pad_for(d.n) != 16 * T || lpad_for(d.l) % 16 != 0) return hipErrorInvalidConfiguration;
        const int64_t g = stream_groups_for(d.p);
        if (g > need) need = g;
    }
    if (need == 0) return hipSuccess;
    const size_t lds = fista_stream_lds_bytes_t(T);
    auto kern = fista_stream_kernel<T, PREC>;
    static bool attr_done = false;  // per instantiation
    if (!attr_done) {
        hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_done = true;
    }
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * kStreamWaves, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t groups = (int64_t)per_cu * cus;
    if (groups > need) groups = need;
    if (groups < 1) groups = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(64 * kStreamWaves), lds, s, t);
    return hipGetLastError();
}

}  // namespace l1ls
