// Matrix-core tile form of the unrolled fixed-step map and its adjoint (complex
// L1LS of arXiv 1805.01759, Eqs. (11)-(12) with a constant step alpha, no
// backtracking, no monotone test).  Same map, same adjoint and the same tape
// semantics as the wave-per-pixel kernels in unrolled.hip; used for N <= 32,
// L <= 256.
//
// A workgroup owns 16 pixel slots and W <= 4 waves; the register layout is the
// one of the FP32 iteration kernel (lane (j, h) holds unknowns m = 64 w + 16 b +
// 4 h + q and residual rows n = 16 t + 4 h + q of pixel j, real and imaginary
// parts apart), A and A diag(s) are staged in LDS zero-padded to 16 T rows.
//
// Forward step k (beta_k = max(0, (k-2)/(k+1)), tau = alpha lambda):
//   r_y = r_x + beta (r_x - r_xp)          residuals of x^{k-1}, x^{k-2} (A linear)
//   g   = 2 A^H r_y                        (per wave, all of n)
//   y   = x + beta (x - xp),  v = y - alpha g,  x^k = S_tau(v)
//   r_x <- A x^k - b                       (per-wave partials reduced through LDS)
// so each step is one adjoint and one forward product on the matrix cores, and a
// checkpoint holds (x, xp, r_x, r_xp).  The reverse sweep of a segment, after
// recomputing it from its checkpoint with the same routine (bit-identical), is
//   v-bar = S'(v)^T x-bar,  lambda-bar -= alpha Re(conj(u) x-bar) on |v| > tau
//   w = A v-bar (reduced),  b-bar += 2 alpha w
//   xi-bar_n += -2 alpha Re[conj(r_y,n) (dA v-bar)_n + conj(w_n) (dA y)_n],
//     dA = d A / d xi_n = -j 2 pi A diag(s): (dA u)_n = 2 pi (Im, -Re)(A diag(s) u)_n,
//     linear in the A diag(s) products, so each wave adds the term of its own
//     partial products and the waves are summed once per pixel
//   y-bar = v-bar - 2 alpha A^H w,  x-bar^{k-1} = x-bar_{k-2 slot} + (1 + beta) y-bar,
//   x-bar^{k-2} = -beta y-bar
#include "fista_mfma.h"

namespace l1ls {
namespace {

using fm::f4;
constexpr int UKB = 4;  // blocks of 16 unknowns per wave (64 unknowns)

struct UTileArgs {
    int n, l, l_pad, waves, K, ckpt;
    int64_t p;
    const float2 *A, *As;  // n x l (A and A diag(s))
    const float2 *B;
    float lambda, alpha;
    float2 *X;             // forward output, p x l
    float2 *ck;            // checkpoints, p x (K/ckpt - 1) x (2 l + 2 n)
    const float2 *dX;
    float2 *dB;
    float *part;           // per pixel [lambda-bar, xi-bar_0..n-1]
    float4 *seg;           // per workgroup: ckpt x W x CH x 64 float4 records
};

// LDS row stride (float2) of the staged matrices
__host__ __device__ inline int u_ld(int l_pad) { return l_pad + 2; }

template <int T>
struct UCtx {
    const float2 *sA, *sAs;
    int ld;
    f4 *sPW;  // [W][2T][64]
    int tid, lane, w, W, j, h, m_base;
};

// stage M (n x l) into LDS as 16 T x ld, zero padded
template <int T>
__device__ void u_stage(const float2 *M, float2 *dst, int n, int l, int l_pad, int ld)
{
    for (int idx = threadIdx.x; idx < 16 * T * l_pad; idx += blockDim.x) {
        const int row = idx / l_pad, c = idx % l_pad;
        dst[row * ld + c] = (row < n && c < l) ? M[(size_t)row * l + c] : make_float2(0.0f, 0.0f);
    }
}

// partial forward products of one block b: Wr/Wi[t] += M[n = 16 t + j][m0 .. m0 + 3] u
template <int T>
__device__ __forceinline__ void u_fwd_block(const float2 *M, int ld, int j, int m0, const float (&ur)[4],
                                            const float (&ui)[4], f4 (&Wr)[T], f4 (&Wi)[T])
{
    float nui[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) nui[q] = -ui[q];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const f4 a01 = *reinterpret_cast<const f4 *>(M + (16 * t + j) * ld + m0);
        const f4 a23 = *reinterpret_cast<const f4 *>(M + (16 * t + j) * ld + m0 + 2);
        // X_re += M_re u_re - M_im u_im;  X_im += M_im u_re + M_re u_im
        Wr[t] = fm::mfma(a01[0], ur[0], Wr[t]);
        Wr[t] = fm::mfma(a01[1], nui[0], Wr[t]);
        Wi[t] = fm::mfma(a01[1], ur[0], Wi[t]);
        Wi[t] = fm::mfma(a01[0], ui[0], Wi[t]);
        Wr[t] = fm::mfma(a01[2], ur[1], Wr[t]);
        Wr[t] = fm::mfma(a01[3], nui[1], Wr[t]);
        Wi[t] = fm::mfma(a01[3], ur[1], Wi[t]);
        Wi[t] = fm::mfma(a01[2], ui[1], Wi[t]);
        Wr[t] = fm::mfma(a23[0], ur[2], Wr[t]);
        Wr[t] = fm::mfma(a23[1], nui[2], Wr[t]);
        Wi[t] = fm::mfma(a23[1], ur[2], Wi[t]);
        Wi[t] = fm::mfma(a23[0], ui[2], Wi[t]);
        Wr[t] = fm::mfma(a23[2], ur[3], Wr[t]);
        Wr[t] = fm::mfma(a23[3], nui[3], Wr[t]);
        Wi[t] = fm::mfma(a23[3], ur[3], Wi[t]);
        Wi[t] = fm::mfma(a23[2], ui[3], Wi[t]);
    }
}

// 2 A^H r for block b (rows m = m_base + 16 b + j of A^H), r given per lane rows
template <int T>
__device__ __forceinline__ void u_adj_block(const float2 *M, int ld, int h, int m, const float (&rr)[T][4],
                                            const float (&ri)[T][4], f4 &gr, f4 &gi)
{
    gr = f4{0.0f, 0.0f, 0.0f, 0.0f};
    gi = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float2 av = M[(16 * t + 4 * h + q) * ld + m];
            const float r2r = 2.0f * rr[t][q], r2i = 2.0f * ri[t][q];
            // G_re += A_re r_re + A_im r_im;  G_im += A_re r_im - A_im r_re
            gr = fm::mfma(av.x, r2r, gr);
            gr = fm::mfma(av.y, r2i, gr);
            gi = fm::mfma(av.x, r2i, gi);
            gi = fm::mfma(av.y, -r2r, gi);
        }
}

// sum of the W waves' partial products (all waves end with the total)
template <int T>
__device__ __forceinline__ void u_reduce(const UCtx<T> &c, f4 (&Wr)[T], f4 (&Wi)[T])
{
#pragma unroll
    for (int t = 0; t < T; ++t) {
        c.sPW[((size_t)c.w * 2 * T + 2 * t) * 64 + c.lane] = Wr[t];
        c.sPW[((size_t)c.w * 2 * T + 2 * t + 1) * 64 + c.lane] = Wi[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < T; ++t) Wr[t] = Wi[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int ww = 0; ww < c.W; ++ww) {
#pragma unroll
        for (int t = 0; t < T; ++t) {
            Wr[t] += c.sPW[((size_t)ww * 2 * T + 2 * t) * 64 + c.lane];
            Wi[t] += c.sPW[((size_t)ww * 2 * T + 2 * t + 1) * 64 + c.lane];
        }
    }
    __syncthreads();
}

// float4 records per lane and step: y and v (UKB x 4 complex each, re and im
// apart: 4 UKB chunks) and r_y (T x 4 complex: 2 T chunks)
template <int T>
__host__ __device__ constexpr int u_chunks() { return 4 * UKB + 2 * T; }

// One forward step k; rec != nullptr records (y, v, r_y) of this step.
template <int T>
__device__ void u_step(const UCtx<T> &c, const UTileArgs &a, int k, float (&Xr)[UKB][4],
                       float (&Xi)[UKB][4], float (&Xpr)[UKB][4], float (&Xpi)[UKB][4],
                       float (&Rr)[T][4], float (&Ri)[T][4], float (&Rpr)[T][4], float (&Rpi)[T][4],
                       const float (&Br)[T][4], const float (&Bi)[T][4], float4 *rec)
{
    const float beta = fmaxf(0.0f, (float)(k - 2) / (float)(k + 1));
    const float tau = a.alpha * a.lambda;
    float yr[T][4], yi[T][4];  // r_y
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            yr[t][q] = fmaf(beta, Rr[t][q] - Rpr[t][q], Rr[t][q]);
            yi[t][q] = fmaf(beta, Ri[t][q] - Rpi[t][q], Ri[t][q]);
        }
    f4 Wr[T], Wi[T];
#pragma unroll
    for (int t = 0; t < T; ++t) Wr[t] = Wi[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int b = 0; b < UKB; ++b) {
        f4 gr, gi;
        u_adj_block<T>(c.sA, c.ld, c.h, c.m_base + 16 * b + c.j, yr, yi, gr, gi);
        float nr[4], ni[4], vr4[4], vi4[4], yr4[4], yi4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float y_r = fmaf(beta, Xr[b][q] - Xpr[b][q], Xr[b][q]);
            const float y_i = fmaf(beta, Xi[b][q] - Xpi[b][q], Xi[b][q]);
            const float v_r = fmaf(-a.alpha, gr[q], y_r), v_i = fmaf(-a.alpha, gi[q], y_i);
            const float m = sqrtf(v_r * v_r + v_i * v_i);
            const float sc = m > tau ? 1.0f - tau / m : 0.0f;
            nr[q] = v_r * sc;
            ni[q] = v_i * sc;
            vr4[q] = v_r;
            vi4[q] = v_i;
            yr4[q] = y_r;
            yi4[q] = y_i;
            Xpr[b][q] = Xr[b][q];
            Xpi[b][q] = Xi[b][q];
            Xr[b][q] = nr[q];
            Xi[b][q] = ni[q];
        }
        if (rec) {
            rec[(2 * b) * 64 + c.lane] = make_float4(yr4[0], yr4[1], yr4[2], yr4[3]);
            rec[(2 * b + 1) * 64 + c.lane] = make_float4(yi4[0], yi4[1], yi4[2], yi4[3]);
            rec[(2 * UKB + 2 * b) * 64 + c.lane] = make_float4(vr4[0], vr4[1], vr4[2], vr4[3]);
            rec[(2 * UKB + 2 * b + 1) * 64 + c.lane] = make_float4(vi4[0], vi4[1], vi4[2], vi4[3]);
        }
        u_fwd_block<T>(c.sA, c.ld, c.j, c.m_base + 16 * b + 4 * c.h, nr, ni, Wr, Wi);
    }
    if (rec) {
#pragma unroll
        for (int t = 0; t < T; ++t) {
            rec[(4 * UKB + 2 * t) * 64 + c.lane] = make_float4(yr[t][0], yr[t][1], yr[t][2], yr[t][3]);
            rec[(4 * UKB + 2 * t + 1) * 64 + c.lane] = make_float4(yi[t][0], yi[t][1], yi[t][2], yi[t][3]);
        }
    }
    u_reduce<T>(c, Wr, Wi);
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Rpr[t][q] = Rr[t][q];
            Rpi[t][q] = Ri[t][q];
            Rr[t][q] = Wr[t][q] - Br[t][q];
            Ri[t][q] = Wi[t][q] - Bi[t][q];
        }
}

template <int T>
__device__ UCtx<T> u_ctx(const UTileArgs &a, unsigned char *smem, bool with_as)
{
    UCtx<T> c;
    c.tid = threadIdx.x;
    c.lane = c.tid & 63;
    c.w = c.tid >> 6;
    c.W = a.waves;
    c.j = c.lane & 15;
    c.h = c.lane >> 4;
    c.m_base = 64 * c.w;
    c.ld = u_ld(a.l_pad);
    const size_t mat = ((size_t)16 * T * c.ld * sizeof(float2) + 15) & ~(size_t)15;
    float2 *sA = reinterpret_cast<float2 *>(smem);
    float2 *sAs = reinterpret_cast<float2 *>(smem + mat);
    c.sA = sA;
    c.sAs = sAs;
    c.sPW = reinterpret_cast<f4 *>(smem + (with_as ? 2 : 1) * mat);
    u_stage<T>(a.A, sA, a.n, a.l, a.l_pad, c.ld);
    if (with_as) u_stage<T>(a.As, sAs, a.n, a.l, a.l_pad, c.ld);
    __syncthreads();
    return c;
}

template <int T>
__device__ void u_load_b(const UTileArgs &a, const UCtx<T> &c, int64_t pix, float (&Br)[T][4],
                         float (&Bi)[T][4])
{
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int nn = 16 * t + 4 * c.h + q;
            const float2 v = (pix < a.p && nn < a.n) ? a.B[(size_t)pix * a.n + nn] : make_float2(0.0f, 0.0f);
            Br[t][q] = v.x;
            Bi[t][q] = v.y;
        }
}

}  // namespace

template <int T>
__global__ void __launch_bounds__(256) unrolled_fwd_tile_kernel(const UTileArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const UCtx<T> c = u_ctx<T>(a, smem, false);
    const int nck = a.K / a.ckpt;
    const int64_t tiles = (a.p + 15) / 16;
    const size_t cks = (size_t)2 * a.l + 2 * a.n;  // checkpoint stride (complex)
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t pix = tile * 16 + c.j;
        float Br[T][4], Bi[T][4];
        u_load_b<T>(a, c, pix, Br, Bi);
        float Xr[UKB][4], Xi[UKB][4], Xpr[UKB][4], Xpi[UKB][4];
        float Rr[T][4], Ri[T][4], Rpr[T][4], Rpi[T][4];
#pragma unroll
        for (int b = 0; b < UKB; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) Xr[b][q] = Xi[b][q] = Xpr[b][q] = Xpi[b][q] = 0.0f;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Rr[t][q] = Rpr[t][q] = -Br[t][q];
                Ri[t][q] = Rpi[t][q] = -Bi[t][q];
            }
        for (int k = 1; k <= a.K; ++k) {
            u_step<T>(c, a, k, Xr, Xi, Xpr, Xpi, Rr, Ri, Rpr, Rpi, Br, Bi, nullptr);
            if (k % a.ckpt == 0 && k / a.ckpt < nck && pix < a.p) {
                // checkpoint: (x, xp, r_x, r_xp) before step k + 1
                float2 *t = a.ck + ((size_t)pix * (nck - 1) + (k / a.ckpt - 1)) * cks;
#pragma unroll
                for (int b = 0; b < UKB; ++b)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int m = c.m_base + 16 * b + 4 * c.h + q;
                        if (m < a.l) {
                            t[m] = make_float2(Xr[b][q], Xi[b][q]);
                            t[a.l + m] = make_float2(Xpr[b][q], Xpi[b][q]);
                        }
                    }
                if (c.w == 0) {
#pragma unroll
                    for (int tt = 0; tt < T; ++tt)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int nn = 16 * tt + 4 * c.h + q;
                            if (nn < a.n) {
                                t[2 * a.l + nn] = make_float2(Rr[tt][q], Ri[tt][q]);
                                t[2 * a.l + a.n + nn] = make_float2(Rpr[tt][q], Rpi[tt][q]);
                            }
                        }
                }
            }
        }
        if (pix < a.p) {
            float2 *xo = a.X + (size_t)pix * a.l;
#pragma unroll
            for (int b = 0; b < UKB; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int m = c.m_base + 16 * b + 4 * c.h + q;
                    if (m < a.l) xo[m] = make_float2(Xr[b][q], Xi[b][q]);
                }
        }
    }
}

template <int T>
__global__ void __launch_bounds__(256) unrolled_bwd_tile_kernel(const UTileArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const UCtx<T> c = u_ctx<T>(a, smem, true);
    const int nck = a.K / a.ckpt;
    const int64_t tiles = (a.p + 15) / 16;
    const size_t cks = (size_t)2 * a.l + 2 * a.n;
    constexpr int CH = u_chunks<T>();
    float4 *segw = a.seg + (size_t)blockIdx.x * a.ckpt * c.W * CH * 64;  // this workgroup's records
    const float tau = a.alpha * a.lambda;
    const float two_a = 2.0f * a.alpha;
    const float twopi = 6.283185307179586f;
    // per-pixel partial sums over the waves: [W][16][1 + 16 T] floats, after sPW
    float *sRed = reinterpret_cast<float *>(c.sPW + (size_t)c.W * 2 * T * 64);
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t pix = tile * 16 + c.j;
        float Br[T][4], Bi[T][4];
        u_load_b<T>(a, c, pix, Br, Bi);
        float Ar1[UKB][4], Ai1[UKB][4], Ar0[UKB][4], Ai0[UKB][4];  // x-bar of x^k, x^{k-1}
#pragma unroll
        for (int b = 0; b < UKB; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = c.m_base + 16 * b + 4 * c.h + q;
                const float2 d = (pix < a.p && m < a.l) ? a.dX[(size_t)pix * a.l + m] : make_float2(0.0f, 0.0f);
                Ar1[b][q] = d.x;
                Ai1[b][q] = d.y;
                Ar0[b][q] = Ai0[b][q] = 0.0f;
            }
        float lamb = 0.0f;
        float xib[T][4], bbr[T][4], bbi[T][4];
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) xib[t][q] = bbr[t][q] = bbi[t][q] = 0.0f;
        for (int sg = nck - 1; sg >= 0; --sg) {
            const int k0 = sg * a.ckpt;
            float Xr[UKB][4], Xi[UKB][4], Xpr[UKB][4], Xpi[UKB][4];
            float Rr[T][4], Ri[T][4], Rpr[T][4], Rpi[T][4];
            if (sg == 0) {
#pragma unroll
                for (int b = 0; b < UKB; ++b)
#pragma unroll
                    for (int q = 0; q < 4; ++q) Xr[b][q] = Xi[b][q] = Xpr[b][q] = Xpi[b][q] = 0.0f;
#pragma unroll
                for (int t = 0; t < T; ++t)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        Rr[t][q] = Rpr[t][q] = -Br[t][q];
                        Ri[t][q] = Rpi[t][q] = -Bi[t][q];
                    }
            } else {
                const float2 *t0 = a.ck + ((size_t)(pix < a.p ? pix : 0) * (nck - 1) + (sg - 1)) * cks;
#pragma unroll
                for (int b = 0; b < UKB; ++b)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int m = c.m_base + 16 * b + 4 * c.h + q;
                        const bool ok = pix < a.p && m < a.l;
                        const float2 x = ok ? t0[m] : make_float2(0.0f, 0.0f);
                        const float2 xp = ok ? t0[a.l + m] : make_float2(0.0f, 0.0f);
                        Xr[b][q] = x.x;
                        Xi[b][q] = x.y;
                        Xpr[b][q] = xp.x;
                        Xpi[b][q] = xp.y;
                    }
#pragma unroll
                for (int t = 0; t < T; ++t)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int nn = 16 * t + 4 * c.h + q;
                        const bool ok = pix < a.p && nn < a.n;
                        const float2 r = ok ? t0[2 * a.l + nn] : make_float2(-Br[t][q], -Bi[t][q]);
                        const float2 rp = ok ? t0[2 * a.l + a.n + nn] : make_float2(-Br[t][q], -Bi[t][q]);
                        Rr[t][q] = r.x;
                        Ri[t][q] = r.y;
                        Rpr[t][q] = rp.x;
                        Rpi[t][q] = rp.y;
                    }
            }
            // recompute the segment, recording (y, v, r_y) of every step
            for (int qs = 0; qs < a.ckpt; ++qs) {
                float4 *rec = segw + ((size_t)qs * c.W + c.w) * CH * 64;
                u_step<T>(c, a, k0 + qs + 1, Xr, Xi, Xpr, Xpi, Rr, Ri, Rpr, Rpi, Br, Bi, rec);
            }
            // reverse sweep over the segment
            for (int qs = a.ckpt - 1; qs >= 0; --qs) {
                const int k = k0 + qs + 1;
                const float beta = fmaxf(0.0f, (float)(k - 2) / (float)(k + 1));
                const float4 *rec = segw + ((size_t)qs * c.W + c.w) * CH * 64;
                float vbr[UKB][4], vbi[UKB][4];
                f4 Wr[T], Wi[T], Pr[T], Pi[T], Qr[T], Qi[T];
#pragma unroll
                for (int t = 0; t < T; ++t)
                    Wr[t] = Wi[t] = Pr[t] = Pi[t] = Qr[t] = Qi[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int b = 0; b < UKB; ++b) {
                    const float4 y_r = rec[(2 * b) * 64 + c.lane], y_i = rec[(2 * b + 1) * 64 + c.lane];
                    const float4 v_r = rec[(2 * UKB + 2 * b) * 64 + c.lane];
                    const float4 v_i = rec[(2 * UKB + 2 * b + 1) * 64 + c.lane];
                    const float yr4[4] = {y_r.x, y_r.y, y_r.z, y_r.w}, yi4[4] = {y_i.x, y_i.y, y_i.z, y_i.w};
                    const float vr4[4] = {v_r.x, v_r.y, v_r.z, v_r.w}, vi4[4] = {v_i.x, v_i.y, v_i.z, v_i.w};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        // v-bar through the prox
                        const float m = sqrtf(vr4[q] * vr4[q] + vi4[q] * vi4[q]);
                        const float Wx = Ar1[b][q], Wy = Ai1[b][q];
                        float br = 0.0f, bi = 0.0f;
                        if (m > tau) {
                            const float ur = vr4[q] / m, ui = vi4[q] / m, cc = tau / m;
                            const float rad = ur * Wx + ui * Wy;  // Re(conj(u) W)
                            br = (1.0f - cc) * Wx + cc * rad * ur;
                            bi = (1.0f - cc) * Wy + cc * rad * ui;
                            lamb -= a.alpha * rad;
                        }
                        vbr[b][q] = br;
                        vbi[b][q] = bi;
                    }
                    const int m0 = c.m_base + 16 * b + 4 * c.h;
                    u_fwd_block<T>(c.sA, c.ld, c.j, m0, vbr[b], vbi[b], Wr, Wi);
                    u_fwd_block<T>(c.sAs, c.ld, c.j, m0, vbr[b], vbi[b], Pr, Pi);
                    u_fwd_block<T>(c.sAs, c.ld, c.j, m0, yr4, yi4, Qr, Qi);
                }
                u_reduce<T>(c, Wr, Wi);  // w = A v-bar, complete
                float ryr[T][4], ryi[T][4];
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const float4 rr = rec[(4 * UKB + 2 * t) * 64 + c.lane];
                    const float4 ri = rec[(4 * UKB + 2 * t + 1) * 64 + c.lane];
                    ryr[t][0] = rr.x; ryr[t][1] = rr.y; ryr[t][2] = rr.z; ryr[t][3] = rr.w;
                    ryi[t][0] = ri.x; ryi[t][1] = ri.y; ryi[t][2] = ri.z; ryi[t][3] = ri.w;
                }
#pragma unroll
                for (int t = 0; t < T; ++t)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        // (dA u)_n = -j 2 pi (A S u)_n = 2 pi (Im, -Re) of this wave's partial
                        const float dvr = twopi * Pi[t][q], dvi = -twopi * Pr[t][q];
                        const float dyr = twopi * Qi[t][q], dyi = -twopi * Qr[t][q];
                        xib[t][q] += -two_a * (ryr[t][q] * dvr + ryi[t][q] * dvi + Wr[t][q] * dyr + Wi[t][q] * dyi);
                        bbr[t][q] += two_a * Wr[t][q];
                        bbi[t][q] += two_a * Wi[t][q];
                    }
                float wr[T][4], wi[T][4];
#pragma unroll
                for (int t = 0; t < T; ++t)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        wr[t][q] = Wr[t][q];
                        wi[t][q] = Wi[t][q];
                    }
#pragma unroll
                for (int b = 0; b < UKB; ++b) {
                    f4 hr, hi;  // 2 A^H w
                    u_adj_block<T>(c.sA, c.ld, c.h, c.m_base + 16 * b + c.j, wr, wi, hr, hi);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float ybr = fmaf(-a.alpha, hr[q], vbr[b][q]);
                        const float ybi = fmaf(-a.alpha, hi[q], vbi[b][q]);
                        const float o_r = Ar0[b][q], o_i = Ai0[b][q];
                        Ar1[b][q] = fmaf(1.0f + beta, ybr, o_r);
                        Ai1[b][q] = fmaf(1.0f + beta, ybi, o_i);
                        Ar0[b][q] = -beta * ybr;
                        Ai0[b][q] = -beta * ybi;
                    }
                }
            }
        }
        // per-pixel outputs: the waves' partials of lambda-bar and xi-bar summed in LDS
        const float lam_px = fm::sum_h(lamb);
        float *red = sRed + (size_t)c.w * 16 * (1 + 16 * T);
        if (c.h == 0) red[c.j * (1 + 16 * T)] = lam_px;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[c.j * (1 + 16 * T) + 1 + 16 * t + 4 * c.h + q] = xib[t][q];
        __syncthreads();
        for (int e = c.tid; e < 16 * (1 + 16 * T); e += blockDim.x) {
            const int jj = e / (1 + 16 * T), col = e % (1 + 16 * T);
            const int64_t pp = tile * 16 + jj;
            if (pp >= a.p || (col > 0 && col - 1 >= a.n)) continue;
            float acc = 0.0f;
            for (int ww = 0; ww < c.W; ++ww) acc += sRed[(size_t)ww * 16 * (1 + 16 * T) + e];
            a.part[(size_t)pp * (a.n + 1) + col] = acc;
        }
        if (c.w == 0 && pix < a.p) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int nn = 16 * t + 4 * c.h + q;
                    if (nn < a.n) a.dB[(size_t)pix * a.n + nn] = make_float2(bbr[t][q], bbi[t][q]);
                }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host side

bool unrolled_tile_supports(int n, int l) { return n <= 32 && l <= 256; }

static int u_waves(int l) { return (l + 63) / 64; }

static size_t u_lds(int n, int l, bool with_as)
{
    const int T = (n + 15) / 16, W = u_waves(l), l_pad = 64 * W;
    const size_t mat = ((size_t)16 * T * u_ld(l_pad) * sizeof(float2) + 15) & ~(size_t)15;
    size_t b = (with_as ? 2 : 1) * mat + (size_t)W * 2 * T * 64 * sizeof(f4);
    if (with_as) b += (size_t)W * 16 * (1 + 16 * T) * sizeof(float);
    return b;
}

// record bytes of one backward workgroup (ckpt steps)
size_t unrolled_tile_seg_bytes(int n, int l, int ckpt)
{
    const int T = (n + 15) / 16, W = u_waves(l);
    const int CH = T == 1 ? u_chunks<1>() : u_chunks<2>();
    return (size_t)ckpt * W * CH * 64 * sizeof(float4);
}

template <int T>
static hipError_t u_launch(bool fwd, const UTileArgs &a, int64_t groups, hipStream_t st)
{
    const size_t lds = u_lds(a.n, a.l, !fwd);
    if (fwd) {
        hipFuncSetAttribute((const void *)unrolled_fwd_tile_kernel<T>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        hipLaunchKernelGGL(unrolled_fwd_tile_kernel<T>, dim3((unsigned)groups), dim3(64 * a.waves), lds, st, a);
    } else {
        hipFuncSetAttribute((const void *)unrolled_bwd_tile_kernel<T>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        hipLaunchKernelGGL(unrolled_bwd_tile_kernel<T>, dim3((unsigned)groups), dim3(64 * a.waves), lds, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_unrolled_tile(bool forward, int n, int l, int64_t p, const float2 *A, const float2 *As,
                                const float2 *B, float lambda, float alpha, int K, int ckpt, float2 *X,
                                float2 *ck, const float2 *dX, float2 *dB, float *part, void *seg,
                                int64_t max_groups, hipStream_t st)
{
    UTileArgs a{};
    a.n = n;
    a.l = l;
    a.waves = u_waves(l);
    a.l_pad = 64 * a.waves;
    a.K = K;
    a.ckpt = ckpt;
    a.p = p;
    a.A = A;
    a.As = As;
    a.B = B;
    a.lambda = lambda;
    a.alpha = alpha;
    a.X = X;
    a.ck = ck;
    a.dX = dX;
    a.dB = dB;
    a.part = part;
    a.seg = (float4 *)seg;
    const int64_t tiles = (p + 15) / 16;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t groups = forward ? (int64_t)cus * 2 : (int64_t)cus;
    if (max_groups > 0 && groups > max_groups) groups = max_groups;
    if (groups > tiles) groups = tiles;
    if (groups < 1) groups = 1;
    return (n + 15) / 16 == 1 ? u_launch<1>(forward, a, groups, st) : u_launch<2>(forward, a, groups, st);
}

}  // namespace l1ls
