// Setup kernel (packing, Lipschitz constant, alpha0) and the dispatch from
// (N, L, precision) to the instantiated persistent iteration kernels.
#include <algorithm>

#include "l1ls_internal.h"

namespace l1ls {

template <int T, int KB, bool ALDS, int PREC, int WMAX>
hipError_t launch_mfma_one(const StackTable &t, int waves, hipStream_t s);
size_t fm_bf_planes_bytes_host(int rows, int l_pad);
hipError_t launch_wave_table(const StackTable &t, int nc, hipStream_t s);
int wave_chunks(int l);

__device__ __forceinline__ int rows_pad_for_dev(int n) { return 16 * ((n + 15) / 16); }

// ---------------------------------------------------------------------------
// Setup, three launches on the caller's stream:
//   setup_pack_kernel   (grid)    A packed zero-padded to rows_pad_for(n) x l_pad, and
//                                 its transpose l_pad x n
//   setup_gram_kernel   (grid)    FP64 Gram M = A A^H, one entry per thread
//   setup_power_kernel  (1 group) queue/counter reset, alpha0 = 1/(2 max_l ||a_l||^2),
//                                 L_f = 2 lambda_max(M) by FP64 power iteration on
//                                 M^(2^kSquarings), the Rayleigh quotient taken on M
// Pointers of stack blockIdx.y's setup inputs and outputs.
struct SetupView {
    int n, l, l_pad;
    const float2 *A;
    float2 *Ap, *At;
    uint16_t *Abf;
    double2 *gram, *H;
    StackConsts *consts;
    uint32_t *queue;
    unsigned long long *work;
};
__device__ inline SetupView setup_view(const StackDesc &d)
{
    const StackWorkspace lay = stack_workspace_layout(d.n, d.l, d.p);
    SetupView v;
    v.n = d.n;
    v.l = d.l;
    v.l_pad = lpad_for(d.l);
    v.A = d.A;
    v.Ap = (float2 *)(d.ws + lay.a_packed);
    v.At = (float2 *)(d.ws + lay.a_trans);
    v.Abf = (uint16_t *)(d.ws + lay.a_bf16);
    v.gram = (double2 *)(d.ws + lay.gram);
    v.H = (double2 *)(d.ws + lay.hgram);
    v.consts = (StackConsts *)(d.ws + lay.consts);
    v.queue = (uint32_t *)(d.ws + lay.queue);
    v.work = (unsigned long long *)(d.ws + lay.work);
    return v;
}

__global__ void __launch_bounds__(256) setup_pack_kernel(const StackTable t)
{
    if (t.d[blockIdx.y].p <= 0) return;
    const SetupView sv = setup_view(t.d[blockIdx.y]);
    const int n = sv.n, l = sv.l, l_pad = sv.l_pad;
    const float2 *A = sv.A;
    float2 *Ap = sv.Ap, *At = sv.At;
    const int rows = rows_pad_for_dev(n);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (int64_t)rows * l_pad; idx += stride) {
        const int r = (int)(idx / l_pad), c = (int)(idx % l_pad);
        Ap[idx] = (r < n && c < l) ? A[(size_t)r * l + c] : make_float2(0.0f, 0.0f);
    }
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (int64_t)l_pad * n; idx += stride) {
        const int c = (int)(idx / n), r = (int)(idx % n);  // transposed copy (column reads coalesce)
        At[idx] = c < l ? A[(size_t)r * l + c] : make_float2(0.0f, 0.0f);
    }
    // split-BF16 planes for the MFMA kernel that reads them from L2: x = hi + lo,
    // hi = RNE bf16(x), lo = RNE bf16(x - hi); planes re hi, im hi, re lo, im lo,
    // row-major (forward product) and transposed (adjoint)
    uint16_t *Fp = sv.Abf, *Tp = sv.Abf + (size_t)4 * rows * l_pad;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (int64_t)rows * l_pad; idx += stride) {
        const int r = (int)(idx / l_pad), c = (int)(idx % l_pad);
        const float2 v = (r < n && c < l) ? A[(size_t)r * l + c] : make_float2(0.0f, 0.0f);
        const __bf16 rh = (__bf16)v.x, ih = (__bf16)v.y;
        const __bf16 rl = (__bf16)(v.x - (float)rh), il = (__bf16)(v.y - (float)ih);
        const uint16_t pv[4] = {__builtin_bit_cast(uint16_t, rh), __builtin_bit_cast(uint16_t, ih),
                                __builtin_bit_cast(uint16_t, rl), __builtin_bit_cast(uint16_t, il)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Fp[((size_t)q * rows + r) * l_pad + c] = pv[q];
            Tp[((size_t)q * l_pad + c) * rows + r] = pv[q];
        }
    }
}

__global__ void __launch_bounds__(256) setup_gram_kernel(const StackTable t)
{
    if (t.d[blockIdx.y].p <= 0) return;
    const SetupView sv = setup_view(t.d[blockIdx.y]);
    const int n = sv.n, l = sv.l;
    const float2 *A = sv.A;
    double2 *M = sv.gram;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
        const int i = e / n, kk = e % n;
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < l; ++c) {
            const float2 p = A[(size_t)i * l + c], q = A[(size_t)kk * l + c];
            sr += (double)p.x * q.x + (double)p.y * q.y;  // p conj(q)
            si += (double)p.y * q.x - (double)p.x * q.y;
        }
        M[e] = make_double2(sr, si);
    }
}

// The power iteration runs on M^(2^kSquarings): where lambda_2 / lambda_1 = 1 - delta
// its Rayleigh quotient on M converges as (1 - delta)^(2^(kSquarings+1)) per step, so
// the 4,000-step cap leaves at most about 1 / (e 4000 2^(kSquarings+1)) relative
// error in lambda_1 (about 5e-5 on M itself, 1e-8 here); the error is also never
// above delta, which covers clustered top eigenvalues.
constexpr int kSquarings = 12;

__global__ void __launch_bounds__(256) setup_power_kernel(const StackTable t)
{
    if (t.d[blockIdx.y].p <= 0) return;
    const SetupView sv = setup_view(t.d[blockIdx.y]);
    const int n = sv.n, l = sv.l;
    const float2 *A = sv.A;
    const double2 *M = sv.gram;
    StackConsts *consts = sv.consts;
    uint32_t *queue = sv.queue;
    unsigned long long *work = sv.work;
    __shared__ double red[3][256];
    __shared__ double2 v[kMaxN];
    __shared__ double2 wv[kMaxN];
    const int tid = threadIdx.x, bd = blockDim.x;
    if (tid < 16) queue[tid] = 0u;
    if (tid < 4) work[tid] = 0ull;
    double cm = 0.0;
    for (int c = tid; c < l; c += bd) {
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
    // P = M^(2^kSquarings) / scale: each square divided by the squared trace of its
    // factor (M is PSD, so the trace of every scaled power lies in [1/N^2, 1])
    const double2 *P = M;
    for (int sq = 0; sq < kSquarings; ++sq) {
        double2 *Q = const_cast<double2 *>(M) + (size_t)(1 + (sq & 1)) * n * n;
        double tr = 0.0;
        for (int i = tid; i < n; i += bd) tr += P[(size_t)i * n + i].x;
        red[0][tid] = tr;
        __syncthreads();
        for (int s = bd / 2; s > 0; s >>= 1) {
            if (tid < s) red[0][tid] += red[0][tid + s];
            __syncthreads();
        }
        const double sc = red[0][0] > 0.0 ? 1.0 / (red[0][0] * red[0][0]) : 0.0;
        __syncthreads();
        for (int e = tid; e < n * n; e += bd) {
            const int i = e / n, j = e % n;
            double sr = 0.0, si = 0.0;
            for (int k = 0; k < n; ++k) {
                const double2 x = P[(size_t)i * n + k], y = P[(size_t)k * n + j];
                sr += x.x * y.x - x.y * y.y;
                si += x.x * y.y + x.y * y.x;
            }
            Q[e] = make_double2(sr * sc, si * sc);
        }
        __threadfence();
        __syncthreads();
        P = Q;
    }
    if (tid < n) v[tid] = make_double2(1.0 + 0.01 * tid, 0.001 * tid);
    __syncthreads();
    int it;
    double lam_prev = -1.0;
    for (it = 0; it < 4000; ++it) {
        // w = P v ; Rayleigh quotient v^H M v / v^H v ; v = w / ||w||  (one fused reduction)
        double pr = 0.0, nv = 0.0, nw = 0.0;
        if (tid < n) {
            double sr = 0.0, si = 0.0, ur = 0.0, ui = 0.0;
            for (int kk = 0; kk < n; ++kk) {
                const double2 m = M[tid * n + kk], q = P[tid * n + kk], x = v[kk];
                ur += m.x * x.x - m.y * x.y;
                ui += m.x * x.y + m.y * x.x;
                sr += q.x * x.x - q.y * x.y;
                si += q.x * x.y + q.y * x.x;
            }
            wv[tid] = make_double2(sr, si);
            pr = v[tid].x * ur + v[tid].y * ui;  // Re(conj(v) M v)
            nv = v[tid].x * v[tid].x + v[tid].y * v[tid].y;
            nw = sr * sr + si * si;
        }
        red[0][tid] = pr;
        red[1][tid] = nv;
        red[2][tid] = nw;
        __syncthreads();
        for (int s = bd / 2; s > 0; s >>= 1) {
            if (tid < s) {
                red[0][tid] += red[0][tid + s];
                red[1][tid] += red[1][tid + s];
                red[2][tid] += red[2][tid + s];
            }
            __syncthreads();
        }
        const double lam_est = red[1][0] > 0.0 ? red[0][0] / red[1][0] : 0.0;  // A = 0: L_f = 0
        const double ww = red[2][0];
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

// Bin Gram H = A^H A (FP64, l x l, row s holds H[s][m] = a_s^H a_m) for the
// refinement's round-end gradient; one entry per thread, m the fast index.
__global__ void __launch_bounds__(256) setup_bin_gram_kernel(const StackTable t)
{
    if (t.d[blockIdx.y].p <= 0) return;
    const SetupView sv = setup_view(t.d[blockIdx.y]);
    const int n = sv.n, l = sv.l;
    const float2 *A = sv.A;
    double2 *H = sv.H;
    const int64_t total = (int64_t)l * l;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += stride) {
        const int sr = (int)(e / l), m = (int)(e % l);
        double hr = 0.0, hi = 0.0;
        for (int i = 0; i < n; ++i) {
            const float2 p = A[(size_t)i * l + sr], q = A[(size_t)i * l + m];
            hr += (double)p.x * q.x + (double)p.y * q.y;  // conj(p) q
            hi += (double)p.x * q.y - (double)p.y * q.x;
        }
        H[e] = make_double2(hr, hi);
    }
}

// Setup of every stack of a table: packing, the N x N Gram, L_f and alpha_0 with
// the queue and counter reset, and (for the refinement) the bin Gram.
hipError_t launch_setup_table(const StackTable &t, bool bin_gram, hipStream_t s)
{
    if (t.count <= 0) return hipSuccess;
    int64_t pack = 0, nn = 0, ll = 0;
    for (int i = 0; i < t.count; ++i) {
        const StackDesc &d = t.d[i];
        pack = std::max<int64_t>(pack, (int64_t)rows_pad_for(d.n) * lpad_for(d.l));
        nn = std::max<int64_t>(nn, (int64_t)d.n * d.n);
        ll = std::max<int64_t>(ll, (int64_t)d.l * d.l);
    }
    const unsigned ys = (unsigned)t.count;
    auto gx = [](int64_t e, int64_t cap) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((e + 255) / 256, cap)); };
    hipLaunchKernelGGL(setup_pack_kernel, dim3(gx(pack, 1024), ys), dim3(256), 0, s, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(setup_gram_kernel, dim3(gx(nn, 64), ys), dim3(256), 0, s, t);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(setup_power_kernel, dim3(1, ys), dim3(256), 0, s, t);
    e = hipGetLastError();
    if (e != hipSuccess || !bin_gram) return e;
    hipLaunchKernelGGL(setup_bin_gram_kernel, dim3(gx(ll, 4096), ys), dim3(256), 0, s, t);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------

// LDS of the split re/im MFMA kernel: A (FP32, or its four split-BF16 planes
// twice) where staged, the cross-wave partials, and at 128 unknowns a wave the
// LDS-held iteration state
size_t fista_mfma_lds_bytes(int n, int l_pad, int waves, bool a_lds, int precision)
{
    const int rows = rows_pad_for(n), T = rows / 16;
    size_t off = 0;
    if (precision == L1LS_SPLIT_BF16 && a_lds)
        off = (fm_bf_planes_bytes_host(rows, l_pad) + 15) & ~(size_t)15;
    else if (a_lds && precision == L1LS_FP32)
        off = ((size_t)rows * (l_pad + 2) * sizeof(float2) + 15) & ~(size_t)15;
    off += (size_t)waves * 2 * T * 64 * 16;
    off += (size_t)waves * 16 * 16;
    off += 16;
    // 128 unknowns a wave: G_{k-1} of the tile's 16 pixels in LDS (float2 each)
    // and each wave's copy of r_{k-1} (16 T rows of the 16 pixels)
    if (l_pad / (16 * waves) >= 8) off += (size_t)16 * l_pad * sizeof(float2) + (size_t)waves * T * 4 * 64 * sizeof(float2);
    return off;
}

// Up to one wave per SIMD: a workgroup of W <= 4 waves may use W/4 of the CU's
// 160 KB; a workgroup of more waves holds the whole CU.
static bool mfma_lds_fits(const FistaArgs &a, int precision)
{
    const size_t cap = (size_t)160 * 1024 * (a.waves < 4 ? a.waves : 4) / 4;
    return fista_mfma_lds_bytes(a.n, a.l_pad, a.waves, true, precision) <= cap;
}

bool mfma_supports(int n, int l);

// The tiling a stack runs (see IterVariant).  FP32: up to 32 rows and 256 bins a
// wave holds 32 unknowns and a workgroup up to eight waves (two per SIMD), else 64
// (L <= 256) or 128 unknowns a wave and up to four waves; A is staged in LDS
// where it fits.  Split-BF16 stages its bf16 planes of A in LDS where they fit,
// else reads them from L2.  Shapes beyond the register tile (N > 64 or L > 512)
// run the streamed MFMA tile (either precision), and so does kAuto for
// 384 < L <= 512 (auto_stream); choice kStream runs it for any shape, kWave the
// wave-per-pixel kernel (FP32), kMfma the register tile.
bool iter_variant(int n, int l, int precision, int choice, int alt, IterVariant *v)
{
    IterVariant r{};
    const int l_pad = lpad_for(l), waves = waves_for(l), T = rows_pad_for(n) / 16;
    if (choice == kWave) {
        if (alt != 0 || precision != L1LS_FP32) return false;
        r.family = kVarWave;
        r.nc = wave_chunks(l);
        r.waves = 1;
        r.prec = L1LS_FP32;
        *v = r;
        return r.nc > 0;
    }
    if (choice == kStream || (choice == kAuto && auto_stream(n, l, precision)) || !mfma_supports(n, l)) {
        if (alt != 0 || T > 8) return false;
        r.family = kVarStream;
        r.T = T;
        r.waves = 4;
        r.wmax = 4;
        r.prec = precision;
        *v = r;
        return true;
    }
    FistaArgs probe{};
    probe.n = n;
    probe.l = l;
    probe.l_pad = l_pad;
    probe.waves = waves;
    if (precision == L1LS_SPLIT_BF16) {
        // the planes of A in LDS where they fit (up to 32 rows at L <= 256), else
        // read from their workspace copy (L2); 64 (L <= 256) or 128 unknowns a wave
        if (alt != 0) return false;
        const int KB = slice_blocks_for(l) == 8 ? 4 : 8;
        const bool lds = KB == 4 && mfma_lds_fits(probe, L1LS_SPLIT_BF16);
        r = IterVariant{kVarMfma, T, KB, lds ? 1 : 0, L1LS_SPLIT_BF16, 4, waves, 0};
        *v = r;
        return true;
    }
    bool kb2 = T <= 2 && slice_blocks_for(l) == 8;
    if (alt == 2) {
        if (!(T <= 2 && slice_blocks_for(l) == 8)) return false;
        kb2 = !kb2;
    }
    if (kb2) {
        FistaArgs b = probe;
        b.waves = l_pad / 32;
        r = IterVariant{kVarMfma, T, 2, mfma_lds_fits(b, L1LS_FP32) ? 1 : 0, L1LS_FP32, 8, b.waves, 0};
    } else {
        r = IterVariant{kVarMfma, T, slice_blocks_for(l) == 8 ? 4 : 8, mfma_lds_fits(probe, L1LS_FP32) ? 1 : 0,
                        L1LS_FP32, 4, waves, 0};
    }
    if (alt == 1) {
        if (!r.alds) return false;  // the LDS copy does not fit: no alternative placement
        r.alds = 0;
    }
    *v = r;
    return true;
}

size_t iter_variant_lds(const IterVariant &v, int n, int l)
{
    if (v.family == kVarWave) return fista_wave_lds(n, l);
    if (v.family == kVarStream) return fista_stream_lds_bytes(v.T);
    return fista_mfma_lds_bytes(n, lpad_for(l), v.waves, v.alds != 0, v.prec);
}

template <int T, int PREC>
static hipError_t launch_mfma_t(const StackTable &t, const IterVariant &v, hipStream_t s)
{
    if constexpr (PREC == L1LS_SPLIT_BF16) {
        if (v.KB == 4)
            return v.alds ? launch_mfma_one<T, 4, true, L1LS_SPLIT_BF16, 4>(t, v.waves, s)
                          : launch_mfma_one<T, 4, false, L1LS_SPLIT_BF16, 4>(t, v.waves, s);
        if (v.KB == 8) return launch_mfma_one<T, 8, false, L1LS_SPLIT_BF16, 4>(t, v.waves, s);
        return hipErrorInvalidValue;
    } else {
        if constexpr (T <= 2) {
            if (v.KB == 2)
                return v.alds ? launch_mfma_one<T, 2, true, L1LS_FP32, 8>(t, v.waves, s)
                              : launch_mfma_one<T, 2, false, L1LS_FP32, 8>(t, v.waves, s);
        }
        if (v.KB == 4)
            return v.alds ? launch_mfma_one<T, 4, true, L1LS_FP32, 4>(t, v.waves, s)
                          : launch_mfma_one<T, 4, false, L1LS_FP32, 4>(t, v.waves, s);
        if (v.KB == 8)
            return v.alds ? launch_mfma_one<T, 8, true, L1LS_FP32, 4>(t, v.waves, s)
                          : launch_mfma_one<T, 8, false, L1LS_FP32, 4>(t, v.waves, s);
        return hipErrorInvalidValue;
    }
}

// One launch for the stacks of a table that all run variant v.
hipError_t launch_iteration_table(const StackTable &t, const IterVariant &v, hipStream_t s)
{
    if (v.family == kVarWave) return launch_wave_table(t, v.nc, s);
    if (v.family == kVarStream) return launch_stream_table(t, v.T, v.prec, s);
    const bool bf = v.prec == L1LS_SPLIT_BF16;
    switch (v.T) {
    case 1: return bf ? launch_mfma_t<1, L1LS_SPLIT_BF16>(t, v, s) : launch_mfma_t<1, L1LS_FP32>(t, v, s);
    case 2: return bf ? launch_mfma_t<2, L1LS_SPLIT_BF16>(t, v, s) : launch_mfma_t<2, L1LS_FP32>(t, v, s);
    case 3: return bf ? launch_mfma_t<3, L1LS_SPLIT_BF16>(t, v, s) : launch_mfma_t<3, L1LS_FP32>(t, v, s);
    case 4: return bf ? launch_mfma_t<4, L1LS_SPLIT_BF16>(t, v, s) : launch_mfma_t<4, L1LS_FP32>(t, v, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace l1ls
