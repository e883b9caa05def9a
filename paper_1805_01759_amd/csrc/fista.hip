// Setup kernel (packing, Lipschitz constant, alpha0) and the dispatch from
// (N, L, precision) to the instantiated persistent iteration kernels.
#include "l1ls_internal.h"

namespace l1ls {

template <int NZB, int KB, bool ALDS, int PREC>
hipError_t launch_one(const FistaArgs &a, int max_groups, hipStream_t s);
template <int T, int KB, bool ALDS, int PREC, int WMAX>
hipError_t launch_mfma_one(const FistaArgs &a, int max_groups, hipStream_t s);
size_t fm_bf_planes_bytes_host(int rows, int l_pad);

__device__ __forceinline__ int rows_pad_for_dev(int n) { return 16 * ((n + 15) / 16); }

// ---------------------------------------------------------------------------
// Setup, three launches on the caller's stream:
//   setup_pack_kernel   (grid)    A packed zero-padded to rows_pad_for(n) x l_pad, and
//                                 its transpose l_pad x n
//   setup_gram_kernel   (grid)    FP64 Gram M = A A^H, one entry per thread
//   setup_power_kernel  (1 group) queue/counter reset, alpha0 = 1/(2 max_l ||a_l||^2),
//                                 L_f = 2 lambda_max(M) by FP64 power iteration
__global__ void __launch_bounds__(256) setup_pack_kernel(int n, int l, int l_pad, const float2 *A,
                                                         float2 *Ap, float2 *At)
{
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
}

__global__ void __launch_bounds__(256) setup_gram_kernel(int n, int l, const float2 *A, double2 *M)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int i = e / n, kk = e % n;
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < l; ++c) {
        const float2 p = A[(size_t)i * l + c], q = A[(size_t)kk * l + c];
        sr += (double)p.x * q.x + (double)p.y * q.y;  // p conj(q)
        si += (double)p.y * q.x - (double)p.x * q.y;
    }
    M[e] = make_double2(sr, si);
}

__global__ void __launch_bounds__(256) setup_power_kernel(int n, int l, const float2 *A, const double2 *M,
                                                          StackConsts *consts, uint32_t *queue,
                                                          unsigned long long *work)
{
    __shared__ double red[3][256];
    __shared__ double2 v[kMaxN];
    __shared__ double2 wv[kMaxN];
    const int tid = threadIdx.x, bd = blockDim.x;
    if (tid < 8) queue[tid] = 0u;
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
    if (tid < n) v[tid] = make_double2(1.0 + 0.01 * tid, 0.001 * tid);
    __syncthreads();
    int it;
    double lam_prev = -1.0;
    for (it = 0; it < 4000; ++it) {
        // w = M v ; Rayleigh quotient v^H M v / v^H v ; v = w / ||w||  (one fused reduction)
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
        const double lam_est = red[0][0] / red[1][0];
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
__global__ void __launch_bounds__(256) setup_bin_gram_kernel(int n, int l, const float2 *A, double2 *H)
{
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

hipError_t launch_setup_bin_gram(int n, int l, const float2 *A, double2 *H, hipStream_t s)
{
    const int64_t total = (int64_t)l * l;
    int groups = (int)((total + 255) / 256);
    if (groups > 4096) groups = 4096;
    hipLaunchKernelGGL(setup_bin_gram_kernel, dim3(groups), dim3(256), 0, s, n, l, A, H);
    return hipGetLastError();
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

hipError_t launch_setup(int n, int l, int l_pad, const float2 *A, float2 *Ap, float2 *At, double2 *gram,
                        StackConsts *consts, uint32_t *queue, unsigned long long *work,
                        hipStream_t s)
{
    const int64_t elems = (int64_t)rows_pad_for(n) * l_pad;
    int groups = (int)((elems + 255) / 256);
    if (groups > 1024) groups = 1024;
    hipLaunchKernelGGL(setup_pack_kernel, dim3(groups), dim3(256), 0, s, n, l, l_pad, A, Ap, At);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(setup_gram_kernel, dim3((n * n + 255) / 256), dim3(256), 0, s, n, l, A, gram);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(setup_power_kernel, dim3(1), dim3(256), 0, s, n, l, A, gram, consts, queue, work);
    return hipGetLastError();
}

template <int NZB, int PREC>
static hipError_t launch_zb(const FistaArgs &a, int max_groups, hipStream_t s)
{
    const bool lds = fista_a_fits_lds(a.n, a.l_pad, a.waves, NZB);
    if (slice_blocks_for(a.l) == 8)
        return lds ? launch_one<NZB, 8, true, PREC>(a, max_groups, s)
                   : launch_one<NZB, 8, false, PREC>(a, max_groups, s);
    return lds ? launch_one<NZB, 16, true, PREC>(a, max_groups, s)
               : launch_one<NZB, 16, false, PREC>(a, max_groups, s);
}

template <int PREC>
static hipError_t launch_prec(const FistaArgs &a, int max_groups, hipStream_t s)
{
    switch (zblocks_for(a.n)) {
    case 1: return launch_zb<1, PREC>(a, max_groups, s);
    case 2: return launch_zb<2, PREC>(a, max_groups, s);
    case 3: return launch_zb<3, PREC>(a, max_groups, s);
    case 4: return launch_zb<4, PREC>(a, max_groups, s);
    case 5: return launch_zb<5, PREC>(a, max_groups, s);
    case 6: return launch_zb<6, PREC>(a, max_groups, s);
    case 7: return launch_zb<7, PREC>(a, max_groups, s);
    case 8: return launch_zb<8, PREC>(a, max_groups, s);
    default: return hipErrorInvalidValue;
    }
}

// FP32 contractions: the kernel with split real/imaginary accumulators
size_t fista_mfma_lds_bytes(int n, int l_pad, int waves, bool a_lds, int precision)
{
    const int rows = rows_pad_for(n), T = rows / 16;
    size_t off = 0;
    if (precision == L1LS_SPLIT_BF16)
        off = (fm_bf_planes_bytes_host(rows, l_pad) + 15) & ~(size_t)15;
    else if (a_lds)
        off = ((size_t)rows * (l_pad + 2) * sizeof(float2) + 15) & ~(size_t)15;
    off += (size_t)waves * 2 * T * 64 * 16;
    off += (size_t)waves * 16 * 16;
    off += 16;
    return off;
}

// Up to one wave per SIMD: a workgroup of W <= 4 waves may use W/4 of the CU's
// 160 KB; a workgroup of more waves holds the whole CU.
static bool mfma_lds_fits(const FistaArgs &a, int precision)
{
    const size_t cap = (size_t)160 * 1024 * (a.waves < 4 ? a.waves : 4) / 4;
    return fista_mfma_lds_bytes(a.n, a.l_pad, a.waves, true, precision) <= cap;
}

template <int T>
static hipError_t launch_mfma_t(const FistaArgs &a, int max_groups, hipStream_t s)
{
    if constexpr (T <= 2) {
        if (slice_blocks_for(a.l) == 8) {
            // 32 unknowns per wave, up to eight waves: the state of a 16-pixel tile
            // fits two waves per SIMD without accumulation-register traffic
            FistaArgs b = a;
            b.waves = a.l_pad / 32;
            return mfma_lds_fits(b, L1LS_FP32) ? launch_mfma_one<T, 2, true, L1LS_FP32, 8>(b, max_groups, s)
                                               : launch_mfma_one<T, 2, false, L1LS_FP32, 8>(b, max_groups, s);
        }
    }
    const bool lds = mfma_lds_fits(a, L1LS_FP32);
    if (slice_blocks_for(a.l) == 8)
        return lds ? launch_mfma_one<T, 4, true, L1LS_FP32, 4>(a, max_groups, s)
                   : launch_mfma_one<T, 4, false, L1LS_FP32, 4>(a, max_groups, s);
    return lds ? launch_mfma_one<T, 8, true, L1LS_FP32, 4>(a, max_groups, s)
               : launch_mfma_one<T, 8, false, L1LS_FP32, 4>(a, max_groups, s);
}

// Whether launch_fista runs a split re/im kernel (fista_mfma.h) for this shape
// and precision; the real-embedded kernels (fista_impl.h) have no warm start.
bool fista_split_kernel(const FistaArgs &a, int precision)
{
    const int T = rows_pad_for(a.n) / 16;
    if (precision == L1LS_SPLIT_BF16) return slice_blocks_for(a.l) == 8 && mfma_lds_fits(a, L1LS_SPLIT_BF16) && T <= 4;
    return T <= 4;
}

hipError_t launch_fista(const FistaArgs &a, int precision, int max_groups, hipStream_t s, bool *keeps_residual)
{
    if (a.warm && !fista_split_kernel(a, precision)) return hipErrorNotSupported;
    const int T = rows_pad_for(a.n) / 16;
    // the split re/im kernels (fista_mfma.h) write a.R; the real-embedded ones do not
    if (keeps_residual)
        *keeps_residual = precision == L1LS_SPLIT_BF16
                              ? (slice_blocks_for(a.l) == 8 && mfma_lds_fits(a, L1LS_SPLIT_BF16) && T <= 4)
                              : T <= 4;
    if (precision == L1LS_SPLIT_BF16) {
        // split re/im layout with bf16 planes in LDS where they fit (64 unknowns per
        // wave); otherwise the real-embedded kernel
        if (slice_blocks_for(a.l) == 8 && mfma_lds_fits(a, L1LS_SPLIT_BF16)) {
            switch (T) {
            case 1: return launch_mfma_one<1, 4, true, L1LS_SPLIT_BF16, 4>(a, max_groups, s);
            case 2: return launch_mfma_one<2, 4, true, L1LS_SPLIT_BF16, 4>(a, max_groups, s);
            case 3: return launch_mfma_one<3, 4, true, L1LS_SPLIT_BF16, 4>(a, max_groups, s);
            case 4: return launch_mfma_one<4, 4, true, L1LS_SPLIT_BF16, 4>(a, max_groups, s);
            default: break;
            }
        }
        return launch_prec<L1LS_SPLIT_BF16>(a, max_groups, s);
    }
    switch (T) {
    case 1: return launch_mfma_t<1>(a, max_groups, s);
    case 2: return launch_mfma_t<2>(a, max_groups, s);
    case 3: return launch_mfma_t<3>(a, max_groups, s);
    case 4: return launch_mfma_t<4>(a, max_groups, s);
    default: return launch_prec<L1LS_FP32>(a, max_groups, s);
    }
}

}  // namespace l1ls
