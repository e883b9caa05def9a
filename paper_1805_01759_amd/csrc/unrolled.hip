// Unrolled fixed-step accelerated proximal-gradient map and its adjoint
// (complex L1LS of arXiv 1805.01759; Eqs. (11)-(12) with a constant step alpha,
// no backtracking and no monotone test, so the map is differentiable almost
// everywhere).  Iteration k = 1..K maps (x^{k-1}, x^{k-2}) to x^k:
//   y_k = x^{k-1} + beta_k (x^{k-1} - x^{k-2}),  beta_k = max(0, (k-2)/(k+1))
//   r_k = A y_k - b,   v_k = y_k - 2 alpha A^H r_k,   x^k = S_{alpha lambda}(v_k)
// with x^0 = x^{-1} = 0 and A[n, l] = exp(-j 2 pi xi_n s_l).
//
// One 64-lane wave per pixel; the pixel's vectors live in LDS.  The forward
// saves (x^k, x^{k-1}) every ckpt_every iterations; the backward pass walks the
// segments in reverse, recomputes each segment from its checkpoint with the
// same device routine (bit-identical trajectory), then sweeps it backwards:
//   v-bar = S'(v_k)^T x-bar^k,   tau-bar = -Re(u-bar W) on |v| > tau
//   w = A v-bar,   y-bar = v-bar - 2 alpha A^H w,   b-bar += 2 alpha w
//   xi-bar_n += Re[-2 alpha (conj(r_n) (dA v-bar)_n + conj(w_n) (dA y_k)_n)],
//     dA = d A / d xi_n = -j 2 pi A diag(s)
//   x-bar^{k-1} += (1 + beta_k) y-bar,  x-bar^{k-2} = -beta_k y-bar
// Gradients follow the convention dL/dRe + j dL/dIm for complex quantities.
#include "l1ls_internal.h"

namespace l1ls {

constexpr int kUWaves = 4;          // pixels (waves) per workgroup
constexpr int kUMaxL = 1024;
constexpr int kUMaxN = 128;

struct UnrolledArgs {
    int n, l, K, ckpt;
    int64_t p;
    const float2 *A;     // n x l
    const float2 *As;    // n x l: A diag(s)
    const float2 *B;
    float lambda, alpha;
    float2 *X;           // p x l output (forward)
    float2 *tape;        // forward: checkpoints p x (K/ckpt - 1) x (2 l + 2 n); (x, xp) used here
    const float2 *dX;    // backward
    float2 *dB;
    float *part;         // backward: per pixel [lambda-bar, xi-bar_0..n-1]
    float2 *seg;         // backward: per wave slot segment tape
    int64_t slots;
};

__global__ void __launch_bounds__(256) unrolled_setup_kernel(int n, int l, const float *xi,
                                                             const float *s, float2 *A, float2 *As)
{
    const int64_t tot = (int64_t)n * l;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / l), j = (int)(e % l);
        const double ph = -2.0 * 3.14159265358979323846 * (double)xi[i] * (double)s[j];
        double sn, cs;
        sincos(ph, &sn, &cs);
        A[e] = make_float2((float)cs, (float)sn);
        As[e] = make_float2((float)(cs * s[j]), (float)(sn * s[j]));
    }
}

struct UPix {
    float2 *x, *xp, *y, *v, *g;  // l entries each (LDS)
    float2 *r, *w;               // n entries each (LDS)
};

__device__ __forceinline__ float wsum32(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// t = M u over the n rows (lanes over n, loop over l); M row-major n x l
__device__ __forceinline__ void rows_times(const float2 *M, int n, int l, const float2 *u, float2 *t,
                                           const float2 *sub)
{
    const int lane = threadIdx.x & 63;
    for (int i = lane; i < n; i += 64) {
        float ar = 0.0f, ai = 0.0f;
        const float2 *row = M + (size_t)i * l;
        for (int j = 0; j < l; ++j) {
            const float2 a = row[j], x = u[j];
            ar = fmaf(a.x, x.x, fmaf(-a.y, x.y, ar));
            ai = fmaf(a.x, x.y, fmaf(a.y, x.x, ai));
        }
        if (sub) {
            ar -= sub[i].x;
            ai -= sub[i].y;
        }
        t[i] = make_float2(ar, ai);
    }
}

// g = M^H t (lanes over l, loop over n)
__device__ __forceinline__ float2 cols_adj(const float2 *M, int n, int l, int j, const float2 *t)
{
    float gr = 0.0f, gi = 0.0f;
    for (int i = 0; i < n; ++i) {
        const float2 a = M[(size_t)i * l + j], q = t[i];
        gr = fmaf(a.x, q.x, fmaf(a.y, q.y, gr));
        gi = fmaf(a.x, q.y, fmaf(-a.y, q.x, gi));
    }
    return make_float2(gr, gi);
}

// One iteration k: from (x = x^{k-1}, xp = x^{k-2}) to x^k; keeps y_k, v_k, r_k.
__device__ void unrolled_step(const UnrolledArgs &a, const UPix &s, const float2 *b, int k)
{
    const int lane = threadIdx.x & 63;
    const float beta = fmaxf(0.0f, (float)(k - 2) / (float)(k + 1));
    for (int j = lane; j < a.l; j += 64) {
        const float2 x = s.x[j], xp = s.xp[j];
        s.y[j] = make_float2(x.x + beta * (x.x - xp.x), x.y + beta * (x.y - xp.y));
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0);
    rows_times(a.A, a.n, a.l, s.y, s.r, b);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0);
    const float tau = a.alpha * a.lambda;
    for (int j = lane; j < a.l; j += 64) {
        const float2 g = cols_adj(a.A, a.n, a.l, j, s.r);
        const float2 y = s.y[j];
        const float vr = y.x - 2.0f * a.alpha * g.x, vi = y.y - 2.0f * a.alpha * g.y;
        s.v[j] = make_float2(vr, vi);
        const float m = sqrtf(vr * vr + vi * vi);
        const float sc = m > tau ? 1.0f - tau / m : 0.0f;
        s.xp[j] = s.x[j];
        s.x[j] = make_float2(vr * sc, vi * sc);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0);
}

__device__ __forceinline__ size_t ulds_per_wave(int n, int l)
{
    return (size_t)(5 * l + 2 * n) * sizeof(float2);
}

__device__ __forceinline__ UPix carve(unsigned char *base, int n, int l)
{
    UPix s;
    float2 *f = reinterpret_cast<float2 *>(base);
    s.x = f;
    s.xp = f + l;
    s.y = f + 2 * l;
    s.v = f + 3 * l;
    s.g = f + 4 * l;
    s.r = f + 5 * l;
    s.w = f + 5 * l + n;
    return s;
}

__global__ void __launch_bounds__(64 * kUWaves) unrolled_forward_kernel(const UnrolledArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    UPix s = carve(smem + wv * ulds_per_wave(a.n, a.l), a.n, a.l);
    const int nck = a.K / a.ckpt;
    for (int64_t p = (int64_t)blockIdx.x * kUWaves + wv; p < a.p; p += (int64_t)gridDim.x * kUWaves) {
        const float2 *b = a.B + (size_t)p * a.n;
        for (int j = lane; j < a.l; j += 64) s.x[j] = s.xp[j] = make_float2(0.0f, 0.0f);
        __builtin_amdgcn_wave_barrier();
        for (int k = 1; k <= a.K; ++k) {
            unrolled_step(a, s, b, k);
            // checkpoint: state before iteration k + 1, at k = c, 2c, ...
            if (k % a.ckpt == 0 && k / a.ckpt < nck) {
                float2 *t = a.tape + ((size_t)p * (nck - 1) + (k / a.ckpt - 1)) * (2 * a.l + 2 * a.n);
                for (int j = lane; j < a.l; j += 64) {
                    t[j] = s.x[j];
                    t[a.l + j] = s.xp[j];
                }
            }
        }
        float2 *xo = a.X + (size_t)p * a.l;
        for (int j = lane; j < a.l; j += 64) xo[j] = s.x[j];
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ void __launch_bounds__(64 * kUWaves) unrolled_backward_kernel(const UnrolledArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    unsigned char *base = smem + wv * (ulds_per_wave(a.n, a.l) + (size_t)(2 * a.l) * sizeof(float2));
    UPix s = carve(base, a.n, a.l);
    float2 *a1 = reinterpret_cast<float2 *>(base + ulds_per_wave(a.n, a.l));  // x-bar of x^{k}
    float2 *a0 = a1 + a.l;                                                    // x-bar of x^{k-1}
    const int nck = a.K / a.ckpt;
    const int64_t slot = (int64_t)blockIdx.x * kUWaves + wv;
    // segment tape of this wave slot: per iteration y (l), v (l), r (n)
    float2 *seg = a.seg + (size_t)slot * a.ckpt * (2 * a.l + a.n);
    const float tau = a.alpha * a.lambda;
    const float two_a = 2.0f * a.alpha;
    const float twopi = 6.283185307179586f;
    for (int64_t p = slot; p < a.p; p += (int64_t)gridDim.x * kUWaves) {
        const float2 *b = a.B + (size_t)p * a.n;
        for (int j = lane; j < a.l; j += 64) {
            a1[j] = a.dX[(size_t)p * a.l + j];
            a0[j] = make_float2(0.0f, 0.0f);
        }
        float lam_bar = 0.0f;               // lane partial
        float xib[2] = {0.0f, 0.0f};        // lanes i, i + 64 of xi-bar
        float2 bb[2] = {make_float2(0.0f, 0.0f), make_float2(0.0f, 0.0f)};
        __builtin_amdgcn_wave_barrier();
        for (int sg = nck - 1; sg >= 0; --sg) {
            const int k0 = sg * a.ckpt;
            // restore (x^{k0}, x^{k0-1})
            if (sg == 0) {
                for (int j = lane; j < a.l; j += 64) s.x[j] = s.xp[j] = make_float2(0.0f, 0.0f);
            } else {
                const float2 *t = a.tape + ((size_t)p * (nck - 1) + (sg - 1)) * (2 * a.l + 2 * a.n);
                for (int j = lane; j < a.l; j += 64) {
                    s.x[j] = t[j];
                    s.xp[j] = t[a.l + j];
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_s_waitcnt(0);
            // recompute the segment, recording y_k, v_k, r_k
            for (int q = 0; q < a.ckpt; ++q) {
                unrolled_step(a, s, b, k0 + q + 1);
                float2 *e = seg + (size_t)q * (2 * a.l + a.n);
                for (int j = lane; j < a.l; j += 64) {
                    e[j] = s.y[j];
                    e[a.l + j] = s.v[j];
                }
                for (int i = lane; i < a.n; i += 64) e[2 * a.l + i] = s.r[i];
            }
            __threadfence_block();
            __builtin_amdgcn_wave_barrier();
            // reverse sweep over the segment
            for (int q = a.ckpt - 1; q >= 0; --q) {
                const int k = k0 + q + 1;
                const float beta = fmaxf(0.0f, (float)(k - 2) / (float)(k + 1));
                const float2 *e = seg + (size_t)q * (2 * a.l + a.n);
                // v-bar through the prox; stash v-bar in s.g and y_k in s.y
                for (int j = lane; j < a.l; j += 64) {
                    const float2 v = e[a.l + j], W = a1[j];
                    s.y[j] = e[j];
                    const float m = sqrtf(v.x * v.x + v.y * v.y);
                    float2 vb = make_float2(0.0f, 0.0f);
                    if (m > tau) {
                        const float ur = v.x / m, ui = v.y / m, c = tau / m;
                        const float rad = ur * W.x + ui * W.y;  // Re(conj(u) W)
                        vb = make_float2((1.0f - c) * W.x + c * rad * ur, (1.0f - c) * W.y + c * rad * ui);
                        lam_bar -= a.alpha * rad;
                    }
                    s.g[j] = vb;
                }
                for (int i = lane; i < a.n; i += 64) s.r[i] = e[2 * a.l + i];
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_s_waitcnt(0);
                // w = A v-bar (into s.w); dA products into registers of lanes i < n
                rows_times(a.A, a.n, a.l, s.g, s.w, nullptr);
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_s_waitcnt(0);
                for (int ii = 0, i = lane; i < a.n; i += 64, ++ii) {
                    float pr = 0.0f, pi = 0.0f, qr = 0.0f, qi = 0.0f;  // (A S v-bar)_i, (A S y)_i
                    const float2 *row = a.As + (size_t)i * a.l;
                    for (int j = 0; j < a.l; ++j) {
                        const float2 c = row[j], vb = s.g[j], y = s.y[j];
                        pr = fmaf(c.x, vb.x, fmaf(-c.y, vb.y, pr));
                        pi = fmaf(c.x, vb.y, fmaf(c.y, vb.x, pi));
                        qr = fmaf(c.x, y.x, fmaf(-c.y, y.y, qr));
                        qi = fmaf(c.x, y.y, fmaf(c.y, y.x, qi));
                    }
                    // d/dxi_i of A = -j 2 pi A S:  (dA u)_i = -j 2 pi (A S u)_i = 2 pi (Im, -Re)
                    const float2 r = s.r[i], w = s.w[i];
                    const float dvr = twopi * pi, dvi = -twopi * pr;  // (dA v-bar)_i
                    const float dyr = twopi * qi, dyi = -twopi * qr;  // (dA y)_i
                    // Re[conj(r) dvb + conj(w) dy]
                    xib[ii] += -two_a * (r.x * dvr + r.y * dvi + w.x * dyr + w.y * dyi);
                    bb[ii].x += two_a * w.x;
                    bb[ii].y += two_a * w.y;
                }
                // y-bar = v-bar - 2 alpha A^H w ; propagate to x-bar^{k-1}, x-bar^{k-2}
                for (int j = lane; j < a.l; j += 64) {
                    const float2 h = cols_adj(a.A, a.n, a.l, j, s.w);
                    const float2 vb = s.g[j];
                    const float ybr = vb.x - two_a * h.x, ybi = vb.y - two_a * h.y;
                    const float2 o0 = a0[j];
                    a1[j] = make_float2(o0.x + (1.0f + beta) * ybr, o0.y + (1.0f + beta) * ybi);
                    a0[j] = make_float2(-beta * ybr, -beta * ybi);
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_s_waitcnt(0);
            }
        }
        // outputs: dB, per-pixel partials of lambda-bar and xi-bar
        for (int ii = 0, i = lane; i < a.n; i += 64, ++ii) {
            a.dB[(size_t)p * a.n + i] = bb[ii];
            a.part[(size_t)p * (a.n + 1) + 1 + i] = xib[ii];
        }
        const float lb = wsum32(lam_bar);
        if (lane == 0) a.part[(size_t)p * (a.n + 1)] = lb;
        __builtin_amdgcn_wave_barrier();
    }
}

// Deterministic reduction of the per-pixel partials (fixed order): out[c] =
// sum_p part[p][c], c = 0..n.  One workgroup per column.
__global__ void __launch_bounds__(256) unrolled_reduce_kernel(const float *part, int64_t p, int cols,
                                                              float *dlambda, float *dxi)
{
    __shared__ double red[256];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < p; q += 256) acc += part[(size_t)q * cols + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (c == 0) *dlambda = (float)red[0];
        else dxi[c - 1] = (float)red[0];
    }
}

// ------------------------------------------------------------------ host side

bool unrolled_tile_supports(int n, int l);
size_t unrolled_tile_seg_bytes(int n, int l, int ckpt);
hipError_t launch_unrolled_tile(bool forward, int n, int l, int64_t p, const float2 *A, const float2 *As,
                                const float2 *B, float lambda, float alpha, int K, int ckpt, float2 *X,
                                float2 *ck, const float2 *dX, float2 *dB, float *part, void *seg,
                                int64_t max_groups, hipStream_t st);

static size_t fwd_lds(int n, int l) { return (size_t)kUWaves * (5 * l + 2 * n) * sizeof(float2); }
static size_t bwd_lds(int n, int l) { return (size_t)kUWaves * (7 * l + 2 * n) * sizeof(float2); }

static int64_t bwd_slots()
{
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return (int64_t)cus * 8 * kUWaves;
}

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// checkpoint = (x, xp, r_x, r_xp): the matrix-core kernels restart the residual
// recursion from it; the wave-per-pixel kernels use the first 2 l entries
size_t unrolled_tape_bytes(int n, int l, int64_t p, int K, int ckpt)
{
    const int nck = K / ckpt;
    return al256((size_t)n * l * sizeof(float2)) * 2 +
           al256((size_t)p * (nck > 1 ? nck - 1 : 0) * (2 * l + 2 * n) * sizeof(float2));
}

static int64_t tile_groups()
{
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus;
}

size_t unrolled_bwd_ws_bytes(int n, int l, int64_t p, int K, int ckpt)
{
    (void)K;
    const size_t wave_seg = (size_t)bwd_slots() * ckpt * (2 * l + n) * sizeof(float2);
    const size_t tile_seg = unrolled_tile_supports(n, l) ? (size_t)tile_groups() * unrolled_tile_seg_bytes(n, l, ckpt) : 0;
    return al256((size_t)p * (n + 1) * sizeof(float)) + al256(wave_seg > tile_seg ? wave_seg : tile_seg);
}

hipError_t launch_unrolled_forward(int n, int l, int64_t p, const float *xi, const float *s,
                                   const float2 *B, float lambda, float alpha, int K, int ckpt,
                                   float2 *X, void *tape, hipStream_t st)
{
    char *t = (char *)tape;
    float2 *A = (float2 *)t;
    float2 *As = (float2 *)(t + al256((size_t)n * l * sizeof(float2)));
    float2 *ck = (float2 *)(t + 2 * al256((size_t)n * l * sizeof(float2)));
    hipLaunchKernelGGL(unrolled_setup_kernel, dim3(64), dim3(256), 0, st, n, l, xi, s, A, As);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p == 0) return e;
    UnrolledArgs a{};
    if (unrolled_tile_supports(n, l))
        return launch_unrolled_tile(true, n, l, p, A, As, B, lambda, alpha, K, ckpt, X, ck, nullptr,
                                    nullptr, nullptr, nullptr, 0, st);
    a.n = n; a.l = l; a.K = K; a.ckpt = ckpt; a.p = p;
    a.A = A; a.As = As; a.B = B; a.lambda = lambda; a.alpha = alpha; a.X = X; a.tape = ck;
    const size_t lds = fwd_lds(n, l);
    hipFuncSetAttribute((const void *)unrolled_forward_kernel,
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    const int64_t groups = (p + kUWaves - 1) / kUWaves;
    const int64_t cap = bwd_slots() / kUWaves * 2;
    hipLaunchKernelGGL(unrolled_forward_kernel, dim3((unsigned)(groups < cap ? groups : cap)),
                       dim3(64 * kUWaves), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_unrolled_backward(int n, int l, int64_t p, const float2 *B, float lambda,
                                    float alpha, int K, int ckpt, const void *tape,
                                    const float2 *dX, float2 *dB, float *dlambda, float *dxi,
                                    void *ws, hipStream_t st)
{
    const char *t = (const char *)tape;
    UnrolledArgs a{};
    a.n = n; a.l = l; a.K = K; a.ckpt = ckpt; a.p = p;
    a.A = (const float2 *)t;
    a.As = (const float2 *)(t + al256((size_t)n * l * sizeof(float2)));
    a.tape = (float2 *)(t + 2 * al256((size_t)n * l * sizeof(float2)));
    a.B = B; a.lambda = lambda; a.alpha = alpha; a.dX = dX; a.dB = dB;
    char *w = (char *)ws;
    a.part = (float *)w;
    a.seg = (float2 *)(w + al256((size_t)p * (n + 1) * sizeof(float)));
    a.slots = bwd_slots();
    if (p > 0 && unrolled_tile_supports(n, l)) {
        hipError_t e = launch_unrolled_tile(false, n, l, p, a.A, a.As, B, lambda, alpha, K, ckpt, nullptr,
                                            a.tape, dX, dB, a.part, a.seg, tile_groups(), st);
        if (e != hipSuccess) return e;
    } else if (p > 0) {
        const size_t lds = bwd_lds(n, l);
        hipFuncSetAttribute((const void *)unrolled_backward_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        const int64_t groups = (p + kUWaves - 1) / kUWaves;
        const int64_t cap = a.slots / kUWaves;
        hipLaunchKernelGGL(unrolled_backward_kernel, dim3((unsigned)(groups < cap ? groups : cap)),
                           dim3(64 * kUWaves), lds, st, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(unrolled_reduce_kernel, dim3(n + 1), dim3(256), 0, st, a.part, p, n + 1,
                       dlambda, dxi);
    return hipGetLastError();
}

}  // namespace l1ls
