// FP64 refinement of the FP32 iterate (complex L1LS of arXiv 1805.01759,
// Eq. (1)); not part of the paper's method, it turns "KKT <= tol" into the
// minimiser to FP64 accuracy and catches pixels the FP32 iteration left.
//
// A pixel whose FP32 KKT test passed is first checked in FP64 and skipped if it
// is solved; one the FP32 stage capped is refined without that check.
//
// Per pixel (one 64-lane workgroup), starting from the working set S of the
// local maxima of |x| of the FP32 iterate and the larger neighbour of each, repeat
//   * damped Newton on phi(z) = ||A_S z - b||^2 + lambda sum |z_s| over the
//     working set (|S| <= kMaxSupp), with the real Hessian
//       2 [[Re G, -Im G], [Im G, Re G]] + lambda blkdiag((I - u u^T)/|z_s|),
//     G = A_S^H A_S, u = (Re z_s, Im z_s)/|z_s|; the coordinate whose Newton step
//     turns it round most leaves the working set; Armijo backtracking on phi;
//     Newton stops once the working-set gradient is below the target or the
//     predicted decrease is below FP64 rounding of phi (then the full step is
//     taken: a line search there only measures rounding noise);
//   * full FP64 gradient: natural KKT residual, and the worst off-set
//     violator of |g_l| <= lambda enters at its exact coordinate minimiser,
// until the KKT residual is at the target or no violator is left.  The point
// with the least objective is kept and written back (complex64).
//
// The Gram G = A_S^H A_S is kept across Newton steps and updated only when the
// working set changes (a row appended on entry, a row and column removed on a
// drop), so a Newton matrix costs O(|S|^2) lookups.  r = A_S z - b, A_S^H r and
// phi are formed once for the seeded working set and then updated exactly: a
// step z += t d by t A_S d, t G d and the change the line search measured (it
// evaluates phi(z + t d) - phi(z) from <r, A_S d> and ||A_S d||^2 in O(|S|) per
// trial point), a drop or an entry by the column's rank-one term.
//
// LDS holds the working set's columns A_S, the residual, the Gram and a packed
// lower-triangular Hessian (for systems too large for the register solver);
// the starting point stays in X, the point with the least objective so far is
// kept as its working set and values and written to X once at the end, and the
// dense iterate is never materialised (a per-bin index into the working set
// stands in for it), which keeps the footprint near 13 KB at N=25, L=256 so
// that twelve pixels are in flight per CU.  Pixels are taken from a shared
// counter.
#include "l1ls_internal.h"
#include "wave_reduce.h"
#include <type_traits>

namespace l1ls {

using wr::lane_value;
using wr::wmax;
using wr::wsum;

// value of the float v held by lane i (i uniform across the wave)
__device__ __forceinline__ float lane_value_f(float v, int i)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}

// Newton on at most kMaxSupp complex unknowns: 8 for the first pass (small
// working sets keep a workgroup's LDS near 10 KB at N = 50, L = 512, so three
// waves share a SIMD); builds with 16 and then 32 take the pixels whose working
// set filled up before the target
#ifndef L1LS_POLISH_SUPP
#define L1LS_POLISH_SUPP 8
#endif
constexpr int kMaxSupp = L1LS_POLISH_SUPP;
static_assert(kMaxSupp == 8 || kMaxSupp == 16 || kMaxSupp == 32, "working sets of 8, 16 or 32 slots");
// violators admitted per round: the 32-slot pass grows its set by up to 8 a round
// (the next-largest violations of distinct lanes), the 8- and 16-slot passes by one
constexpr int kEnter = kMaxSupp == 32 ? 8 : 1;
constexpr int kTier = kMaxSupp == 8 ? 0 : (kMaxSupp == 16 ? 1 : 2);
constexpr int kMaxM = 2 * kMaxSupp;   // real Hessian order
constexpr int kTri = kMaxM * (kMaxM + 1) / 2;
constexpr int kGc = kMaxSupp * (kMaxSupp + 1) / 2;
// the register solver's transpose (order <= 16) sits past the packed Hessian
constexpr int kHLen = kTri >= 136 + 256 ? kTri : 136 + 256;

__device__ __forceinline__ int tri(int i, int k) { return i * (i + 1) / 2 + k; }  // k <= i

// Dynamic LDS of one workgroup: r and w (n double2 each; the FP32 copy of r that
// a pass reads lives in w's space), A_S (n x kMaxSupp float2, whose space first
// holds the nonzero-bin list of the starting point), the slot index of each bin.
static __host__ __device__ inline size_t polish_as_bytes(int n, int l_pad)  // per build (16 or 32 slots)
{
    const size_t as = (size_t)n * kMaxSupp * sizeof(float2), nz = (size_t)l_pad * sizeof(int16_t);
    return ((as > nz ? as : nz) + 15) / 16 * 16;
}

struct PolishShared {
    double2 *r;         // n: residual A x - b (dynamic LDS)
    double2 *w;         // n: A_S d of the current Newton direction (dynamic LDS)
    float2 *r32;        // n: the residual rounded to FP32 for the full pass (dynamic LDS)
    float2 *AS;         // n x kMaxSupp: columns of the working set (dynamic LDS)
    int16_t *nzl;       // l_pad: nonzero bins of the starting point (dynamic LDS)
    int8_t *sidx;       // l_pad: slot of bin m in the working set, or -1 (dynamic LDS)
    double H[kHLen];    // packed lower triangle of the real Hessian / its Cholesky factor
    double2 Gc[kGc];    // packed lower triangle of the Gram G = A_S^H A_S (Hermitian)
    double2 z[kMaxSupp], c[kMaxSupp];  // working-set point and A_S^H r
    double ur[kMaxSupp], ui[kMaxSupp], iz[kMaxSupp];  // z/|z| and 1/|z| per slot
    double grd[kMaxM], dir[kMaxM], invd[kMaxM];
    int S[kMaxSupp];
    int cnt;
    double2 zb[kMaxSupp];  // the point with the least objective so far, on slots Sb[0..sb)
    int Sb[kMaxSupp];
    int sb;                // -1: the starting point (already in X) is the best
    int vl[kEnter];        // violators to admit, largest first (full pass, kEnter > 1)
    int nv;
};

__device__ __forceinline__ double2 Aat(const PolishArgsDev &a, int n, int m)
{
    const float2 v = a.A[(size_t)n * a.l_pad + m];
    return make_double2(v.x, v.y);
}

__device__ __forceinline__ double2 ASat(const PolishShared &sh, int n, int t)
{
    const float2 v = sh.AS[n * kMaxSupp + t];
    return make_double2(v.x, v.y);
}

// r = A x0 - b for the starting point (its nonzero bins listed first)
__device__ void residual_start(const PolishArgsDev &a, PolishShared &sh, const float2 *b, const float2 *x0)
{
    const int lane = threadIdx.x;
    if (lane == 0) sh.cnt = 0;
    __syncthreads();
    for (int m0 = 0; m0 < a.l; m0 += 64) {
        const int m = m0 + lane;
        bool nz = false;
        if (m < a.l) {
            const float2 v = x0[m];
            nz = v.x != 0.0f || v.y != 0.0f;
        }
        const uint64_t bal = __ballot(nz);
        const int base = sh.cnt;
        if (nz) sh.nzl[base + __popcll(bal & ((1ull << lane) - 1ull))] = (int16_t)m;
        __syncthreads();
        if (lane == 0) sh.cnt = base + __popcll(bal);
        __syncthreads();
    }
    // r = A x0 - b over the listed bins in list order, eight bins' loads in flight
    // (the FP32 iterate handed over can have hundreds of nonzeros)
    const int cnt = sh.cnt;
    for (int nn = lane; nn < a.n; nn += 64) {
        double rr = -(double)b[nn].x, ri = -(double)b[nn].y;
        int q = 0;
        for (; q + 8 <= cnt; q += 8) {
            float2 xf[8], af[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int m = sh.nzl[q + u];
                xf[u] = x0[m];
                af[u] = a.A[(size_t)nn * a.l_pad + m];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                rr += (double)af[u].x * xf[u].x - (double)af[u].y * xf[u].y;
                ri += (double)af[u].x * xf[u].y + (double)af[u].y * xf[u].x;
            }
        }
        for (; q < cnt; ++q) {
            const int m = sh.nzl[q];
            const float2 xf = x0[m];
            const double2 av = Aat(a, nn, m);
            rr += av.x * xf.x - av.y * xf.y;
            ri += av.x * xf.y + av.y * xf.x;
        }
        sh.r[nn] = make_double2(rr, ri);
    }
    __syncthreads();
}

// phi(z) on the working set, r <- A_S z - b; returns phi (all lanes).  b0, b1:
// the data b of rows lane and lane + 64, held in registers.
__device__ double phi_support(const PolishArgsDev &a, PolishShared &sh, float2 b0, float2 b1,
                              const double2 *z, int s, double lam)
{
    const int lane = threadIdx.x;
    double acc = 0.0;
    for (int nn = lane, i = 0; nn < a.n; nn += 64, ++i) {
        const float2 bb = i == 0 ? b0 : b1;
        double rr = -(double)bb.x, ri = -(double)bb.y;
#pragma unroll 4
        for (int t = 0; t < s; ++t) {
            const double2 av = ASat(sh, nn, t);
            const double2 zv = z[t];
            rr += av.x * zv.x - av.y * zv.y;
            ri += av.x * zv.y + av.y * zv.x;
        }
        sh.r[nn] = make_double2(rr, ri);
        acc += rr * rr + ri * ri;
    }
    for (int t = lane; t < s; t += 64) acc += lam * sqrt(z[t].x * z[t].x + z[t].y * z[t].y);
    const double out = wsum(acc);
    __syncthreads();
    return out;
}

// Full pass at the current point (sh.r its residual): natural KKT residual,
// objective, and the worst off-support violator of |g| <= lambda.
// START: the point is the starting iterate x0 (its nonzero bins listed
// in sh.nzl[0..nnz)); else it is z on the working set (sh.sidx, s entries).
// The objective, the point and the KKT formula are FP64; the gradient
// g = 2 A^H r is accumulated in FP64, or with F32 in FP32 from the residual
// rounded once: its error, about 1e-7 of lambda, is far below the round-end
// target tol/10 it is tested against (not below mode 2's); the check of the
// starting point against tol itself stays FP64.
// Magnitudes are compared squared; the prox scale (a square root and a
// division) is formed only on lanes whose |v| passes the threshold.
template <bool START>
__device__ void pass_finish(PolishShared &sh, double acc, double l1, double km, double vbest,
                            double lam, double lf, double &F, double &kk, int &vidx);

template <bool START, bool F32>
__device__ void full_pass(const PolishArgsDev &a, PolishShared &sh, const float2 *x0, int s, int nnz,
                          double lam, double lf, double inv_lf, double &F, double &kk, int &vidx)
{
    using acc_t = typename std::conditional<F32, float, double>::type;
    const int lane = threadIdx.x;
    double acc = 0.0, l1 = 0.0, km = 0.0, vbest = 0.0;
    vidx = -1;
    for (int nn = lane; nn < a.n; nn += 64) {
        const double2 rv = sh.r[nn];
        acc += rv.x * rv.x + rv.y * rv.y;
        if (F32) sh.r32[nn] = make_float2((float)rv.x, (float)rv.y);
    }
    if (F32) __syncthreads();
    if (START) {
        for (int q = lane; q < nnz; q += 64) {
            const float2 v = x0[sh.nzl[q]];
            l1 += sqrt((double)v.x * v.x + (double)v.y * v.y);
        }
    } else {
        for (int t = lane; t < s; t += 64) l1 += sqrt(sh.z[t].x * sh.z[t].x + sh.z[t].y * sh.z[t].y);
    }
    const double tau = lam * inv_lf, tau2 = tau * tau;
    const double lv = lam * (1.0 + 1e-12), lv2 = lv * lv;
    // Lane bins m = lane + 64 c, two at a time: each batch of eight rows loads the
    // two columns together (16 loads in flight) and reuses each r_n across them.
    const int nb = (a.l + 63) / 64;
    for (int c0 = 0; c0 < nb; c0 += 2) {
        int mk[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int m = lane + 64 * (c0 + k);
            mk[k] = m < a.l ? m : 0;  // a column in range; its result is discarded
        }
        acc_t gr[2] = {}, gi[2] = {};
        auto rrow = [&](int n_) {
            if constexpr (F32) return sh.r32[n_];
            else return sh.r[n_];
        };
        int nn = 0;
        for (; nn + 8 <= a.n; nn += 8) {
            float2 af[2][8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int k = 0; k < 2; ++k) af[k][u] = a.A[(unsigned)((nn + u) * a.l_pad + mk[k])];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const auto rv = rrow(nn + u);
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    gr[k] += (acc_t)af[k][u].x * rv.x + (acc_t)af[k][u].y * rv.y;
                    gi[k] += (acc_t)af[k][u].x * rv.y - (acc_t)af[k][u].y * rv.x;
                }
            }
        }
        for (; nn < a.n; ++nn) {
            const auto rv = rrow(nn);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const float2 af = a.A[(unsigned)(nn * a.l_pad + mk[k])];
                gr[k] += (acc_t)af.x * rv.x + (acc_t)af.y * rv.y;
                gi[k] += (acc_t)af.x * rv.y - (acc_t)af.y * rv.x;
            }
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int m = lane + 64 * (c0 + k);
            if (m >= a.l) continue;
            double xr, xi;
            if (START) {
                const float2 v = x0[m];
                xr = v.x;
                xi = v.y;
            } else {
                const int t = sh.sidx[m];
                const double2 v = t >= 0 ? sh.z[t] : make_double2(0.0, 0.0);
                xr = v.x;
                xi = v.y;
            }
            const double g_r = 2.0 * gr[k], g_i = 2.0 * gi[k];  // g_m = 2 a_m^H r
            const double vr = xr - g_r * inv_lf, vi = xi - g_i * inv_lf;
            const double m2 = vr * vr + vi * vi;
            double er = xr, ei = xi;  // x - prox(v), prox(v) = 0 when |v| <= tau
            if (m2 > tau2) {
                const double sc = 1.0 - tau / sqrt(m2);
                er = xr - vr * sc;
                ei = xi - vi * sc;
            }
            km = fmax(km, er * er + ei * ei);
            const double gm2 = g_r * g_r + g_i * g_i;
            if (xr == 0.0 && xi == 0.0 && gm2 > lv2 && gm2 > vbest) {
                vbest = gm2;
                vidx = m;
            }
        }
    }
    pass_finish<START>(sh, acc, l1, km, vbest, lam, lf, F, kk, vidx);
}

// Reductions that end a pass: the objective, the natural KKT residual and the
// violators (the worst one in vidx; with kEnter > 1 the list sh.vl / sh.nv).
template <bool START>
__device__ void pass_finish(PolishShared &sh, double acc, double l1, double km, double vbest,
                            double lam, double lf, double &F, double &kk, int &vidx)
{
    const int lane = threadIdx.x;
    F = wsum(acc + lam * l1);
    kk = sqrt(wmax(km)) * lf / lam;
    if constexpr (kEnter > 1) {
        // the largest violations of distinct lanes, largest first (ties: lowest bin)
        if (!START) {
            double vrem = vbest;
            int nv = 0;
            for (int e = 0; e < kEnter; ++e) {
                const double vm = wmax(vrem);
                if (!(vm > 0.0)) break;
                uint64_t cl = __ballot(vrem == vm);
                int bm = -1;
                while (cl) {
                    const int ln = __ffsll((unsigned long long)cl) - 1;
                    cl &= cl - 1;
                    const int m = __builtin_amdgcn_readlane(vidx, ln);
                    if (bm < 0 || m < bm) bm = m;
                }
                if (vidx == bm) vrem = 0.0;
                if (lane == 0) sh.vl[nv] = bm;
                ++nv;
            }
            if (lane == 0) sh.nv = nv;
        }
    }
    // wave argmax of the violation (ties: lowest bin)
    const double vmax = wmax(vbest);
    uint64_t cand = __ballot(vmax > 0.0 && vbest == vmax);
    int best = -1;
    while (cand) {
        const int ln = __ffsll((unsigned long long)cand) - 1;
        cand &= cand - 1;
        const int m = __builtin_amdgcn_readlane(vidx, ln);
        if (best < 0 || m < best) best = m;
    }
    vidx = best;
}

// c = A^H b of the pixel in FP64 into the workgroup's buffer `cb` (lane m
// writes and later reads its own bins m = lane + 64 k); b is staged in sh.w.
__device__ void bin_rhs(const PolishArgsDev &a, PolishShared &sh, float2 b0, float2 b1, double2 *cb)
{
    const int lane = threadIdx.x;
    if (lane < a.n) sh.w[lane] = make_double2(b0.x, b0.y);
    if (lane + 64 < a.n) sh.w[lane + 64] = make_double2(b1.x, b1.y);
    __syncthreads();
    for (int m = lane; m < a.l; m += 64) {
        double cr = 0.0, ci = 0.0;
        int nn = 0;
        for (; nn + 8 <= a.n; nn += 8) {
            float2 af[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) af[u] = a.A[(unsigned)((nn + u) * a.l_pad + m)];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double2 bv = sh.w[nn + u];
                cr += (double)af[u].x * bv.x + (double)af[u].y * bv.y;  // conj(a) b
                ci += (double)af[u].x * bv.y - (double)af[u].y * bv.x;
            }
        }
        for (; nn < a.n; ++nn) {
            const float2 af = a.A[(unsigned)(nn * a.l_pad + m)];
            const double2 bv = sh.w[nn];
            cr += (double)af.x * bv.x + (double)af.y * bv.y;
            ci += (double)af.x * bv.y - (double)af.y * bv.x;
        }
        cb[m] = make_double2(cr, ci);
    }
    __syncthreads();
}

// The round-end pass in Gram form: g_m / 2 = sum_t H[m][S_t] z_t - c_m with
// H = A^H A (FP64; H[m][s] = conj(H[s][m]), row S_t read contiguously) and
// c = A^H b from bin_rhs, then the same natural KKT residual, objective (from
// the exact residual sh.r) and violators as full_pass.  It reads 16 (|S| + 1)
// bytes a bin where the residual form reads a column of A (8 N bytes), so it
// is the cheaper one while 2 (|S| + 1) <= N; everything stays FP64.
__device__ void gram_pass(const PolishArgsDev &a, PolishShared &sh, const double2 *cb, int s,
                          double lam, double lf, double inv_lf, double &F, double &kk, int &vidx)
{
    const int lane = threadIdx.x;
    double acc = 0.0, l1 = 0.0, km = 0.0, vbest = 0.0;
    vidx = -1;
    for (int nn = lane; nn < a.n; nn += 64) {
        const double2 rv = sh.r[nn];
        acc += rv.x * rv.x + rv.y * rv.y;
    }
    for (int t = lane; t < s; t += 64) l1 += sqrt(sh.z[t].x * sh.z[t].x + sh.z[t].y * sh.z[t].y);
    const double tau = lam * inv_lf, tau2 = tau * tau;
    const double lv = lam * (1.0 + 1e-12), lv2 = lv * lv;
    auto bin_done = [&](int m, double gr, double gi) {
        const int ts = sh.sidx[m];
        const double2 v = ts >= 0 ? sh.z[ts] : make_double2(0.0, 0.0);
        const double xr = v.x, xi = v.y;
        const double g_r = 2.0 * gr, g_i = 2.0 * gi;
        const double vr = xr - g_r * inv_lf, vi = xi - g_i * inv_lf;
        const double m2 = vr * vr + vi * vi;
        double er = xr, ei = xi;  // x - prox(v), prox(v) = 0 when |v| <= tau
        if (m2 > tau2) {
            const double sc = 1.0 - tau / sqrt(m2);
            er = xr - vr * sc;
            ei = xi - vi * sc;
        }
        km = fmax(km, er * er + ei * ei);
        const double gm2 = g_r * g_r + g_i * g_i;
        if (xr == 0.0 && xi == 0.0 && gm2 > lv2 && gm2 > vbest) {
            vbest = gm2;
            vidx = m;
        }
    };
    // two bins a lane (m0, m0 + 64) and four working-set rows per batch: the pass
    // is latency bound on the rows of H (4 MB at L = 512, beyond one XCD's L2), so
    // a batch's eight loads are issued before any is used (eight rows a batch
    // spill more and measured slower)
    for (int m0 = lane; m0 < a.l; m0 += 128) {
        const int m1 = m0 + 64;
        const bool two = m1 < a.l;
        const int m1c = two ? m1 : m0;
        const double2 c0 = cb[m0], c1 = cb[m1c];
        double gr0 = -c0.x, gi0 = -c0.y, gr1 = -c1.x, gi1 = -c1.y;
        for (int t0 = 0; t0 < s; t0 += 4) {
            double2 h0[4], h1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (t0 + u < s) {
                    const size_t row = (size_t)sh.S[t0 + u] * a.l;
                    h0[u] = a.H[row + m0];
                    h1[u] = a.H[row + m1c];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (t0 + u < s) {
                    const double2 zv = sh.z[t0 + u];  // conj(H[S_t][m]) z_t
                    gr0 += h0[u].x * zv.x + h0[u].y * zv.y;
                    gi0 += h0[u].x * zv.y - h0[u].y * zv.x;
                    gr1 += h1[u].x * zv.x + h1[u].y * zv.y;
                    gi1 += h1[u].x * zv.y - h1[u].y * zv.x;
                }
            }
        }
        bin_done(m0, gr0, gi0);
        if (two) bin_done(m1, gr1, gi1);
    }
    pass_finish<false>(sh, acc, l1, km, vbest, lam, lf, F, kk, vidx);
}

// Gram entries G_tu = a_t^H a_u (t >= u) for the packed indices [e0, e1) into
// sh.Gc.  Lanes are split into 64/E groups over the rows of A_S when the
// entries fit E lanes, and the group partial sums are combined with shuffles.
__device__ void gram_entries(const PolishArgsDev &a, PolishShared &sh, int e0, int e1)
{
    const int lane = threadIdx.x;
    const int ne = e1 - e0;
    const int E = ne <= 16 ? 16 : (ne <= 32 ? 32 : 64), G = 64 / E;
    const int q = lane / E;
    for (int f0 = 0; f0 < ne; f0 += E) {
        const int e = e0 + f0 + lane % E;
        const bool act = e < e1;
        int t = 0;
        if (act)
            while ((t + 1) * (t + 2) / 2 <= e) ++t;
        const int u = act ? e - t * (t + 1) / 2 : 0;
        double gr = 0.0, gi = 0.0;
        if (act) {
#pragma unroll 4
            for (int nn = q; nn < a.n; nn += G) {
                const double2 p1 = ASat(sh, nn, t), p2 = ASat(sh, nn, u);
                gr += p1.x * p2.x + p1.y * p2.y;  // conj(p1) p2
                gi += p1.x * p2.y - p1.y * p2.x;
            }
        }
        if (G >= 4) {
            gr += __shfl_xor(gr, 16, 64);
            gi += __shfl_xor(gi, 16, 64);
        }
        if (G >= 2) {
            gr += __shfl_xor(gr, 32, 64);
            gi += __shfl_xor(gi, 32, 64);
        }
        if (act && q == 0) sh.Gc[e] = make_double2(gr, gi);
    }
    __syncthreads();
}

// Remove slot t from the packed Gram of order s (the rows and columns after it
// move up by one).
__device__ void gram_drop(PolishShared &sh, int s, int t)
{
    const int lane = threadIdx.x;
    constexpr int KD = ((kMaxSupp - 1) * kMaxSupp / 2 + 63) / 64;  // entries per lane
    const int ne = (s - 1) * s / 2;
    double2 v[KD];
#pragma unroll
    for (int k = 0; k < KD; ++k) {
        const int e = lane + 64 * k;
        v[k] = make_double2(0.0, 0.0);
        if (e < ne) {
            int i = 0;
            while ((i + 1) * (i + 2) / 2 <= e) ++i;
            const int j = e - i * (i + 1) / 2;
            v[k] = sh.Gc[tri(i + (i >= t), j + (j >= t))];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KD; ++k)
        if (lane + 64 * k < ne) sh.Gc[lane + 64 * k] = v[k];
    __syncthreads();
}

// G_tu for any t, u < s from the packed lower triangle (G_ut = conj(G_tu)).
__device__ __forceinline__ double2 gram_at(const PolishShared &sh, int t, int u)
{
    if (t >= u) return sh.Gc[tri(t, u)];
    const double2 g = sh.Gc[tri(u, t)];
    return make_double2(g.x, -g.y);
}

// The packed Newton matrix of order m2 = 2s,
//   2 [[Re G, -Im G], [Im G, Re G]] + lambda blkdiag((I - u u^T)/|z|) + mu I,
// in sh.H, one entry per lane: index i < s is the real and s + i the imaginary
// part of slot i; u and 1/|z| per slot come from sh.ur, sh.ui, sh.iz.
__device__ void build_hessian(PolishShared &sh, int s, double lam, double mu)
{
    const int lane = threadIdx.x;
    const int m2 = 2 * s, ne = m2 * (m2 + 1) / 2;
    for (int e = lane; e < ne; e += 64) {
        // row i of packed index e: the root of i (i + 1) / 2 = e, then corrected
        int i = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
        if ((i + 1) * (i + 2) / 2 <= e) ++i;
        if (i * (i + 1) / 2 > e) --i;
        const int k = e - i * (i + 1) / 2;
        const bool pi = i >= s, pk = k >= s;
        const int ti = pi ? i - s : i, tk = pk ? k - s : k;
        const int hi = ti > tk ? ti : tk, lo = ti > tk ? tk : ti;
        const double2 g = sh.Gc[tri(hi, lo)];
        const double gy = ti >= tk ? g.y : -g.y;  // Im G[ti][tk]
        double h = pi == pk ? 2.0 * g.x : (pi ? 2.0 * gy : -2.0 * gy);
        if (ti == tk) {
            const double ur = sh.ur[ti], ui = sh.ui[ti], iz = sh.iz[ti];
            if (pi == pk) h += lam * (1.0 - (pi ? ui * ui : ur * ur)) * iz + mu;
            else h -= lam * ur * ui * iz;
        }
        sh.H[e] = h;
    }
    __syncthreads();
}

// In-place Cholesky of the packed matrix of order m2 (strict lower part of the
// factor in sh.H, reciprocal of its diagonal in sh.invd); false if not positive definite.
__device__ bool cholesky(PolishShared &sh, int m2)
{
    const int lane = threadIdx.x;
    bool good = true;
    for (int jj = 0; jj < m2; ++jj) {
        double djj = sh.H[tri(jj, jj)];
#pragma unroll 4
        for (int k = 0; k < jj; ++k) djj -= sh.H[tri(jj, k)] * sh.H[tri(jj, k)];
        if (!(djj > 0.0)) {
            good = false;
            break;
        }
        // 1/sqrt(djj): hardware estimate refined by two Newton-Raphson steps
        double inv = __builtin_amdgcn_rsq(djj);
        inv = inv * fma(-0.5 * djj, inv * inv, 1.5);
        inv = inv * fma(-0.5 * djj, inv * inv, 1.5);
        for (int i = jj + 1 + lane; i < m2; i += 64) {
            double t = sh.H[tri(i, jj)];
#pragma unroll 4
            for (int k = 0; k < jj; ++k) t -= sh.H[tri(i, k)] * sh.H[tri(jj, k)];
            sh.H[tri(i, jj)] = t * inv;
        }
        if (lane == 0) sh.invd[jj] = inv;
        __syncthreads();
    }
    __syncthreads();
    return good;
}

// Solve L L^T d = -grd with the factor in sh.H / sh.invd; lane k ends holding d_k
// (column-oriented substitutions, one broadcast per column).
__device__ double newton_dir(const PolishShared &sh, int m2)
{
    const int lane = threadIdx.x;
    double v = lane < m2 ? -sh.grd[lane] : 0.0;
    const double invl = lane < m2 ? sh.invd[lane] : 0.0;
    for (int i = 0; i < m2; ++i) {
        const double yi = lane_value(v, i) * lane_value(invl, i);
        if (lane == i) v = yi;
        else if (lane > i && lane < m2) v -= sh.H[tri(lane, i)] * yi;
    }
    for (int i = m2 - 1; i >= 0; --i) {
        const double di = lane_value(v, i) * lane_value(invl, i);
        if (lane == i) v = di;
        else if (lane < i) v -= sh.H[tri(i, lane)] * di;
    }
    return v;
}

// The Newton system (H + mu I) d = -grd of order m2 <= NS solved in registers:
// lane i < NS holds row i of H (the identity pads rows and columns m2..NS-1),
// a right-looking U D U^T factorisation broadcasts each column with readlane,
// so that both substitutions need one broadcast per column and no selects; U
// is transposed once through LDS for the backward substitution.
// Returns false (wave-uniform) if H is not positive definite; lane i ends
// holding d_i.
template <int NS>
__device__ bool newton_regs(PolishShared &sh, int m2, double mu, double &d)
{
    const int lane = threadIdx.x;
    double row[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        if (lane < m2 && k < m2)
            row[k] = (k <= lane ? sh.H[tri(lane, k)] : sh.H[tri(k, lane)]) + (k == lane ? mu : 0.0);
        else
            row[k] = k == lane ? 1.0 : 0.0;
    }
    // H = U D U^T, U unit lower, D diagonal (a square-root-free Cholesky): lane i
    // keeps U_ij in row[j] below the diagonal (0 on and above it) and 1/D_ii in
    // dinv.  Column j is eliminated with its unscaled entries c_kj = D_j U_kj,
    // whose broadcasts do not wait for the reciprocal of the pivot.
    double dinv = 0.0;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const double piv = lane_value(row[j], j);
        if (!(piv > 0.0)) return false;
        // 1/piv: hardware estimate refined by one Newton-Raphson step
        double rp = __builtin_amdgcn_rcp(piv);
        rp = fma(rp, fma(-piv, rp, 1.0), rp);
        if (lane == j) dinv = rp;
        const double cj = row[j];                 // lane i >= j: c_ij
        const double uj = lane > j ? cj * rp : 0.0;  // U_ij
#pragma unroll
        for (int k = j + 1; k < NS; ++k) row[k] -= uj * lane_value(cj, k);  // - U_ij c_kj
        row[j] = uj;
    }
    // U y = -grd (unit diagonal: y_j is final when its column is reached)
    double v = lane < m2 ? -sh.grd[lane] : 0.0;
#pragma unroll
    for (int j = 0; j < NS; ++j) v -= row[j] * lane_value(v, j);
    // D w = y on each lane
    v *= dinv;
    // U^T d = w: U_ji (i < j) is lane j's row[i]; the factor is transposed through
    // LDS (past the packed Hessian, which a retry with a shift still needs) so
    // that lane i holds column i of U
    double *T = sh.H + kHLen - NS * NS;
    if (lane < NS) {
#pragma unroll
        for (int k = 0; k < NS; ++k) T[lane * NS + k] = row[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NS; ++k) row[k] = lane < NS ? T[k * NS + lane] : 0.0;  // U_ki
#pragma unroll
    for (int j = NS - 1; j >= 0; --j) v -= row[j] * lane_value(v, j);
    __syncthreads();
    d = v;
    return true;
}

__device__ __forceinline__ void polish_stack(const PolishArgsDev &a)
{
    __shared__ PolishShared sh;
    extern __shared__ __align__(16) unsigned char dyn[];
    const int lane = threadIdx.x;
    if (lane == 0) {
        unsigned char *p = dyn;
        sh.r = reinterpret_cast<double2 *>(p);
        p += (size_t)a.n * sizeof(double2);
        sh.w = reinterpret_cast<double2 *>(p);
        sh.r32 = reinterpret_cast<float2 *>(p);  // the pass's copy of r shares w's space
        p += (size_t)a.n * sizeof(double2);
        sh.AS = reinterpret_cast<float2 *>(p);
        sh.nzl = reinterpret_cast<int16_t *>(p);  // used before A_S is staged
        p += polish_as_bytes(a.n, a.l_pad);
        sh.sidx = reinterpret_cast<int8_t *>(p);
    }
    __syncthreads();
    const double lf = a.consts->lf;
    const double inv_lf = 1.0 / lf;
    const double gstop = a.mode == 2 ? 1e-13 : 1e-2 * (double)a.tol;
    const double kstop = a.mode == 2 ? 1e-10 : 1e-1 * (double)a.tol;
    const uint32_t count = *a.count;
    double2 *cb = a.cbuf + (size_t)blockIdx.x * a.l;  // A^H b of this workgroup's pixel
    bool have_c = false;
    // flops of the algorithm (wave-uniform), 8 per complex multiply-add: FP64
    // work in fl, the FP32 round-end gradient of mode 1 in fl32
    unsigned long long fl = 0, fl32 = 0;
    const unsigned long long f8n = 8ull * (unsigned long long)a.n;
    // pixels are taken from a shared counter, so a workgroup that becomes
    // resident late only finds what is left
    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(a.next, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= count) break;
        const int64_t p = a.list[item];
        const float lam_f = a.lambda[p * a.lambda_stride];
        if (!(lam_f > 0.0f) || !isfinite(lam_f)) continue;
        const double lam = lam_f;
        const float2 *b = a.B + (size_t)p * a.n;
        const float2 b0 = lane < a.n ? b[lane] : make_float2(0.0f, 0.0f);
        const float2 b1 = lane + 64 < a.n ? b[lane + 64] : make_float2(0.0f, 0.0f);
        float2 *xo = a.X + (size_t)p * a.l;
        for (int m = lane; m < a.l_pad; m += 64) sh.sidx[m] = -1;
        if (lane == 0) sh.sb = -1;
        __syncthreads();
        double fbest;
        if (a.mode == 1 && (a.status[p] & L1LS_PX_MAX_ITER) != 0 && a.R) {
            // the FP32 stage's own KKT test failed: the pixel is refined, and only
            // the objective of the starting point is needed, from the residual
            // that stage kept and ||x0||_1.  That residual is carried by recursion
            // in FP32 and drifts (about 1e-6 relative after tens of iterations),
            // more than F(x0) - F* of a pixel that only just missed tol; the
            // starting point is a guard against a failed refinement, so its
            // estimate is raised by a margin well above that drift
            const float2 *rp = a.R + (size_t)p * a.n;
            double acc = 0.0;
            for (int nn = lane; nn < a.n; nn += 64) {
                const float2 rv = rp[nn];
                acc += (double)rv.x * rv.x + (double)rv.y * rv.y;
            }
            for (int m = lane; m < a.l; m += 64) {
                const float2 v = xo[m];
                acc += lam * sqrt((double)v.x * v.x + (double)v.y * v.y);
            }
            fbest = wsum(acc) * (1.0 + 1e-3);
        } else if (a.mode == 2 || (a.status[p] & L1LS_PX_MAX_ITER) != 0) {
            // only the objective of the starting point is needed (mode 2 refines
            // every pixel; a capped pixel without a kept residual): FP64 from the
            // residual of its nonzero bins
            residual_start(a, sh, b, xo);
            fl += f8n * (unsigned long long)sh.cnt;
            double acc = 0.0;
            for (int nn = lane; nn < a.n; nn += 64) acc += sh.r[nn].x * sh.r[nn].x + sh.r[nn].y * sh.r[nn].y;
            for (int q = lane; q < sh.cnt; q += 64) {
                const float2 v = xo[sh.nzl[q]];
                acc += lam * sqrt((double)v.x * v.x + (double)v.y * v.y);
            }
            fbest = wsum(acc);
        } else {
            // mode 1, a pixel the FP32 stage retired: objective and FP64 natural
            // KKT residual of the starting point decide whether it is solved
            residual_start(a, sh, b, xo);
            fl += f8n * (unsigned long long)sh.cnt;
            double kk0;
            int vdummy;
            // FP64 throughout: this decides "already solved" against tol itself
            full_pass<true, false>(a, sh, xo, 0, sh.cnt, lam, lf, inv_lf, fbest, kk0, vdummy);
            fl += f8n * (unsigned long long)a.l;
            __syncthreads();
            if (kk0 <= (double)a.tol) continue;  // already solved
        }
        have_c = false;
        // -- working set: the local maxima of |x| (FISTA spreads one scatterer
        //    over neighbouring bins); at most kMaxSupp, the largest kept
        if (lane == 0) sh.cnt = 0;
        __syncthreads();
        for (int m0 = 0; m0 < a.l; m0 += 64) {
            const int m = m0 + lane;
            bool pk = false;
            float2 xv = make_float2(0.0f, 0.0f);
            if (m < a.l) {
                xv = xo[m];
                const float2 xl = m > 0 ? xo[m - 1] : make_float2(0.0f, 0.0f);
                const float2 xr = m + 1 < a.l ? xo[m + 1] : make_float2(0.0f, 0.0f);
                const double mag = (double)xv.x * xv.x + (double)xv.y * xv.y;
                const double ml = (double)xl.x * xl.x + (double)xl.y * xl.y;
                const double mr = (double)xr.x * xr.x + (double)xr.y * xr.y;
                pk = mag > 0.0 && mag >= ml && mag >= mr;
            }
            const uint64_t bal = __ballot(pk);
            if (bal && lane == 0) {
                // keep the kMaxSupp largest peaks (replace the smallest kept one)
                uint64_t bits = bal;
                while (bits) {
                    const int q = __ffsll((unsigned long long)bits) - 1;
                    bits &= bits - 1;
                    const int mm = m0 + q;
                    const double2 xq = make_double2(lane_value_f(xv.x, q), lane_value_f(xv.y, q));
                    const double mag = xq.x * xq.x + xq.y * xq.y;
                    const int s = sh.cnt;
                    if (s < kMaxSupp) {
                        sh.S[s] = mm;
                        sh.z[s] = xq;
                        sh.cnt = s + 1;
                    } else {
                        int wi = 0;
                        double wm = sh.z[0].x * sh.z[0].x + sh.z[0].y * sh.z[0].y;
                        for (int t = 1; t < s; ++t) {
                            const double qv = sh.z[t].x * sh.z[t].x + sh.z[t].y * sh.z[t].y;
                            if (qv < wm) { wm = qv; wi = t; }
                        }
                        if (mag > wm) {
                            sh.S[wi] = mm;
                            sh.z[wi] = xq;
                        }
                    }
                }
            }
            __syncthreads();
        }
        // ... and the larger neighbour of each peak (the exact solution of an
        // off-grid scatterer usually sits on two adjacent bins; seeding both saves
        // the round that would admit the second as a violator)
        {
            // lane t < np reads the neighbours of peak t; lane 0 appends them in order
            const int np = sh.cnt;
            int nb = -1;
            float2 xn = make_float2(0.0f, 0.0f);
            if (lane < np) {
                const int m = sh.S[lane];
                const float2 xl = m > 0 ? xo[m - 1] : make_float2(0.0f, 0.0f);
                const float2 xr = m + 1 < a.l ? xo[m + 1] : make_float2(0.0f, 0.0f);
                const double ml = (double)xl.x * xl.x + (double)xl.y * xl.y;
                const double mr = (double)xr.x * xr.x + (double)xr.y * xr.y;
                const double mn = ml >= mr ? ml : mr;
                if (mn > 0.0) {
                    nb = ml >= mr ? m - 1 : m + 1;
                    xn = ml >= mr ? xl : xr;
                }
            }
            if (lane == 0) {
                int cnt = np;
                for (int t = 0; t < np && cnt < kMaxSupp; ++t) {
                    const int nbt = __builtin_amdgcn_readlane(nb, t);
                    if (nbt < 0) continue;
                    bool dup = false;
                    for (int u = 0; u < cnt; ++u) dup = dup || sh.S[u] == nbt;
                    if (dup) continue;
                    sh.S[cnt] = nbt;
                    sh.z[cnt] = make_double2(lane_value_f(xn.x, t), lane_value_f(xn.y, t));
                    ++cnt;
                }
                sh.cnt = cnt;
            }
        }
        __syncthreads();
        int s = sh.cnt;
        for (int e = lane; e < a.n * s; e += 64) {  // all columns of the working set at once
            const int nn = e / s, t = e % s;
            sh.AS[nn * kMaxSupp + t] = a.A[(size_t)nn * a.l_pad + sh.S[t]];
        }
        __syncthreads();
        gram_entries(a, sh, 0, s * (s + 1) / 2);
        fl += f8n * (unsigned long long)(s * (s + 1) / 2);
        // r = A_S z - b, c = A_S^H r and phi are formed afresh for the seeded
        // working set; afterwards every change updates them exactly: a step
        // z += t d by r += t A_S d, c += t G d and the change the line search
        // measured, a drop or an entry by the column's rank-one term.
        bool fresh = true;
        double kfin = 1e300;  // KKT residual of the last round-end pass
        // Newton on a working set stops at gstop, except in mode 2 while the full
        // pass still finds violators: there the set is about to change and a
        // subproblem solved to mode 1's accuracy picks the same violator, so the
        // tight target is taken only once the set looks final
        double gcur = a.mode == 2 ? 1e-2 * (double)a.tol : gstop;
        double ph = 0.0;
        for (int round = 0; round < a.rounds; ++round) {
            for (int it = 0; it < 50 && s > 0; ++it) {
                const int m2 = 2 * s;
                if (fresh) {
                    ph = phi_support(a, sh, b0, b1, sh.z, s, lam);
                    // c = A_S^H r (64 / kMaxSupp lane groups over the rows of A_S)
                    constexpr int NG = 64 / kMaxSupp;
                    const int t = lane % kMaxSupp, q = lane / kMaxSupp;
                    double gr = 0.0, gi = 0.0;
                    if (t < s) {
#pragma unroll 4
                        for (int nn = q; nn < a.n; nn += NG) {
                            const double2 av = ASat(sh, nn, t), rv = sh.r[nn];
                            gr += av.x * rv.x + av.y * rv.y;
                            gi += av.x * rv.y - av.y * rv.x;
                        }
                    }
                    if (NG >= 8) {
                        gr += __shfl_xor(gr, 8, 64);
                        gi += __shfl_xor(gi, 8, 64);
                    }
                    if (NG >= 4) {
                        gr += __shfl_xor(gr, 16, 64);
                        gi += __shfl_xor(gi, 16, 64);
                    }
                    gr += __shfl_xor(gr, 32, 64);
                    gi += __shfl_xor(gi, 32, 64);
                    if (t < s && q == 0) sh.c[t] = make_double2(gr, gi);
                    __syncthreads();
                    fl += 2ull * f8n * (unsigned long long)s;
                    fresh = false;
                }
                // gradient of phi on the working set (real pairs)
                double gmax = 0.0;
                if (lane < s) {
                    const double2 zv = sh.z[lane], cv = sh.c[lane];
                    const double iz = 1.0 / sqrt(zv.x * zv.x + zv.y * zv.y);
                    const double gr = 2.0 * cv.x + lam * zv.x * iz;
                    const double gi = 2.0 * cv.y + lam * zv.y * iz;
                    sh.grd[lane] = gr;
                    sh.grd[lane + s] = gi;
                    sh.ur[lane] = zv.x * iz;
                    sh.ui[lane] = zv.y * iz;
                    sh.iz[lane] = iz;
                    gmax = sqrt(gr * gr + gi * gi);
                }
                gmax = wmax(gmax);
                __syncthreads();
                if (gmax <= gcur * lam) break;
                // Newton direction; shifted retries while the Hessian is not PD
                double mu = 0.0, dv = 0.0;
                bool ok = false;
                if (m2 <= 16) build_hessian(sh, s, lam, 0.0);
                for (int attempt = 0; attempt < 8 && !ok; ++attempt) {
                    fl += (unsigned long long)(m2 * m2 * m2 / 3 + 2 * m2 * m2);
                    if (m2 <= 4) {
                        ok = newton_regs<4>(sh, m2, mu, dv);
                    } else if (m2 <= 6) {
                        ok = newton_regs<6>(sh, m2, mu, dv);
                    } else if (m2 <= 8) {
                        ok = newton_regs<8>(sh, m2, mu, dv);
                    } else if (m2 <= 10) {
                        ok = newton_regs<10>(sh, m2, mu, dv);
                    } else if (m2 <= 12) {
                        ok = newton_regs<12>(sh, m2, mu, dv);
                    } else if (m2 <= 16) {
                        ok = newton_regs<16>(sh, m2, mu, dv);
                    } else {
                        build_hessian(sh, s, lam, mu);
                        ok = cholesky(sh, m2);
                        if (ok) dv = newton_dir(sh, m2);
                    }
                    mu = mu == 0.0 ? 1e-14 * lf : mu * 100.0;
                }
                if (!ok) break;
                if (lane < m2) sh.dir[lane] = dv;
                __syncthreads();
                // the coordinate the step turns round most leaves the working set
                // (lanes over coordinates; ties: the lowest slot)
                double cq = 1.0;
                if (lane < s) {
                    const double2 zv = sh.z[lane];
                    const double nr = zv.x + sh.dir[lane], ni = zv.y + sh.dir[lane + s];
                    cq = (zv.x * nr + zv.y * ni) / (zv.x * zv.x + zv.y * zv.y);
                }
                uint64_t cand = __ballot(lane < s && cq <= 0.0);
                int drop = -1;
                double worst = 0.0;
                while (cand) {
                    const int t = __ffsll((unsigned long long)cand) - 1;
                    cand &= cand - 1;
                    const double c = lane_value(cq, t);
                    if (drop < 0 || c < worst) {
                        drop = t;
                        worst = c;
                    }
                }
                if (drop >= 0) {
                    // z_drop -> 0: r -= a z_drop, c_t -= G[t][drop] z_drop and
                    // phi changes by -2 Re(conj(z_drop) c_drop) + G[drop][drop] |z_drop|^2 - lambda |z_drop|
                    const double2 zd = sh.z[drop], cd = sh.c[drop], gdd = sh.Gc[tri(drop, drop)];
                    const double azd = sqrt(zd.x * zd.x + zd.y * zd.y);
                    ph += -2.0 * (zd.x * cd.x + zd.y * cd.y) + gdd.x * azd * azd - lam * azd;
                    for (int nn = lane; nn < a.n; nn += 64) {
                        const double2 av = ASat(sh, nn, drop);
                        sh.r[nn] = make_double2(sh.r[nn].x - (av.x * zd.x - av.y * zd.y),
                                                sh.r[nn].y - (av.x * zd.y + av.y * zd.x));
                    }
                    double2 cnew = make_double2(0.0, 0.0);
                    if (lane < s) {
                        const double2 g = gram_at(sh, lane, drop), cv = sh.c[lane];
                        cnew = make_double2(cv.x - (g.x * zd.x - g.y * zd.y), cv.y - (g.x * zd.y + g.y * zd.x));
                    }
                    __syncthreads();
                    // remove column `drop` from the working set (lanes over rows of A_S)
                    for (int nn = lane; nn < a.n; nn += 64)
                        for (int t = drop; t + 1 < s; ++t) sh.AS[nn * kMaxSupp + t] = sh.AS[nn * kMaxSupp + t + 1];
                    if (lane < s && lane != drop) sh.c[lane > drop ? lane - 1 : lane] = cnew;
                    if (lane == 0) {
                        for (int t = drop; t + 1 < s; ++t) {
                            sh.S[t] = sh.S[t + 1];
                            sh.z[t] = sh.z[t + 1];
                        }
                    }
                    gram_drop(sh, s, drop);
                    --s;
                    continue;
                }
                const double slope = wsum(lane < m2 ? sh.grd[lane] * dv : 0.0);
                // w = A_S d with <r, w> and ||w||^2: phi(z + t d) - phi(z) =
                //   t (2 Re<r, w> + t ||w||^2) + lambda (||z + t d||_1 - ||z||_1)
                double rw = 0.0, ww = 0.0;
                for (int nn = lane; nn < a.n; nn += 64) {
                    double wr_ = 0.0, wi_ = 0.0;
#pragma unroll 4
                    for (int t = 0; t < s; ++t) {
                        const double2 av = ASat(sh, nn, t);
                        const double dr = sh.dir[t], di = sh.dir[t + s];
                        wr_ += av.x * dr - av.y * di;
                        wi_ += av.x * di + av.y * dr;
                    }
                    sh.w[nn] = make_double2(wr_, wi_);
                    const double2 rv = sh.r[nn];
                    rw += rv.x * wr_ + rv.y * wi_;
                    ww += wr_ * wr_ + wi_ * wi_;
                }
                rw = wsum(rw);
                ww = wsum(ww);
                fl += f8n * (unsigned long long)s;
                if (-slope <= 1e-14 * ph) {
                    // predicted decrease below the rounding of phi: take the step, stop
                    for (int t = lane; t < s; t += 64)
                        sh.z[t] = make_double2(sh.z[t].x + sh.dir[t], sh.z[t].y + sh.dir[t + s]);
                    for (int nn = lane; nn < a.n; nn += 64)
                        sh.r[nn] = make_double2(sh.r[nn].x + sh.w[nn].x, sh.r[nn].y + sh.w[nn].y);
                    __syncthreads();
                    break;
                }
                // Armijo backtracking on phi
                double step = 1.0, delta = 0.0;
                bool acc = false;
                double az = 0.0;  // |z_t| of lane t
                if (lane < s) az = sqrt(sh.z[lane].x * sh.z[lane].x + sh.z[lane].y * sh.z[lane].y);
                for (int ls = 0; ls < 40; ++ls) {
                    double dl1 = 0.0;
                    if (lane < s) {
                        const double nr = sh.z[lane].x + step * sh.dir[lane];
                        const double ni = sh.z[lane].y + step * sh.dir[lane + s];
                        dl1 = sqrt(nr * nr + ni * ni) - az;
                    }
                    delta = step * (2.0 * rw + step * ww) + lam * wsum(dl1);
                    if (delta <= 1e-4 * step * slope) {
                        acc = true;
                        break;
                    }
                    step *= 0.5;
                }
                if (!acc) break;
                // z += t d, r += t w, c += t G d
                if (lane < s) {
                    double gdr = 0.0, gdi = 0.0;
                    for (int u = 0; u < s; ++u) {
                        const double2 g = gram_at(sh, lane, u);
                        const double dr = sh.dir[u], di = sh.dir[u + s];
                        gdr += g.x * dr - g.y * di;
                        gdi += g.x * di + g.y * dr;
                    }
                    sh.c[lane] = make_double2(sh.c[lane].x + step * gdr, sh.c[lane].y + step * gdi);
                    sh.z[lane] = make_double2(sh.z[lane].x + step * sh.dir[lane], sh.z[lane].y + step * sh.dir[lane + s]);
                }
                for (int nn = lane; nn < a.n; nn += 64)
                    sh.r[nn] = make_double2(sh.r[nn].x + step * sh.w[nn].x, sh.r[nn].y + step * sh.w[nn].y);
                fl += 8ull * (unsigned long long)(s * s);
                ph += delta;
                __syncthreads();
            }
            // the working set as the current point; its residual
            for (int t = lane; t < s; t += 64) sh.sidx[sh.S[t]] = (int8_t)t;
            __syncthreads();
            if (fresh) phi_support(a, sh, b0, b1, sh.z, s, lam);  // r only: c is formed afresh next round
            double F, kk;
            int vidx;
            if (round > 0 && 2 * (s + 1) <= a.n) {
                // Gram form (FP64): |S| rows of A^H A and A^H b instead of a column of A a bin
                // (from the second round on: A^H b costs one pass of its own)
                if (!have_c) {
                    bin_rhs(a, sh, b0, b1, cb);
                    fl += f8n * (unsigned long long)a.l;
                    have_c = true;
                }
                gram_pass(a, sh, cb, s, lam, lf, inv_lf, F, kk, vidx);
                fl += f8n * (unsigned long long)s + 8ull * (unsigned long long)a.l * (unsigned long long)s;
            } else if (a.mode == 1) {
                full_pass<false, true>(a, sh, xo, s, 0, lam, lf, inv_lf, F, kk, vidx);
                fl += f8n * (unsigned long long)s;
                fl32 += f8n * (unsigned long long)a.l;
            } else {
                full_pass<false, false>(a, sh, xo, s, 0, lam, lf, inv_lf, F, kk, vidx);
                fl += f8n * (unsigned long long)(s + a.l);
            }
            kfin = kk;
            if (F <= fbest) {
                fbest = F;
                if (lane < s) {
                    sh.Sb[lane] = sh.S[lane];
                    sh.zb[lane] = sh.z[lane];
                }
                if (lane == 0) sh.sb = s;
            }
            __syncthreads();
            for (int t = lane; t < s; t += 64) sh.sidx[sh.S[t]] = -1;
            __syncthreads();
            if (kk <= kstop) break;
            if (vidx < 0) {
                if (gcur > gstop) {  // no violator left: the same set to the tight target
                    gcur = gstop;
                    continue;
                }
                break;
            }
            if (s >= kMaxSupp) {
                // the working set is full and the point is not solved: a wider pass
                // (a later launch) takes the pixel from its best point so far
                if (kTier < 2 && a.overflow && kk > (double)a.tol && lane == 0)
                    a.overflow[atomicAdd(a.overflow_count, 1u)] = (int32_t)p;
                break;
            }
            // the worst violator enters at its exact coordinate minimiser (the wide
            // pass: up to kEnter of them, one after another against the updated r)
            // (lanes over rows: the column is staged and a^H r, ||a||^2 formed at once)
            const int nv = kEnter > 1 ? sh.nv : 1;
            int entered = 0;
            for (int e = 0; e < nv && s < kMaxSupp; ++e) {
            if (kEnter > 1) vidx = sh.vl[e];
            double gr = 0.0, gi = 0.0, cn = 0.0;
            for (int nn = lane; nn < a.n; nn += 64) {
                const float2 af = a.A[(size_t)nn * a.l_pad + vidx];
                sh.AS[nn * kMaxSupp + s] = af;
                const double2 rv = sh.r[nn];
                gr += af.x * rv.x + af.y * rv.y;
                gi += af.x * rv.y - af.y * rv.x;
                cn += (double)af.x * af.x + (double)af.y * af.y;
            }
            gr = wsum(gr);
            gi = wsum(gi);
            cn = wsum(cn);
            fl += f8n;
            // argmin_z |a z + r|^2 + lambda |z| = -S_{lambda/2}(a^H r) / ||a||^2
            const double mag = sqrt(gr * gr + gi * gi), tau = 0.5 * lam;
            const double sc = mag > tau ? (1.0 - tau / mag) / cn : 0.0;
            const double2 zn = make_double2(-gr * sc, -gi * sc);
            if (lane == 0) {
                sh.S[s] = vidx;
                sh.z[s] = zn;
            }
            __syncthreads();
            if (sc == 0.0) continue;  // no longer a violator
            ++entered;
            ++s;
            gram_entries(a, sh, (s - 1) * s / 2, s * (s + 1) / 2);  // the new row of G
            fl += f8n * (unsigned long long)s;
            if (!fresh) {
                // the entry's rank-one term: r += a z_new, c_t += G[t][new] z_new,
                // c_new = a^H r + ||a||^2 z_new, phi += 2 Re(conj(z_new) a^H r) + ||a||^2 |z_new|^2 + lambda |z_new|
                const int tn = s - 1;
                const double azn = sqrt(zn.x * zn.x + zn.y * zn.y);
                ph += 2.0 * (zn.x * gr + zn.y * gi) + cn * azn * azn + lam * azn;
                for (int nn = lane; nn < a.n; nn += 64) {
                    const double2 av = ASat(sh, nn, tn);
                    sh.r[nn] = make_double2(sh.r[nn].x + (av.x * zn.x - av.y * zn.y),
                                            sh.r[nn].y + (av.x * zn.y + av.y * zn.x));
                }
                if (lane < tn) {
                    const double2 g = gram_at(sh, lane, tn), cv = sh.c[lane];
                    sh.c[lane] = make_double2(cv.x + (g.x * zn.x - g.y * zn.y), cv.y + (g.x * zn.y + g.y * zn.x));
                } else if (lane == tn) {
                    sh.c[lane] = make_double2(gr + cn * zn.x, gi + cn * zn.y);
                }
                __syncthreads();
                fl += f8n + 8ull * (unsigned long long)s;
            }
            }
            if (entered == 0) {
                if (gcur > gstop) {
                    gcur = gstop;
                    continue;
                }
                break;
            }
        }
        // the 32-slot pass hands what it leaves above tol to the FP64 continuation
        if (kTier == 2 && a.overflow && kfin > (double)a.tol && lane == 0)
            a.overflow[atomicAdd(a.overflow_count, 1u)] = (int32_t)p;
        // write the best point (complex64) unless it is the starting one
        if (sh.sb >= 0) {
            const int sb = sh.sb;
            for (int t = lane; t < sb; t += 64) sh.sidx[sh.Sb[t]] = (int8_t)t;
            __syncthreads();
            for (int m = lane; m < a.l; m += 64) {
                const int t = sh.sidx[m];
                xo[m] = t >= 0 ? make_float2((float)sh.zb[t].x, (float)sh.zb[t].y) : make_float2(0.0f, 0.0f);
            }
            __syncthreads();
            for (int t = lane; t < sb; t += 64) sh.sidx[sh.Sb[t]] = -1;
        }
        if (lane == 0) a.status[p] |= L1LS_PX_POLISHED;
        __syncthreads();
    }
    if (lane == 0 && fl) atomicAdd(&a.work[2], fl);
    if (lane == 0 && fl32) atomicAdd(&a.work[3], fl32);
}

// The stacks of a table one after another: each workgroup takes listed pixels
// of a stack from that stack's counter, then moves on.  A workgroup beyond a
// stack's number of A^H b buffers skips that stack (the others cover it).
// The 8-slot pass is built for four waves a SIMD (128 VGPRs, some of the register
// solver's rows spill): it is latency bound, and the extra wave per SIMD more than
// pays for the spills (close pairs: 704 -> 642 ms); the larger passes keep three.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kMaxSupp == 8 ? 4 : 3)))
polish_kernel(const StackTable t)
{
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        const PolishArgsDev a = polish_args_for(t.d[i], t.o, kTier);
        if ((int)blockIdx.x >= a.max_groups) continue;
        polish_stack(a);
        __syncthreads();
    }
}

size_t polish_lds_bytes(int n, int l_pad)
{
    return (size_t)2 * n * sizeof(double2) + polish_as_bytes(n, l_pad) + (size_t)l_pad * sizeof(int8_t);
}

hipError_t launch_polish_table(const StackTable &t, hipStream_t s)
{
    size_t dyn = 0;
    int want = 0;
    for (int i = 0; i < t.count; ++i) {
        if (t.d[i].p <= 0) continue;
        dyn = dyn > polish_lds_bytes(t.d[i].n, lpad_for(t.d[i].l)) ? dyn : polish_lds_bytes(t.d[i].n, lpad_for(t.d[i].l));
        const int mg = (int)(t.d[i].p < kMaxRefineGroups ? t.d[i].p : kMaxRefineGroups);
        want = want > mg ? want : mg;
    }
    if (want == 0) return hipSuccess;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, polish_kernel, 64, dyn);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int g = per_cu > 0 ? per_cu * cus : cus * 4;
    if (g > want) g = want;  // one A^H b buffer per workgroup
    if (g < 1) g = 1;
    hipLaunchKernelGGL(polish_kernel, dim3(g), dim3(64), dyn, s, t);
    return hipGetLastError();
}

}  // namespace l1ls
