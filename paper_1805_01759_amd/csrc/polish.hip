// FP64 refinement of the FP32 iterate (complex L1LS of arXiv 1805.01759,
// Eq. (1)); not part of the paper's method, it turns "KKT <= tol" into the
// minimiser to FP64 accuracy and catches pixels the FP32 iteration left.
//
// Per pixel (one 64-lane workgroup), starting from the working set S of the
// local maxima of |x| of the FP32 iterate, repeat
//   * damped Newton on phi(z) = ||A_S z - b||^2 + lambda sum |z_s| over the
//     working set (|S| <= kMaxSupp), with the real Hessian
//       2 [[Re G, -Im G], [Im G, Re G]] + lambda blkdiag((I - u u^T)/|z_s|),
//     G = A_S^H A_S, u = (Re z_s, Im z_s)/|z_s|; the coordinate whose Newton step
//     turns it round most leaves the working set; Armijo backtracking on phi;
//   * full FP64 gradient: natural KKT residual, and the worst off-set
//     violator of |g_l| <= lambda enters at its exact coordinate minimiser,
// until the KKT residual is at the target or no violator is left.  The point
// with the least objective is kept and written back (complex64).
//
// The working set's columns A_S are staged in LDS, so phi, its gradient and the
// Hessian read LDS only; the full-gradient pass reads A coalesced.
#include "l1ls_internal.h"

namespace l1ls {

constexpr int kMaxSupp = 16;          // Newton on at most 16 complex unknowns
constexpr int kMaxM = 2 * kMaxSupp;   // real Hessian order

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wmax(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

struct PolishShared {
    double2 *x;       // l_pad entries (dynamic LDS): dense iterate
    float2 *best;     // l_pad entries (dynamic LDS): best point, in output precision
    float2 *AS;       // n x kMaxSupp (dynamic LDS): columns of the working set
    double2 r[kMaxN];
    double2 z[kMaxSupp], zt[kMaxSupp];
    int S[kMaxSupp];
    double H[kMaxM * kMaxM];
    double rhs[kMaxM], grd[kMaxM], hdiag[kMaxM];
    int cnt;
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

// column t of the working set <- column m of A
__device__ void stage_col(const PolishArgsDev &a, PolishShared &sh, int t, int m)
{
    for (int nn = threadIdx.x; nn < a.n; nn += 64) sh.AS[nn * kMaxSupp + t] = a.A[(size_t)nn * a.l_pad + m];
}

// r = A x - b over the dense x in LDS (zero entries skipped, uniform branch)
__device__ void residual_dense(const PolishArgsDev &a, PolishShared &sh, const float2 *b)
{
    const int lane = threadIdx.x;
    for (int nn = lane; nn < a.n; nn += 64) {
        double rr = 0.0, ri = 0.0;
        for (int m = 0; m < a.l; ++m) {
            const double2 xv = sh.x[m];
            if (xv.x != 0.0 || xv.y != 0.0) {
                const double2 av = Aat(a, nn, m);
                rr += av.x * xv.x - av.y * xv.y;
                ri += av.x * xv.y + av.y * xv.x;
            }
        }
        sh.r[nn] = make_double2(rr - b[nn].x, ri - b[nn].y);
    }
    __syncthreads();
}

// phi(z) on the working set, r <- A_S z - b; returns phi (all lanes)
__device__ double phi_support(const PolishArgsDev &a, PolishShared &sh, const float2 *b,
                              const double2 *z, int s, double lam)
{
    const int lane = threadIdx.x;
    double acc = 0.0;
    for (int nn = lane; nn < a.n; nn += 64) {
        double rr = -(double)b[nn].x, ri = -(double)b[nn].y;
        for (int t = 0; t < s; ++t) {
            const double2 av = ASat(sh, nn, t);
            const double2 zv = z[t];
            rr += av.x * zv.x - av.y * zv.y;
            ri += av.x * zv.y + av.y * zv.x;
        }
        sh.r[nn] = make_double2(rr, ri);
        acc += rr * rr + ri * ri;
    }
    double l1 = 0.0;
    for (int t = lane; t < s; t += 64) l1 += sqrt(z[t].x * z[t].x + z[t].y * z[t].y);
    const double out = wsum(acc) + lam * wsum(l1);
    __syncthreads();
    return out;
}

// Full FP64 pass at the dense x (with sh.r its residual): natural KKT residual,
// objective, and the worst off-support violator of |g| <= lambda.
__device__ void full_pass(const PolishArgsDev &a, PolishShared &sh, double lam, double lf,
                          double &F, double &kk, int &vidx)
{
    const int lane = threadIdx.x;
    double acc = 0.0, l1 = 0.0, km = 0.0, vbest = 0.0;
    vidx = -1;
    for (int nn = lane; nn < a.n; nn += 64) acc += sh.r[nn].x * sh.r[nn].x + sh.r[nn].y * sh.r[nn].y;
    for (int m = lane; m < a.l; m += 64) {
        const double xr = sh.x[m].x, xi = sh.x[m].y;
        l1 += sqrt(xr * xr + xi * xi);
        double gr = 0.0, gi = 0.0;
        for (int nn = 0; nn < a.n; ++nn) {
            const double2 av = Aat(a, nn, m), rv = sh.r[nn];
            gr += av.x * rv.x + av.y * rv.y;
            gi += av.x * rv.y - av.y * rv.x;
        }
        gr *= 2.0;
        gi *= 2.0;
        const double vr = xr - gr / lf, vi = xi - gi / lf;
        const double mag = sqrt(vr * vr + vi * vi), tau = lam / lf;
        const double sc = mag > tau ? 1.0 - tau / mag : 0.0;
        const double er = xr - vr * sc, ei = xi - vi * sc;
        km = fmax(km, sqrt(er * er + ei * ei));
        const double gm = sqrt(gr * gr + gi * gi);
        if (xr == 0.0 && xi == 0.0 && gm > lam * (1.0 + 1e-12) && gm > vbest) {
            vbest = gm;
            vidx = m;
        }
    }
    F = wsum(acc) + lam * wsum(l1);
    kk = wmax(km) * lf / lam;
    for (int o = 32; o > 0; o >>= 1) {  // wave argmax of the violation (ties: lowest index)
        const double ov = __shfl_xor(vbest, o, 64);
        const int oi = __shfl_xor(vidx, o, 64);
        if (ov > vbest || (ov == vbest && oi >= 0 && (vidx < 0 || oi < vidx))) {
            vbest = ov;
            vidx = oi;
        }
    }
}

__global__ void __launch_bounds__(64) polish_kernel(const PolishArgsDev a)
{
    __shared__ PolishShared sh;
    extern __shared__ __align__(16) unsigned char dyn[];
    const int lane = threadIdx.x;
    if (lane == 0) {
        sh.x = reinterpret_cast<double2 *>(dyn);
        sh.best = reinterpret_cast<float2 *>(dyn + (size_t)a.l_pad * sizeof(double2));
        sh.AS = reinterpret_cast<float2 *>(dyn + (size_t)a.l_pad * (sizeof(double2) + sizeof(float2)));
    }
    __syncthreads();
    const double lf = a.consts->lf;
    const uint32_t count = *a.count;
    for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
        const int64_t p = a.list[item];
        const float lam_f = a.lambda[p * a.lambda_stride];
        if (!(lam_f > 0.0f) || !isfinite(lam_f)) continue;
        const double lam = lam_f;
        const float2 *b = a.B + (size_t)p * a.n;
        float2 *xo = a.X + (size_t)p * a.l;
        for (int m = lane; m < a.l_pad; m += 64) {
            const float2 v = m < a.l ? xo[m] : make_float2(0.0f, 0.0f);
            sh.x[m] = make_double2(v.x, v.y);
            sh.best[m] = v;
        }
        __syncthreads();
        // objective and FP64 natural KKT residual of the starting point
        residual_dense(a, sh, b);
        double fbest, kk0;
        int vdummy;
        full_pass(a, sh, lam, lf, fbest, kk0, vdummy);
        __syncthreads();
        if (a.mode == 1 && kk0 <= (double)a.tol) continue;  // already solved
        // -- working set: the local maxima of |x| (FISTA spreads one scatterer
        //    over neighbouring bins); at most kMaxSupp, the largest kept
        if (lane == 0) sh.cnt = 0;
        __syncthreads();
        for (int m0 = 0; m0 < a.l; m0 += 64) {
            const int m = m0 + lane;
            bool pk = false;
            if (m < a.l) {
                const double2 xv = sh.x[m];
                const double mag = xv.x * xv.x + xv.y * xv.y;
                const double ml = m > 0 ? sh.x[m - 1].x * sh.x[m - 1].x + sh.x[m - 1].y * sh.x[m - 1].y : 0.0;
                const double mr = m + 1 < a.l ? sh.x[m + 1].x * sh.x[m + 1].x + sh.x[m + 1].y * sh.x[m + 1].y : 0.0;
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
                    const double2 xv = sh.x[mm];
                    const double mag = xv.x * xv.x + xv.y * xv.y;
                    const int s = sh.cnt;
                    if (s < kMaxSupp) {
                        sh.S[s] = mm;
                        sh.z[s] = xv;
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
                            sh.z[wi] = xv;
                        }
                    }
                }
            }
            __syncthreads();
        }
        int s = sh.cnt;
        for (int t = 0; t < s; ++t) stage_col(a, sh, t, sh.S[t]);
        __syncthreads();
        for (int round = 0; round < a.rounds; ++round) {
            for (int it = 0; it < 50 && s > 0; ++it) {
                const int m2 = 2 * s;
                const double ph = phi_support(a, sh, b, sh.z, s, lam);
                // gradient of phi on the working set (real pairs)
                double gmax = 0.0;
                for (int t = lane; t < s; t += 64) {
                    double gr = 0.0, gi = 0.0;
                    for (int nn = 0; nn < a.n; ++nn) {
                        const double2 av = ASat(sh, nn, t), rv = sh.r[nn];
                        gr += av.x * rv.x + av.y * rv.y;
                        gi += av.x * rv.y - av.y * rv.x;
                    }
                    const double2 zv = sh.z[t];
                    const double az = sqrt(zv.x * zv.x + zv.y * zv.y);
                    gr = 2.0 * gr + lam * zv.x / az;
                    gi = 2.0 * gi + lam * zv.y / az;
                    sh.grd[t] = gr;
                    sh.grd[t + s] = gi;
                    gmax = fmax(gmax, sqrt(gr * gr + gi * gi));
                }
                gmax = wmax(gmax);
                __syncthreads();
                if (gmax <= 1e-13 * lam) break;
                // Hessian: 2 realify(A_S^H A_S) + lambda (I - u u^T)/|z|
                for (int e = lane; e < s * s; e += 64) {
                    const int t = e / s, u = e % s;
                    double gr = 0.0, gi = 0.0;
                    for (int nn = 0; nn < a.n; ++nn) {
                        const double2 p1 = ASat(sh, nn, t), p2 = ASat(sh, nn, u);
                        gr += p1.x * p2.x + p1.y * p2.y;  // conj(p1) p2
                        gi += p1.x * p2.y - p1.y * p2.x;
                    }
                    sh.H[t * m2 + u] = 2.0 * gr;
                    sh.H[(t + s) * m2 + (u + s)] = 2.0 * gr;
                    sh.H[t * m2 + (u + s)] = -2.0 * gi;
                    sh.H[(t + s) * m2 + u] = 2.0 * gi;
                }
                __syncthreads();
                for (int t = lane; t < s; t += 64) {
                    const double2 zv = sh.z[t];
                    const double az = sqrt(zv.x * zv.x + zv.y * zv.y);
                    const double ur = zv.x / az, ui = zv.y / az;
                    sh.H[t * m2 + t] += lam * (1.0 - ur * ur) / az;
                    sh.H[(t + s) * m2 + (t + s)] += lam * (1.0 - ui * ui) / az;
                    sh.H[t * m2 + (t + s)] -= lam * ur * ui / az;
                    sh.H[(t + s) * m2 + t] -= lam * ur * ui / az;
                }
                __syncthreads();
                for (int i = lane; i < m2; i += 64) sh.hdiag[i] = sh.H[i * m2 + i];
                __syncthreads();
                // Cholesky (lower, in place, upper triangle kept); shifted retry if not PD
                double mu = 0.0;
                bool ok = false;
                for (int attempt = 0; attempt < 8 && !ok; ++attempt) {
                    if (attempt > 0) {
                        for (int e = lane; e < m2 * m2; e += 64) {
                            const int i = e / m2, k = e % m2;
                            if (k < i) sh.H[i * m2 + k] = sh.H[k * m2 + i];
                            if (k == i) sh.H[i * m2 + i] = sh.hdiag[i] + mu;
                        }
                        __syncthreads();
                    }
                    bool good = true;
                    for (int jj = 0; jj < m2; ++jj) {
                        double djj = sh.H[jj * m2 + jj];
                        for (int k = 0; k < jj; ++k) djj -= sh.H[jj * m2 + k] * sh.H[jj * m2 + k];
                        if (!(djj > 0.0)) { good = false; break; }
                        djj = sqrt(djj);
                        for (int i = jj + 1 + lane; i < m2; i += 64) {
                            double t = sh.H[i * m2 + jj];
                            for (int k = 0; k < jj; ++k) t -= sh.H[i * m2 + k] * sh.H[jj * m2 + k];
                            sh.H[i * m2 + jj] = t / djj;
                        }
                        __syncthreads();
                        if (lane == 0) sh.H[jj * m2 + jj] = djj;
                        __syncthreads();
                    }
                    ok = good;
                    mu = mu == 0.0 ? 1e-14 * lf : mu * 100.0;
                    __syncthreads();
                }
                if (!ok) break;
                // solve L L^T d = -g (lane 0, order <= 32); find the coordinate the
                // step turns round most
                if (lane == 0) {
                    for (int i = 0; i < m2; ++i) {
                        double t = -sh.grd[i];
                        for (int k = 0; k < i; ++k) t -= sh.H[i * m2 + k] * sh.rhs[k];
                        sh.rhs[i] = t / sh.H[i * m2 + i];
                    }
                    for (int i = m2 - 1; i >= 0; --i) {
                        double t = sh.rhs[i];
                        for (int k = i + 1; k < m2; ++k) t -= sh.H[k * m2 + i] * sh.rhs[k];
                        sh.rhs[i] = t / sh.H[i * m2 + i];
                    }
                    int drop = -1;
                    double worst = 0.0;
                    for (int t = 0; t < s; ++t) {
                        const double2 zv = sh.z[t];
                        const double nr = zv.x + sh.rhs[t], ni = zv.y + sh.rhs[t + s];
                        const double c = (zv.x * nr + zv.y * ni) / (zv.x * zv.x + zv.y * zv.y);
                        if (c <= 0.0 && (drop < 0 || c < worst)) { drop = t; worst = c; }
                    }
                    sh.cnt = drop;
                }
                __syncthreads();
                const int drop = sh.cnt;
                if (drop >= 0) {
                    // remove column `drop` from the working set (lanes over rows of A_S)
                    for (int nn = lane; nn < a.n; nn += 64)
                        for (int t = drop; t + 1 < s; ++t) sh.AS[nn * kMaxSupp + t] = sh.AS[nn * kMaxSupp + t + 1];
                    if (lane == 0) {
                        for (int t = drop; t + 1 < s; ++t) {
                            sh.S[t] = sh.S[t + 1];
                            sh.z[t] = sh.z[t + 1];
                        }
                    }
                    __syncthreads();
                    --s;
                    continue;
                }
                // Armijo backtracking on phi
                double slope = 0.0;
                for (int t = lane; t < m2; t += 64) slope += sh.grd[t] * sh.rhs[t];
                slope = wsum(slope);
                double step = 1.0;
                bool acc = false;
                for (int ls = 0; ls < 40; ++ls) {
                    for (int t = lane; t < s; t += 64)
                        sh.zt[t] = make_double2(sh.z[t].x + step * sh.rhs[t], sh.z[t].y + step * sh.rhs[t + s]);
                    __syncthreads();
                    const double pn = phi_support(a, sh, b, sh.zt, s, lam);
                    if (pn <= ph + 1e-4 * step * slope) { acc = true; break; }
                    step *= 0.5;
                }
                if (!acc) break;
                for (int t = lane; t < s; t += 64) sh.z[t] = sh.zt[t];
                __syncthreads();
            }
            // scatter the working set into the dense x; residual from the working set
            for (int m = lane; m < a.l_pad; m += 64) sh.x[m] = make_double2(0.0, 0.0);
            __syncthreads();
            for (int t = lane; t < s; t += 64) sh.x[sh.S[t]] = sh.z[t];
            __syncthreads();
            phi_support(a, sh, b, sh.z, s, lam);
            double F, kk;
            int vidx;
            full_pass(a, sh, lam, lf, F, kk, vidx);
            if (F <= fbest) {
                fbest = F;
                for (int m = lane; m < a.l_pad; m += 64)
                    sh.best[m] = make_float2((float)sh.x[m].x, (float)sh.x[m].y);
            }
            __syncthreads();
            if (kk <= (a.mode == 2 ? 1e-10 : 1e-2 * (double)a.tol)) break;
            if (vidx < 0 || s >= kMaxSupp) break;
            // the worst violator enters at its exact coordinate minimiser
            stage_col(a, sh, s, vidx);
            if (lane == 0) {
                double gr = 0.0, gi = 0.0, cn = 0.0;
                for (int nn = 0; nn < a.n; ++nn) {
                    const double2 av = Aat(a, nn, vidx), rv = sh.r[nn];
                    gr += av.x * rv.x + av.y * rv.y;
                    gi += av.x * rv.y - av.y * rv.x;
                    cn += av.x * av.x + av.y * av.y;
                }
                // argmin_z |a z + r|^2 + lambda |z| = -S_{lambda/2}(a^H r) / ||a||^2
                const double mag = sqrt(gr * gr + gi * gi), tau = 0.5 * lam;
                const double sc = mag > tau ? (1.0 - tau / mag) / cn : 0.0;
                sh.S[s] = vidx;
                sh.z[s] = make_double2(-gr * sc, -gi * sc);
            }
            __syncthreads();
            if (sh.z[s].x == 0.0 && sh.z[s].y == 0.0) break;
            ++s;
        }
        for (int m = lane; m < a.l; m += 64) xo[m] = sh.best[m];
        if (lane == 0) a.status[p] |= L1LS_PX_POLISHED;
        __syncthreads();
    }
}

hipError_t launch_polish(const PolishArgsDev &a, int groups, hipStream_t s)
{
    const size_t dyn = (size_t)a.l_pad * (sizeof(double2) + sizeof(float2)) +
                       (size_t)a.n * kMaxSupp * sizeof(float2);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, polish_kernel, 64, dyn);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int g = per_cu > 0 ? per_cu * cus : groups;
    hipLaunchKernelGGL(polish_kernel, dim3(g), dim3(64), dyn, s, a);
    return hipGetLastError();
}

}  // namespace l1ls
