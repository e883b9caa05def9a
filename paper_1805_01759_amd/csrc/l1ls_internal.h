// Internal declarations shared by the C-ABI layer and the HIP kernels of the
// gfx950 solver.  Not part of the public interface (include/l1ls.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/l1ls.h"

namespace l1ls {

// A wave owns 8 KB complex unknowns of every pixel in its tile (KB MFMA row
// blocks of 16 real rows, KB = 8 for L <= 256, 16 for L <= 512); a workgroup
// of W <= 4 waves (one per SIMD) covers L <= 8 KB W.
constexpr int kTile = 16;        // pixels per workgroup (MFMA N dimension)
constexpr int kMaxWavesIter = 4;
constexpr int kMaxWaves = 16;    // staging bound: L <= 1024
constexpr int kMaxN = 128;
constexpr int kMaxZB = 16;       // ceil(2 N / 16) <= 16

// Device-side per-stack constants written by the setup kernel.
struct StackConsts {
    double lf;       // 2 lambda_max(A A^H)
    double alpha0;   // 1 / (2 max_l ||a_l||^2)
    double lmax_it;  // power iterations used (diagnostic)
    double pad;
};

struct FistaArgs {
    int n, l, l_pad, waves;
    int64_t p;
    const float2 *A;          // packed: rows_pad_for(n) x l_pad, zero padded rows and columns
    const float2 *At;         // transposed: l_pad x n (At[m n + i] = A[i][m])
    const float2 *B;          // p x n
    const float *lambda;
    int64_t lambda_stride;
    float2 *X;                // p x l
    int32_t *iters;
    float *kkt32;             // FP32 KKT at exit of the iteration (workspace)
    uint32_t *status;         // workspace status (always present)
    const StackConsts *consts;
    uint32_t *queue;          // [0] next pixel
    uint32_t *polish_count;   // number of pixels appended to polish_list
    unsigned long long *work; // [0] pixel forward products, [1] pixel adjoint products,
                              // [2] refinement FP64 flops, [3] refinement FP32 flops
    int32_t *polish_list;
    float2 *R;                // p x n: residual A x - b of the returned x (FP32), or null
    int32_t fista_cap;        // retire unsolved pixels after this many iterations
    float tol, c_alpha;
    int32_t backtracking, monotone, polish;
    int32_t warm;             // 1: X holds each pixel's initial point x^(0) on entry
};

// Per-block constants of the block-coordinate form (J <= kMaxBlocks).
constexpr int kMaxBlocks = 64;
struct BlockConsts {
    double L;       // 2 lambda_max(A_i A_i^H)
    double alpha0;  // 1 / (2 max_{l in i} ||a_l||^2)
    double afloor;  // 1 / L
    double pad;
};

struct BlocksArgs {
    FistaArgs f;           // work[0] accumulates the iteration's FP32 flops
    int J;
    const double *u;       // draws in [0, 1), one per iteration
    const BlockConsts *bc;
};

struct CertifyArgs {
    int n, l, l_pad;
    int64_t p;
    const float2 *A;          // packed n x l_pad
    const float2 *B;
    const float *lambda;
    int64_t lambda_stride;
    float2 *X;
    const int32_t *iters_in;
    const uint32_t *status_in;
    const StackConsts *consts;
    float tol;
    int32_t polish;           // 1: refine pixels above tol
    // outputs (any may be null)
    int32_t *iters;
    float *kkt;
    float *objective;
    uint32_t *status;
    int32_t *nnz;
};

struct PolishArgsDev {
    int n, l, l_pad;
    const float2 *A;          // packed n x l_pad
    const float2 *B;
    const float *lambda;
    int64_t lambda_stride;
    float2 *X;
    const StackConsts *consts;
    const uint32_t *count;    // number of listed pixels
    uint32_t *next;           // next list entry to take (zero before the launch)
    const int32_t *list;      // pixel indices
    const float2 *R;          // p x n residual the iteration kept (FP32), or null
    int32_t *overflow;        // pixels left unsolved on a full working set (or null)
    uint32_t *overflow_count;
    uint32_t *status;         // workspace status: POLISHED is or-ed in
    unsigned long long *work; // [2] accumulates the refinement's FP64 flops, [3] its FP32 flops
    const double2 *H;         // l x l bin Gram A^H A (FP64), H[s l + m] = a_s^H a_m
    double2 *cbuf;            // kMaxRefineGroups x l: A^H b of each workgroup's pixel (FP64)
    int32_t rounds;
    int32_t mode;             // 1: refine pixels whose FP64 KKT > tol; 2: refine all
    float tol;
    int32_t max_groups;       // workgroups the launch may use (<= kMaxRefineGroups)
};

// The refinement launches at most this many workgroups (12 per CU on 256 CUs):
// each holds A^H b of its current pixel in the workspace.
constexpr int kMaxRefineGroups = 3072;

// Workspace layout for one stack.
struct StackWorkspace {
    size_t a_packed, a_trans, consts, queue, work, status, iters, kkt32, polish_list, gram, blocks, resid,
        overflow, hgram, cbuf, total;
};
StackWorkspace stack_workspace_layout(int n, int l, int64_t p);

int slice_blocks_for(int l);   // KB
int waves_for(int l);          // W
int lpad_for(int l);           // 8 KB W
int zblocks_for(int n);
int rows_pad_for(int n);       // rows of the packed A: N rounded up to 16

hipError_t launch_setup(int n, int l, int l_pad, const float2 *A, float2 *Ap, float2 *At, double2 *gram,
                        StackConsts *consts, uint32_t *queue, unsigned long long *work,
                        hipStream_t s);
hipError_t launch_setup_bin_gram(int n, int l, const float2 *A, double2 *H, hipStream_t s);
hipError_t launch_fista(const FistaArgs &a, int precision, int max_groups, hipStream_t s,
                        bool *keeps_residual = nullptr);
hipError_t launch_fista_wave(const FistaArgs &a, hipStream_t s);
bool fista_split_kernel(const FistaArgs &a, int precision);
hipError_t launch_setup_blocks(int n, int l, int J, const float2 *A, BlockConsts *bc, hipStream_t s);
hipError_t launch_fista_blocks(const BlocksArgs &ba, hipStream_t s);
size_t fista_blocks_lds(int n, int l_pad, int J);
size_t fista_wave_lds(int n, int l);

// Which iteration kernel runs a stack.
enum KernelChoice { kAuto = 0, kMfma = 1, kWave = 2, kBlocks = 3 };
bool mfma_supports(int n, int l);
l1ls_status solve_stack(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B,
                        const float *lambda, int64_t lambda_stride, const l1ls_options *opt,
                        l1ls_c32 *X, const l1ls_diag *diag, void *ws, size_t ws_bytes,
                        hipStream_t s, int choice, int blocks = 0,
                        const double *draws = nullptr);
l1ls_status set_error(l1ls_status st, const char *fmt, ...);
hipError_t launch_certify(const CertifyArgs &a, hipStream_t s);
hipError_t launch_polish(const PolishArgsDev &a, int groups, hipStream_t s);       // 16 slots
hipError_t launch_polish_wide(const PolishArgsDev &a, int groups, hipStream_t s);  // 32 slots
size_t unrolled_tape_bytes(int n, int l, int64_t p, int K, int ckpt);
size_t unrolled_bwd_ws_bytes(int n, int l, int64_t p, int K, int ckpt);
hipError_t launch_unrolled_forward(int n, int l, int64_t p, const float *xi, const float *s,
                                   const float2 *B, float lambda, float alpha, int K, int ckpt,
                                   float2 *X, void *tape, hipStream_t st);
hipError_t launch_unrolled_backward(int n, int l, int64_t p, const float2 *B, float lambda,
                                    float alpha, int K, int ckpt, const void *tape,
                                    const float2 *dX, float2 *dB, float *dlambda, float *dxi,
                                    void *ws, hipStream_t st);
size_t fista_lds_bytes(int n, int l_pad, int waves, int zb, bool a_lds);
size_t fista_mfma_lds_bytes(int n, int l_pad, int waves, bool a_lds, int precision);
bool fista_a_fits_lds(int n, int l_pad, int waves, int zb);

}  // namespace l1ls
