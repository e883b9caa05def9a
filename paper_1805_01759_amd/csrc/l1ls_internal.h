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
// The FP64 continuation of Algorithm 1 keeps a pixel's iterate in registers (up
// to 16 chunks of 64 bins) and its history in LDS; beyond kContMaxL bins its six
// L-vectors (x^k, x^{k-1}, G_k, G_{k-1}, x-bar, d) live in a workspace slot per
// workgroup (kContGroups of them at most).
constexpr int kContMaxL = 1024;
constexpr int kContGroups = 4096;
__host__ __device__ inline int64_t cont_groups_for(int64_t p) { return p < kContGroups ? p : kContGroups; }
__host__ __device__ inline size_t cont_slot_bytes(int l_pad) { return (size_t)6 * l_pad * 16; }
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
    const uint16_t *Abf;      // split-BF16 planes (re hi, im hi, re lo, im lo) of the packed A:
                              // [4][rows_pad][l_pad], then transposed [4][l_pad][rows_pad]
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
    float2 *fstate;           // streamed tile: iterate state, stream_tile_bytes(l_pad) per workgroup
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

// The refinement launches at most this many workgroups (16 per CU on 256 CUs,
// four single-wave workgroups a SIMD): each holds A^H b of its current pixel in
// the workspace.
constexpr int kMaxRefineGroups = 4096;

// Tiling helpers (host and device): KB MFMA row blocks of 16 unknowns per wave
// slice, W waves, l padded to 8 KB W, 2N real rows in 16-row blocks, N padded to 16.
__host__ __device__ inline int slice_blocks_for(int l) { return l <= 256 ? 8 : 16; }
__host__ __device__ inline int waves_for(int l)
{
    const int slice = 8 * slice_blocks_for(l);
    return (l + slice - 1) / slice;
}
__host__ __device__ inline int lpad_for(int l) { return waves_for(l) * 8 * slice_blocks_for(l); }
__host__ __device__ inline int zblocks_for(int n) { return (2 * n + 15) / 16; }
__host__ __device__ inline int rows_pad_for(int n) { return 16 * ((n + 15) / 16); }
__host__ __device__ inline size_t ws_align(size_t x) { return (x + 255) / 256 * 256; }

// The register-resident MFMA tile takes up to 64 rows and 512 bins; larger shapes
// run the streamed MFMA tile, whose iterate state (two x and three G arrays of 16
// pixels: l_pad x 640 bytes a tile) lives in a workspace region, one slot per
// persistent workgroup (at most kStreamGroups of them).
__host__ __device__ inline bool mfma_tile_shape(int n, int l) { return n <= 64 && l <= 512; }
constexpr int kStreamGroups = 512;
// The automatic choice: the streamed tile beyond the register tile, and also for
// 384 < L <= 512, where the two split the unknowns alike (bit-identical results,
// either precision) and the streamed tile, at two waves per SIMD, is the faster.
__host__ __device__ inline bool auto_stream(int n, int l, int /*precision*/)
{
    return !mfma_tile_shape(n, l) || l > 384;
}
__host__ __device__ inline int64_t stream_groups_for(int64_t p)
{
    const int64_t tiles = (p + 15) / 16;
    return tiles < kStreamGroups ? tiles : kStreamGroups;
}
__host__ __device__ inline size_t stream_tile_bytes(int l_pad) { return (size_t)l_pad * 640; }

// Workspace layout for one stack (byte offsets; every region 256-byte aligned).
struct StackWorkspace {
    size_t a_packed, a_trans, a_bf16, consts, queue, work, status, iters, kkt32, polish_list, gram, blocks, resid,
        overflow, hgram, cbuf, cstate, fstate, total;
};
__host__ __device__ inline StackWorkspace stack_workspace_layout(int n, int l, int64_t p)
{
    StackWorkspace w;
    const int l_pad = lpad_for(l);
    size_t off = 0;
    w.a_packed = off;
    off = ws_align(off + (size_t)rows_pad_for(n) * l_pad * sizeof(float2));
    w.a_trans = off;
    off = ws_align(off + (size_t)l_pad * n * sizeof(float2));
    w.a_bf16 = off;  // split-BF16 planes of the packed A, row-major and transposed
    off = ws_align(off + (size_t)2 * 4 * rows_pad_for(n) * l_pad * sizeof(uint16_t));
    w.gram = off;  // M = A A^H, then two N x N buffers for its repeated squares
    off = ws_align(off + (size_t)3 * n * n * sizeof(double2));
    w.consts = off;
    off = ws_align(off + sizeof(StackConsts));
    w.queue = off;
    off = ws_align(off + 16 * sizeof(uint32_t));
    w.work = off;
    off = ws_align(off + 4 * sizeof(unsigned long long));
    w.status = off;
    off = ws_align(off + (size_t)p * sizeof(uint32_t));
    w.iters = off;
    off = ws_align(off + (size_t)p * sizeof(int32_t));
    w.kkt32 = off;
    off = ws_align(off + (size_t)p * sizeof(float));
    w.polish_list = off;
    off = ws_align(off + (size_t)p * sizeof(int32_t));
    w.blocks = off;
    off = ws_align(off + (size_t)kMaxBlocks * sizeof(BlockConsts));
    w.resid = off;
    off = ws_align(off + (size_t)p * n * sizeof(float2));
    w.overflow = off;
    off = ws_align(off + (size_t)p * sizeof(int32_t));
    // the refinement's bin Gram A^H A and the A^H b of its workgroups' pixels
    w.hgram = off;
    off = ws_align(off + (size_t)l * l * sizeof(double2));
    w.cbuf = off;
    const int64_t groups = p < kMaxRefineGroups ? p : kMaxRefineGroups;
    off = ws_align(off + (size_t)groups * l * sizeof(double2));
    // the FP64 continuation's slots for stacks beyond kContMaxL bins
    w.cstate = off;
    if (l_pad > kContMaxL) off = ws_align(off + (size_t)cont_groups_for(p) * cont_slot_bytes(l_pad));
    // the streamed MFMA tile's iterate state comes last, where that kernel runs
    // the stack (stack_workspace_bytes)
    w.fstate = off;
    w.total = off;
    return w;
}

// Bytes of a stack's workspace, with or without the streamed tile's state.
__host__ __device__ inline size_t stack_workspace_bytes(int n, int l, int64_t p, bool stream)
{
    const StackWorkspace w = stack_workspace_layout(n, l, p);
    return stream ? ws_align(w.fstate + (size_t)stream_groups_for(p) * stream_tile_bytes(lpad_for(l))) : w.total;
}

// ---------------------------------------------------------------------------
// Stack tables.  Every kernel of a solve takes up to kMaxStacksPerLaunch stacks
// (a single solve is a table of one) and sweeps them in table order: persistent
// workgroups take pixels from a stack's own queue until it is empty, then move
// on to the next stack (restaging that stack's A), so a batch of stacks of one
// tile class is one launch.  The table travels as the kernel argument.
struct StackDesc {
    const float2 *A;          // caller's A (n x l, row-major)
    const float2 *B;          // p x n
    const float *lambda;
    float2 *X;                // p x l
    char *ws;                 // the stack's workspace (stack_workspace_layout)
    int32_t *iters;           // diagnostics (any may be null)
    float *kkt;
    float *objective;
    uint32_t *status;
    int32_t *nnz;
    int64_t p, lambda_stride;
    int32_t n, l;
    int32_t keep_residual;    // the stack's iteration kernel writes the residual of each retired pixel
    int32_t pad;
};
struct SolveOpts {
    int32_t fista_cap;        // retire unsolved pixels after this many iterations
    float tol, c_alpha;
    int32_t backtracking, monotone, polish, warm;
    int32_t max_iter;         // iterations of Algorithm 1 in all (the FP64 continuation's budget)
    int32_t cont;             // 1: FP64 continuation of the pixels the refinement leaves above tol
    int32_t pad[2];
};
constexpr int kMaxStacksPerLaunch = 32;
struct StackTable {
    int32_t count;
    SolveOpts o;
    StackDesc d[kMaxStacksPerLaunch];
};
static_assert(sizeof(StackTable) <= 4000, "a stack table travels as a kernel argument");

// Per-stack argument blocks of the kernels, from a table entry (host and device).
__host__ __device__ inline FistaArgs fista_args_for(const StackDesc &d, const SolveOpts &o)
{
    const StackWorkspace lay = stack_workspace_layout(d.n, d.l, d.p);
    FistaArgs fa;
    fa.n = d.n;
    fa.l = d.l;
    fa.l_pad = lpad_for(d.l);
    fa.waves = waves_for(d.l);
    fa.p = d.p;
    fa.A = (const float2 *)(d.ws + lay.a_packed);
    fa.At = (const float2 *)(d.ws + lay.a_trans);
    fa.Abf = (const uint16_t *)(d.ws + lay.a_bf16);
    fa.B = d.B;
    fa.lambda = d.lambda;
    fa.lambda_stride = d.lambda_stride;
    fa.X = d.X;
    fa.iters = (int32_t *)(d.ws + lay.iters);
    fa.kkt32 = (float *)(d.ws + lay.kkt32);
    fa.status = (uint32_t *)(d.ws + lay.status);
    fa.consts = (const StackConsts *)(d.ws + lay.consts);
    fa.queue = (uint32_t *)(d.ws + lay.queue);
    fa.polish_count = fa.queue + 1;
    fa.polish_list = (int32_t *)(d.ws + lay.polish_list);
    fa.work = (unsigned long long *)(d.ws + lay.work);
    fa.R = d.keep_residual ? (float2 *)(d.ws + lay.resid) : nullptr;
    fa.fstate = (float2 *)(d.ws + lay.fstate);
    fa.fista_cap = o.fista_cap;
    fa.tol = o.tol;
    fa.c_alpha = o.c_alpha;
    fa.backtracking = o.backtracking;
    fa.monotone = o.monotone;
    fa.polish = o.polish;
    fa.warm = o.warm;
    return fa;
}

// The refinement runs in three passes of growing working sets (tier 0: 8 slots,
// 1: 16, 2: 32); each takes the pixels the previous one listed because its working
// set filled above tol.  The lists alternate between two regions: tier 0 reads
// the refinement list and writes the overflow region, tier 1 reads that and
// writes the (by then finished) refinement list, tier 2 reads it.
__host__ __device__ inline PolishArgsDev polish_args_for(const StackDesc &d, const SolveOpts &o, int tier)
{
    const StackWorkspace lay = stack_workspace_layout(d.n, d.l, d.p);
    uint32_t *queue = (uint32_t *)(d.ws + lay.queue);
    int32_t *plist = (int32_t *)(d.ws + lay.polish_list), *oflow = (int32_t *)(d.ws + lay.overflow);
    PolishArgsDev pa;
    pa.n = d.n;
    pa.l = d.l;
    pa.l_pad = lpad_for(d.l);
    pa.A = (const float2 *)(d.ws + lay.a_packed);
    pa.B = d.B;
    pa.lambda = d.lambda;
    pa.lambda_stride = d.lambda_stride;
    pa.X = d.X;
    pa.consts = (const StackConsts *)(d.ws + lay.consts);
    pa.count = queue + 1 + 2 * tier;  // counts in queue[1], [3], [5]; next pixel in [2], [4], [6]
                                      // (the FP64 continuation: [7], [8])
    pa.next = queue + 2 + 2 * tier;
    pa.list = tier == 1 ? oflow : plist;
    pa.R = (tier == 0 && d.keep_residual) ? (const float2 *)(d.ws + lay.resid) : nullptr;
    // tier 2 lists the pixels it leaves above tol for the FP64 continuation
    // (queue[7]), when that runs
    const bool cont = o.cont != 0;
    pa.overflow = tier == 0 ? oflow : (tier == 1 ? plist : (cont ? oflow : nullptr));
    pa.overflow_count = tier < 2 || cont ? queue + 3 + 2 * tier : nullptr;
    pa.status = (uint32_t *)(d.ws + lay.status);
    pa.work = (unsigned long long *)(d.ws + lay.work);
    pa.H = (const double2 *)(d.ws + lay.hgram);
    pa.cbuf = (double2 *)(d.ws + lay.cbuf);
    pa.rounds = 64;
    pa.mode = o.polish;
    pa.tol = o.tol;
    pa.max_groups = (int)(d.p < kMaxRefineGroups ? d.p : kMaxRefineGroups);
    return pa;
}

__host__ __device__ inline CertifyArgs certify_args_for(const StackDesc &d, const SolveOpts &o)
{
    const StackWorkspace lay = stack_workspace_layout(d.n, d.l, d.p);
    CertifyArgs ca;
    ca.n = d.n;
    ca.l = d.l;
    ca.l_pad = lpad_for(d.l);
    ca.p = d.p;
    ca.A = (const float2 *)(d.ws + lay.a_packed);
    ca.B = d.B;
    ca.lambda = d.lambda;
    ca.lambda_stride = d.lambda_stride;
    ca.X = d.X;
    ca.iters_in = (const int32_t *)(d.ws + lay.iters);
    ca.status_in = (const uint32_t *)(d.ws + lay.status);
    ca.consts = (const StackConsts *)(d.ws + lay.consts);
    ca.tol = o.tol;
    ca.polish = o.polish;
    ca.iters = d.iters;
    ca.kkt = d.kkt;
    ca.objective = d.objective;
    ca.status = d.status;
    ca.nnz = d.nnz;
    return ca;
}

// Launches over a stack table (every entry with p > 0).
hipError_t launch_setup_table(const StackTable &t, bool bin_gram, hipStream_t s);
hipError_t launch_certify_table(const StackTable &t, hipStream_t s);
hipError_t launch_polish_table(const StackTable &t, hipStream_t s);       // 8 slots
hipError_t launch_polish_mid_table(const StackTable &t, hipStream_t s);   // 16 slots
hipError_t launch_polish_wide_table(const StackTable &t, hipStream_t s);  // 32 slots
hipError_t launch_continue_table(const StackTable &t, hipStream_t s);     // FP64 Algorithm 1

// The iteration kernel that runs a stack: the split re/im MFMA tile (T row
// blocks, KB unknown blocks per wave, A staged in LDS or read from L2, up to
// WMAX waves of which `waves` run), the streamed MFMA tile (T row blocks, four
// waves, iterate state in the workspace), or the wave-per-pixel kernel (NC chunks).
struct IterVariant {
    int family;   // kVarMfma, kVarStream, kVarWave
    int T, KB, alds, prec, wmax, waves, nc;
    bool operator==(const IterVariant &o) const
    {
        return family == o.family && T == o.T && KB == o.KB && alds == o.alds && prec == o.prec &&
               wmax == o.wmax && waves == o.waves && nc == o.nc;
    }
};
enum { kVarMfma = 1, kVarWave = 2, kVarStream = 3 };
// The default variant for a shape and precision (kMfma: the MFMA families, kWave:
// the wave kernel); `alt` selects an alternative tiling for the autotuner
// (0 default, 1 the other A placement, 2 the other unknowns-per-wave split);
// returns false when the alternative does not exist.
bool iter_variant(int n, int l, int precision, int choice, int alt, IterVariant *v);
// LDS bytes of a variant for one stack, and the launch over a table whose
// stacks all run that variant.
size_t iter_variant_lds(const IterVariant &v, int n, int l);
hipError_t launch_iteration_table(const StackTable &t, const IterVariant &v, hipStream_t s);



hipError_t launch_setup_blocks(int n, int l, int J, const float2 *A, BlockConsts *bc, hipStream_t s);
hipError_t launch_fista_blocks(const BlocksArgs &ba, hipStream_t s);
size_t fista_blocks_lds(int n, int l_pad, int J);
size_t fista_wave_lds(int n, int l);

// Which iteration kernel runs a stack.
enum KernelChoice { kAuto = 0, kMfma = 1, kWave = 2, kBlocks = 3, kStream = 4 };
bool mfma_supports(int n, int l);
l1ls_status solve_stack(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B,
                        const float *lambda, int64_t lambda_stride, const l1ls_options *opt,
                        l1ls_c32 *X, const l1ls_diag *diag, void *ws, size_t ws_bytes,
                        hipStream_t s, int choice, int blocks = 0,
                        const double *draws = nullptr, int alt = 0);
l1ls_status check_options(const l1ls_options *o);
l1ls_status check_stack(int32_t n, int32_t l, int64_t p, const void *A, const void *B, const float *lambda,
                        int64_t lambda_stride, const void *X, const void *ws, size_t ws_bytes, bool stream);
// Whether the options' iteration kernel for this shape is the streamed tile (its
// state then needs workspace), and the kernel choice the options ask for.
bool needs_stream_state(int n, int l, const l1ls_options *opt);
int options_choice(const l1ls_options *opt);
l1ls_status stack_variant(int32_t n, int32_t l, const l1ls_options *opt, int choice, int alt, IterVariant *v);
StackDesc stack_desc(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B, const float *lambda,
                     int64_t lambda_stride, l1ls_c32 *X, const l1ls_diag *diag, void *ws, const IterVariant &v);
l1ls_status run_stacks(const StackDesc *d, const IterVariant *var, int count, const l1ls_options *opt,
                       hipStream_t s);
l1ls_status set_error(l1ls_status st, const char *fmt, ...);
size_t unrolled_tape_bytes(int n, int l, int64_t p, int K, int ckpt);
size_t unrolled_bwd_ws_bytes(int n, int l, int64_t p, int K, int ckpt);
hipError_t launch_unrolled_forward(int n, int l, int64_t p, const float *xi, const float *s,
                                   const float2 *B, float lambda, float alpha, int K, int ckpt,
                                   float2 *X, void *tape, hipStream_t st);
hipError_t launch_unrolled_backward(int n, int l, int64_t p, const float2 *B, float lambda,
                                    float alpha, int K, int ckpt, const void *tape,
                                    const float2 *dX, float2 *dB, float *dlambda, float *dxi,
                                    void *ws, hipStream_t st);
size_t fista_mfma_lds_bytes(int n, int l_pad, int waves, bool a_lds, int precision);
size_t fista_stream_lds_bytes(int T);
hipError_t launch_stream_table(const StackTable &t, int T, int precision, hipStream_t s);

}  // namespace l1ls
