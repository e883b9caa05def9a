// C ABI of the gfx950 L1LS solver: argument validation, workspace layout and
// the launch sequence (setup -> persistent iteration -> FP64 refinement ->
// FP64 optimality check).  All work is queued on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "l1ls_internal.h"

namespace l1ls {

static thread_local char g_err[512];

static l1ls_status fail(l1ls_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

// Largest supported shapes: the register-resident MFMA tile takes N <= 64,
// L <= 512; the streamed MFMA tile every shape up to N = 128, L = 4096 (the
// wave-per-pixel kernel up to L = 1024, the block form up to 1,024 columns a
// block; the FP64 continuation in registers up to 1,024 bins, beyond in
// workspace slots).
constexpr int kMaxNSolve = 128;
constexpr int kMaxLSolve = 4096;

bool mfma_supports(int n, int l) { return mfma_tile_shape(n, l); }

l1ls_status set_error(l1ls_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

l1ls_status check_options(const l1ls_options *o)
{
    if (!o) return fail(L1LS_ERR_INVALID_ARG, "options pointer is NULL");
    if (o->max_iter < 0) return fail(L1LS_ERR_INVALID_ARG, "max_iter must be >= 0 (got %d)", o->max_iter);
    if (!(o->tol > 0.0f) || !isfinite(o->tol))
        return fail(L1LS_ERR_INVALID_ARG, "tol must be finite and > 0");
    if (!(o->c_alpha > 0.0f && o->c_alpha < 1.0f))
        return fail(L1LS_ERR_INVALID_ARG, "c_alpha must lie in (0, 1)");
    if (o->precision != L1LS_FP32 && o->precision != L1LS_SPLIT_BF16)
        return fail(L1LS_ERR_INVALID_ARG, "unknown precision %d", o->precision);
    if (o->warm_start != 0 && o->warm_start != 1) return fail(L1LS_ERR_INVALID_ARG, "warm_start must be 0 or 1");
    if (o->fp64_continue != 0 && o->fp64_continue != 1)
        return fail(L1LS_ERR_INVALID_ARG, "fp64_continue must be 0 or 1");
    if (o->fp64_polish < 0 || o->fp64_polish > 2)
        return fail(L1LS_ERR_INVALID_ARG, "fp64_polish must be 0, 1 or 2");
    if (o->iteration_kernel < L1LS_ITER_AUTO || o->iteration_kernel > L1LS_ITER_STREAM)
        return fail(L1LS_ERR_INVALID_ARG, "unknown iteration_kernel %d", o->iteration_kernel);
    return L1LS_OK;
}

int options_choice(const l1ls_options *opt)
{
    switch (opt ? opt->iteration_kernel : L1LS_ITER_AUTO) {
    case L1LS_ITER_MFMA: return kMfma;
    case L1LS_ITER_WAVE: return kWave;
    case L1LS_ITER_STREAM: return kStream;
    default: return kAuto;
    }
}

bool needs_stream_state(int n, int l, const l1ls_options *opt)
{
    const int c = options_choice(opt);
    return c == kStream || (c == kAuto && auto_stream(n, l, opt ? opt->precision : L1LS_FP32));
}

static l1ls_status check_shape(int32_t n, int32_t l, int64_t p)
{
    if (n < 1 || l < 1 || p < 0) return fail(L1LS_ERR_INVALID_ARG, "need n >= 1, l >= 1, p >= 0");
    if (p >= ((int64_t)1 << 31)) return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "p must be < 2^31");
    if (n > kMaxNSolve || l > kMaxLSolve)
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "supported sizes: n <= %d, l <= %d (got %d, %d)",
                    kMaxNSolve, kMaxLSolve, n, l);
    return L1LS_OK;
}

// Split-BF16 contractions exist in the MFMA tiles only; the wave-per-pixel
// kernel refuses it rather than run FP32.
static l1ls_status check_precision(int32_t n, int32_t l, const l1ls_options *o)
{
    if (o->precision == L1LS_SPLIT_BF16 && o->iteration_kernel == L1LS_ITER_WAVE)
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "split-BF16 runs on the MFMA tiles only (not the wave kernel)");
    if (o->iteration_kernel == L1LS_ITER_MFMA && !mfma_supports(n, l))
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "the register-resident MFMA tile needs n <= 64, l <= 512");
    if (o->iteration_kernel == L1LS_ITER_WAVE && l > 1024)
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "the wave-per-pixel kernel needs l <= 1024");
    return L1LS_OK;
}

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Event timing of the solve's kernels (opt-in, for measurement), one list per
// kernel class (l1ls_kernel_class).
static std::mutex g_tmu;
static bool g_timing = false;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events[3];

// Calls that must not allocate (l1ls_solve_noalloc) leave the events out.
static thread_local bool g_no_events = false;

struct TimedLaunch {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s;
    int cls;
    TimedLaunch(hipStream_t st, int c) : s(st), cls(c)
    {
        if (g_no_events) return;
        std::lock_guard<std::mutex> g(g_tmu);
        if (!g_timing) return;
        hipEventCreate(&e0);
        hipEventCreate(&e1);
        hipEventRecord(e0, s);
    }
    ~TimedLaunch()
    {
        if (!e0) return;
        hipEventRecord(e1, s);
        std::lock_guard<std::mutex> g(g_tmu);
        g_events[cls].push_back({e0, e1});
    }
};

SolveOpts solve_opts(const l1ls_options *opt)
{
    SolveOpts o{};
    int cap = opt->max_iter;
    if (opt->polish_after > 0 && opt->polish_after < cap) cap = opt->polish_after;
    o.fista_cap = cap;
    o.tol = opt->tol;
    o.c_alpha = opt->c_alpha;
    o.backtracking = opt->backtracking ? 1 : 0;
    o.monotone = opt->monotone ? 1 : 0;
    o.polish = opt->fp64_polish;
    o.warm = opt->warm_start;
    o.max_iter = opt->max_iter;
    o.cont = opt->fp64_continue && opt->fp64_polish ? 1 : 0;
    return o;
}

// Checks of one stack's arguments before anything is queued.
l1ls_status check_stack(int32_t n, int32_t l, int64_t p, const void *A, const void *B, const float *lambda,
                        int64_t lambda_stride, const void *X, const void *ws, size_t ws_bytes, bool stream)
{
    l1ls_status st = check_shape(n, l, p);
    if (st != L1LS_OK) return st;
    if (p == 0) return L1LS_OK;
    if (!A || !B || !lambda || !X || !ws) return fail(L1LS_ERR_INVALID_ARG, "NULL pointer argument");
    if (!aligned(A, 8) || !aligned(B, 8) || !aligned(X, 8) || !aligned(lambda, 4))
        return fail(L1LS_ERR_INVALID_ARG, "A, B, X must be 8-byte aligned and lambda 4-byte aligned");
    if (!aligned(ws, 256)) return fail(L1LS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (lambda_stride < 0) return fail(L1LS_ERR_INVALID_ARG, "lambda_stride must be >= 0");
    const size_t need = stack_workspace_bytes(n, l, p, stream);
    if (ws_bytes < need) return fail(L1LS_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    return L1LS_OK;
}

// The iteration variant of a stack (choice kAuto / kMfma / kWave / kStream, `alt`
// an alternative tiling).
l1ls_status stack_variant(int32_t n, int32_t l, const l1ls_options *opt, int choice, int alt, IterVariant *v)
{
    const l1ls_status st = check_precision(n, l, opt);
    if (st != L1LS_OK) return st;
    if (choice == kMfma && !mfma_supports(n, l))
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "MFMA kernel needs n <= 64, l <= 512");
    if (!iter_variant(n, l, opt->precision, choice, alt, v))
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "no iteration kernel variant %d for n = %d, l = %d", alt, n, l);
    return L1LS_OK;
}

StackDesc stack_desc(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B, const float *lambda,
                     int64_t lambda_stride, l1ls_c32 *X, const l1ls_diag *diag, void *ws, const IterVariant &v)
{
    StackDesc d{};
    d.A = (const float2 *)A;
    d.B = (const float2 *)B;
    d.lambda = lambda;
    d.X = (float2 *)X;
    d.ws = (char *)ws;
    if (diag) {
        d.iters = diag->iters;
        d.kkt = diag->kkt;
        d.objective = diag->objective;
        d.status = diag->status;
        d.nnz = diag->nnz;
    }
    d.p = p;
    d.lambda_stride = lambda_stride;
    d.n = n;
    d.l = l;
    d.keep_residual = v.family == kVarMfma || v.family == kVarStream ? 1 : 0;
    return d;
}

// Queue the whole solve of `count` stacks (their variants in `var`): setup of
// every stack, one iteration launch per variant (tables of up to
// kMaxStacksPerLaunch), the two refinement passes and the certificate.
l1ls_status run_stacks(const StackDesc *d, const IterVariant *var, int count, const l1ls_options *opt,
                       hipStream_t s)
{
    const SolveOpts o = solve_opts(opt);
    auto chunks = [&](auto &&fn) -> hipError_t {
        StackTable t{};
        t.o = o;
        for (int i = 0; i < count; i += kMaxStacksPerLaunch) {
            t.count = std::min(kMaxStacksPerLaunch, count - i);
            for (int k = 0; k < t.count; ++k) t.d[k] = d[i + k];
            const hipError_t e = fn(t);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipError_t e = chunks([&](const StackTable &t) { return launch_setup_table(t, opt->fp64_polish != 0, s); });
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "setup launch: %s", hipGetErrorString(e));
    {
        TimedLaunch tl(s, L1LS_KERNEL_ITERATION);
        std::vector<bool> done(count, false);
        for (int i = 0; i < count && e == hipSuccess; ++i) {
            if (done[i]) continue;
            StackTable t{};
            t.o = o;
            for (int k = i; k < count && e == hipSuccess; ++k) {
                if (done[k] || !(var[k] == var[i])) continue;
                done[k] = true;
                t.d[t.count++] = d[k];
                if (t.count == kMaxStacksPerLaunch) {
                    e = launch_iteration_table(t, var[i], s);
                    t.count = 0;
                }
            }
            if (e == hipSuccess && t.count > 0) e = launch_iteration_table(t, var[i], s);
        }
    }
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "iteration launch: %s", hipGetErrorString(e));
    if (opt->fp64_polish) {
        TimedLaunch tl(s, L1LS_KERNEL_REFINE);
        e = chunks([&](const StackTable &t) { return launch_polish_table(t, s); });
        // pixels whose 8-slot (then 16-slot) working set filled above tol: the next
        // pass starts from the point the last one left in X (its FP64 objective is
        // recomputed)
        if (e == hipSuccess) e = chunks([&](const StackTable &t) { return launch_polish_mid_table(t, s); });
        if (e == hipSuccess) e = chunks([&](const StackTable &t) { return launch_polish_wide_table(t, s); });
        // what the 32-slot pass leaves above tol: Algorithm 1 in FP64 (fp64_continue)
        if (e == hipSuccess) e = chunks([&](const StackTable &t) { return launch_continue_table(t, s); });
        if (e != hipSuccess) return fail(L1LS_ERR_HIP, "refinement launch: %s", hipGetErrorString(e));
    }
    {
        TimedLaunch tl(s, L1LS_KERNEL_CERTIFY);
        e = chunks([&](const StackTable &t) { return launch_certify_table(t, s); });
    }
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "certify launch: %s", hipGetErrorString(e));
    return L1LS_OK;
}

l1ls_status solve_stack(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B,
                        const float *lambda, int64_t lambda_stride, const l1ls_options *opt,
                        l1ls_c32 *X, const l1ls_diag *diag, void *ws, size_t ws_bytes,
                        hipStream_t s, int choice, int blocks, const double *draws, int alt)
{
    l1ls_status st = check_shape(n, l, p);
    if (st != L1LS_OK) return st;
    st = check_options(opt);
    if (st != L1LS_OK) return st;
    if (p == 0) return L1LS_OK;
    if (choice == kAuto) choice = options_choice(opt);
    IterVariant v{};
    if (choice != kBlocks) {
        st = stack_variant(n, l, opt, choice, alt, &v);
        if (st != L1LS_OK) return st;
    }
    st = check_stack(n, l, p, A, B, lambda, lambda_stride, X, ws, ws_bytes, v.family == kVarStream);
    if (st != L1LS_OK) return st;
    if (choice != kBlocks) {
        const StackDesc d = stack_desc(n, l, p, A, B, lambda, lambda_stride, X, diag, ws, v);
        return run_stacks(&d, &v, 1, opt, s);
    }
    // Algorithm 1 with J column blocks: its own iteration kernel, then the same
    // refinement and certificate
    if (opt->warm_start) return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "warm_start is not available in the block form");
    IterVariant none{};
    const StackDesc d = stack_desc(n, l, p, A, B, lambda, lambda_stride, X, diag, ws, none);
    const SolveOpts o = solve_opts(opt);
    StackTable t{};
    t.count = 1;
    t.o = o;
    t.d[0] = d;
    hipError_t e = launch_setup_table(t, opt->fp64_polish != 0, s);
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "setup launch: %s", hipGetErrorString(e));
    const StackWorkspace lay = stack_workspace_layout(n, l, p);
    BlocksArgs ba;
    ba.f = fista_args_for(d, o);
    ba.J = blocks;
    ba.u = draws;
    ba.bc = (const BlockConsts *)((char *)ws + lay.blocks);
    e = launch_setup_blocks(n, l, blocks, (const float2 *)A, (BlockConsts *)((char *)ws + lay.blocks), s);
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "block setup launch: %s", hipGetErrorString(e));
    {
        TimedLaunch tl(s, L1LS_KERNEL_ITERATION);
        e = launch_fista_blocks(ba, s);
    }
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "iteration launch: %s", hipGetErrorString(e));
    if (opt->fp64_polish) {
        TimedLaunch tl(s, L1LS_KERNEL_REFINE);
        e = launch_polish_table(t, s);
        if (e == hipSuccess) e = launch_polish_mid_table(t, s);
        if (e == hipSuccess) e = launch_polish_wide_table(t, s);
        if (e == hipSuccess) e = launch_continue_table(t, s);
        if (e != hipSuccess) return fail(L1LS_ERR_HIP, "refinement launch: %s", hipGetErrorString(e));
    }
    {
        TimedLaunch tl(s, L1LS_KERNEL_CERTIFY);
        e = launch_certify_table(t, s);
    }
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "certify launch: %s", hipGetErrorString(e));
    return L1LS_OK;
}

// Workspace of l1ls_solve_noalloc: one statically sized array in the code
// object, so each device the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: its device address is looked up once per device (with that
// device current) and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[L1LS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices];

static l1ls_status scratch_for_current_device(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "device %d beyond the %d devices with scratch", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(L1LS_ERR_HIP, "scratch address on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return L1LS_OK;
}

}  // namespace l1ls

using namespace l1ls;

extern "C" {

l1ls_options l1ls_options_default(void)
{
    l1ls_options o;
    o.max_iter = 500;
    o.tol = 1e-4f;
    o.c_alpha = 0.5f;
    o.precision = L1LS_FP32;
    o.backtracking = 1;
    o.monotone = 1;
    o.fp64_polish = 1;
    o.polish_after = 0;
    o.warm_start = 0;
    o.fp64_continue = 1;
    o.iteration_kernel = L1LS_ITER_AUTO;
    return o;
}

l1ls_status l1ls_workspace_size(int32_t n, int32_t l, int64_t p, const l1ls_options *opt,
                                size_t *bytes)
{
    if (!bytes) return fail(L1LS_ERR_INVALID_ARG, "bytes pointer is NULL");
    l1ls_status st = check_shape(n, l, p);
    if (st != L1LS_OK) return st;
    if (opt) {
        st = check_options(opt);
        if (st == L1LS_OK) st = check_precision(n, l, opt);
        if (st != L1LS_OK) return st;
    }
    *bytes = stack_workspace_bytes(n, l, p, needs_stream_state(n, l, opt));
    return L1LS_OK;
}

l1ls_status l1ls_solve(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B,
                       const float *lambda, int64_t lambda_stride, const l1ls_options *opt,
                       l1ls_c32 *X, const l1ls_diag *diag, void *workspace, size_t ws_bytes,
                       hipStream_t stream)
{
    return solve_stack(n, l, p, A, B, lambda, lambda_stride, opt, X, diag, workspace, ws_bytes,
                       stream, kAuto);
}

l1ls_status l1ls_solve_noalloc(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B,
                               const float *lambda, int64_t lambda_stride, const l1ls_options *opt,
                               l1ls_c32 *X, const l1ls_diag *diag, hipStream_t stream)
{
    l1ls_status st = check_shape(n, l, p);
    if (st != L1LS_OK) return st;
    st = check_options(opt);
    if (st != L1LS_OK) return st;
    bool state = needs_stream_state(n, l, opt);
    int choice = options_choice(opt);
    if (state && choice == kAuto && mfma_supports(n, l) &&
        stack_workspace_bytes(n, l, p, true) > (size_t)L1LS_NOALLOC_SCRATCH_BYTES) {
        // the automatic choice takes the register tile when the streamed tile's
        // state does not fit the scratch (the same results bit for bit)
        state = false;
        choice = kMfma;
    }
    const size_t need = stack_workspace_bytes(n, l, p, state);
    if (need > (size_t)L1LS_NOALLOC_SCRATCH_BYTES)
        return fail(L1LS_ERR_WORKSPACE,
                    "l1ls_solve_noalloc: n=%d, l=%d, p=%lld needs %zu bytes of scratch, above its "
                    "fixed %zu (use l1ls_solve with a workspace)",
                    n, l, (long long)p, need, (size_t)L1LS_NOALLOC_SCRATCH_BYTES);
    if (p == 0) return L1LS_OK;
    void *ws = nullptr;
    st = scratch_for_current_device(&ws);
    if (st != L1LS_OK) return st;
    g_no_events = true;
    st = solve_stack(n, l, p, A, B, lambda, lambda_stride, opt, X, diag, ws,
                     (size_t)L1LS_NOALLOC_SCRATCH_BYTES, stream, choice);
    g_no_events = false;
    return st;
}

l1ls_status l1ls_solve_blocks(int32_t n, int32_t l, int64_t p, const l1ls_c32 *A, const l1ls_c32 *B,
                              const float *lambda, int64_t lambda_stride, const l1ls_options *opt,
                              int32_t blocks, const double *draws, l1ls_c32 *X, const l1ls_diag *diag,
                              void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (blocks < 1 || blocks > kMaxBlocks || blocks > l)
        return fail(L1LS_ERR_INVALID_ARG, "blocks must be in [1, min(64, l)], got %d", blocks);
    if (n > 64) return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "the block form takes n <= 64");
    if (opt && opt->precision == L1LS_SPLIT_BF16)
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "the block form computes its products in FP32 only");
    if (!draws && p > 0) return fail(L1LS_ERR_INVALID_ARG, "draws is NULL");
    if ((l + blocks - 1) / blocks > 1024)
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "the block form takes blocks of at most 1024 columns");
    if (opt && fista_blocks_lds(n, lpad_for(l), blocks) > 64 * 1024)
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "block form needs more than 64 KB of LDS per pixel");
    return solve_stack(n, l, p, A, B, lambda, lambda_stride, opt, X, diag, workspace, ws_bytes,
                       stream, kBlocks, blocks, draws);
}

const char *l1ls_status_string(l1ls_status s)
{
    switch (s) {
    case L1LS_OK: return "L1LS_OK";
    case L1LS_ERR_INVALID_ARG: return "L1LS_ERR_INVALID_ARG";
    case L1LS_ERR_UNSUPPORTED_SHAPE: return "L1LS_ERR_UNSUPPORTED_SHAPE";
    case L1LS_ERR_WORKSPACE: return "L1LS_ERR_WORKSPACE";
    case L1LS_ERR_HIP: return "L1LS_ERR_HIP";
    case L1LS_ERR_INTERNAL: return "L1LS_ERR_INTERNAL";
    }
    return "unknown status";
}

const char *l1ls_last_error(void) { return g_err; }

l1ls_status l1ls_solve_counters(int32_t n, int32_t l, int64_t p, const void *workspace,
                                hipStream_t stream, uint64_t out[5])
{
    if (!workspace || !out) return fail(L1LS_ERR_INVALID_ARG, "NULL pointer argument");
    const StackWorkspace lay = stack_workspace_layout(n, l, p);
    unsigned long long w2[4] = {0, 0, 0, 0};
    uint32_t q[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(w2, (const char *)workspace + lay.work, sizeof w2,
                                  hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(q, (const char *)workspace + lay.queue, sizeof q, hipMemcpyDeviceToHost,
                           stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "counter read: %s", hipGetErrorString(e));
    out[0] = w2[0];
    out[1] = w2[1];
    out[2] = q[1];
    out[3] = w2[2];
    out[4] = w2[3];
    return L1LS_OK;
}

l1ls_status l1ls_solve_constants(int32_t n, int32_t l, int64_t p, const void *workspace, hipStream_t stream,
                                 double out[3])
{
    if (!workspace || !out) return fail(L1LS_ERR_INVALID_ARG, "NULL pointer argument");
    l1ls_status st = check_shape(n, l, p);
    if (st != L1LS_OK) return st;
    const StackWorkspace lay = stack_workspace_layout(n, l, p);
    StackConsts c{};
    hipError_t e = hipMemcpyAsync(&c, (const char *)workspace + lay.consts, sizeof c, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "constants read: %s", hipGetErrorString(e));
    out[0] = c.lf;
    out[1] = c.alpha0;
    out[2] = c.lmax_it;
    return L1LS_OK;
}

void l1ls_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> g(g_tmu);
    g_timing = on != 0;
}

int32_t l1ls_timing_read_kernel(int32_t kernel_class, double *total_ms, int32_t *launches)
{
    if (kernel_class < 0 || kernel_class > 2) {
        if (total_ms) *total_ms = 0.0;
        if (launches) *launches = 0;
        return -1;
    }
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> g(g_tmu);
        ev.swap(g_events[kernel_class]);
    }
    double tot = 0.0;
    int cnt = 0;
    for (auto &pr : ev) {
        float ms = 0.0f;
        if (hipEventSynchronize(pr.second) == hipSuccess &&
            hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
            tot += ms;
            ++cnt;
        }
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    return cnt;
}

int32_t l1ls_timing_read(double *total_ms, int32_t *launches)
{
    return l1ls_timing_read_kernel(L1LS_KERNEL_ITERATION, total_ms, launches);
}

static l1ls_status check_unrolled(int32_t n, int32_t l, int64_t p, int32_t K, int32_t ckpt)
{
    if (n < 1 || l < 1 || p < 0) return fail(L1LS_ERR_INVALID_ARG, "need n >= 1, l >= 1, p >= 0");
    if (K < 1 || ckpt < 1 || K % ckpt != 0)
        return fail(L1LS_ERR_INVALID_ARG, "need K >= 1, ckpt_every >= 1 dividing K (got %d, %d)", K, ckpt);
    if (n > 128 || (7 * l + 2 * n) * 8 * 4 > 160 * 1024)
        return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "unrolled map supports n <= 128 and 7 l + 2 n <= 5120");
    if (p >= ((int64_t)1 << 31)) return fail(L1LS_ERR_UNSUPPORTED_SHAPE, "p must be < 2^31");
    return L1LS_OK;
}

l1ls_status l1ls_unrolled_tape_size(int32_t n, int32_t l, int64_t p, int32_t K, int32_t ckpt,
                                    size_t *bytes)
{
    if (!bytes) return fail(L1LS_ERR_INVALID_ARG, "bytes pointer is NULL");
    l1ls_status st = check_unrolled(n, l, p, K, ckpt);
    if (st != L1LS_OK) return st;
    *bytes = unrolled_tape_bytes(n, l, p, K, ckpt);
    return L1LS_OK;
}

l1ls_status l1ls_unrolled_backward_ws_size(int32_t n, int32_t l, int64_t p, int32_t K, int32_t ckpt,
                                           size_t *bytes)
{
    if (!bytes) return fail(L1LS_ERR_INVALID_ARG, "bytes pointer is NULL");
    l1ls_status st = check_unrolled(n, l, p, K, ckpt);
    if (st != L1LS_OK) return st;
    *bytes = unrolled_bwd_ws_bytes(n, l, p, K, ckpt);
    return L1LS_OK;
}

l1ls_status l1ls_unrolled_forward(int32_t n, int32_t l, int64_t p, const float *xi, const float *s,
                                  const l1ls_c32 *B, float lambda, float alpha, int32_t K,
                                  int32_t ckpt, l1ls_c32 *X_K, void *tape, size_t tape_bytes,
                                  hipStream_t stream)
{
    l1ls_status st = check_unrolled(n, l, p, K, ckpt);
    if (st != L1LS_OK) return st;
    if (!xi || !s || !tape || (p > 0 && (!B || !X_K)))
        return fail(L1LS_ERR_INVALID_ARG, "NULL pointer argument");
    if (!(lambda >= 0.0f) || !isfinite(lambda) || !(alpha > 0.0f) || !isfinite(alpha))
        return fail(L1LS_ERR_INVALID_ARG, "need finite lambda >= 0 and alpha > 0");
    if (!aligned(tape, 256)) return fail(L1LS_ERR_INVALID_ARG, "tape must be 256-byte aligned");
    if (tape_bytes < unrolled_tape_bytes(n, l, p, K, ckpt))
        return fail(L1LS_ERR_WORKSPACE, "tape too small");
    hipError_t e = launch_unrolled_forward(n, l, p, xi, s, (const float2 *)B, lambda, alpha, K, ckpt,
                                           (float2 *)X_K, tape, stream);
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "unrolled forward: %s", hipGetErrorString(e));
    return L1LS_OK;
}

l1ls_status l1ls_unrolled_backward(int32_t n, int32_t l, int64_t p, const float *xi, const float *s,
                                   const l1ls_c32 *B, float lambda, float alpha, int32_t K,
                                   int32_t ckpt, const void *tape, size_t tape_bytes,
                                   const l1ls_c32 *dX, l1ls_c32 *dB, float *dlambda, float *dxi,
                                   void *ws, size_t ws_bytes, hipStream_t stream)
{
    (void)xi;
    (void)s;
    l1ls_status st = check_unrolled(n, l, p, K, ckpt);
    if (st != L1LS_OK) return st;
    if (!tape || !dlambda || !dxi || !ws || (p > 0 && (!B || !dX || !dB)))
        return fail(L1LS_ERR_INVALID_ARG, "NULL pointer argument");
    if (!(lambda >= 0.0f) || !isfinite(lambda) || !(alpha > 0.0f) || !isfinite(alpha))
        return fail(L1LS_ERR_INVALID_ARG, "need finite lambda >= 0 and alpha > 0");
    if (!aligned(ws, 256) || !aligned(tape, 256))
        return fail(L1LS_ERR_INVALID_ARG, "tape and workspace must be 256-byte aligned");
    if (tape_bytes < unrolled_tape_bytes(n, l, p, K, ckpt)) return fail(L1LS_ERR_WORKSPACE, "tape too small");
    if (ws_bytes < unrolled_bwd_ws_bytes(n, l, p, K, ckpt))
        return fail(L1LS_ERR_WORKSPACE, "workspace too small");
    hipError_t e = launch_unrolled_backward(n, l, p, (const float2 *)B, lambda, alpha, K, ckpt, tape,
                                            (const float2 *)dX, (float2 *)dB, dlambda, dxi, ws, stream);
    if (e != hipSuccess) return fail(L1LS_ERR_HIP, "unrolled backward: %s", hipGetErrorString(e));
    return L1LS_OK;
}

}  // extern "C"
