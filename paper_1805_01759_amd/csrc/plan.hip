// Batched stacks of uneven shape: a plan assigns each stack an iteration tiling
// (register-resident MFMA tiles with A in LDS or from L2 and 32 or 64 unknowns
// a wave, the streamed MFMA tile, or the wave-per-pixel form), chosen by an
// autotuner (or named by the options' iteration_kernel) that times the
// candidates on a synthetic stack of the same (N, L) and keeps the result on
// disk, and lays out one workspace slice per stack.  Execution queues the
// solve of all stacks as stack tables: one setup launch, one persistent
// iteration launch per tiling class (its workgroups sweep the class's stacks,
// longest first, taking tiles from each stack's queue), the refinement passes
// and the certificate; it only enqueues work (no allocation, no host
// synchronisation), hence it can be captured into a HIP graph.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "l1ls_internal.h"

using namespace l1ls;

struct l1ls_plan {
    struct Item {
        int32_t n, l;
        int64_t p;
        IterVariant var;
        size_t ws_off, ws_bytes;
        double cost;
    };
    std::vector<Item> items;
    std::vector<int> order;  // longest first
    l1ls_options opt;
    size_t ws_total = 0;
    int device = 0;
};

namespace {

// ---------------------------------------------------------------------------
// Autotuner: per (device, n, l, precision, refinement mode) the fastest of the
// iteration tilings that exist for the shape (the MFMA tile with A in LDS or
// from L2, 32 or 64 unknowns a wave for short stacks; the streamed tile; and the
// wave-per-pixel kernel), timed on a synthetic stack of that shape.  Results are kept for the
// process and in a text cache file (one "device n l precision mode family T KB
// alds waves nc" line per shape): $L1LS_TUNE_CACHE, else
// $XDG_CACHE_HOME/l1ls/tune.txt, else $HOME/.cache/l1ls/tune.txt; "off" disables it.
std::mutex g_tune_mu;
std::map<std::string, IterVariant> g_tune_cache;
bool g_tune_loaded = false;

std::string tune_path()
{
    const char *e = getenv("L1LS_TUNE_CACHE");
    if (e && *e) return strcmp(e, "off") == 0 ? std::string() : std::string(e);
    const char *x = getenv("XDG_CACHE_HOME");
    if (x && *x) return std::string(x) + "/l1ls/tune.txt";
    const char *h = getenv("HOME");
    if (h && *h) return std::string(h) + "/.cache/l1ls/tune.txt";
    return std::string();
}

std::string device_tag(int dev)
{
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    std::string t = pr.gcnArchName;
    for (auto &c : t)
        if (c == ' ' || c == ':') c = '_';
    return t + "_" + std::to_string(pr.multiProcessorCount);
}

std::string tune_key(const std::string &dev, int n, int l, const l1ls_options &o)
{
    char b[128];
    snprintf(b, sizeof b, "%s %d %d %d %d", dev.c_str(), n, l, o.precision, o.fp64_polish);
    return b;
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const std::string path = tune_path();
    if (path.empty()) return;
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    char dev[96];
    int n, l, prec, mode;
    IterVariant v{};
    while (fscanf(f, "%95s %d %d %d %d %d %d %d %d %d %d", dev, &n, &l, &prec, &mode, &v.family, &v.T, &v.KB,
                  &v.alds, &v.waves, &v.nc) == 11) {
        l1ls_options o{};
        o.precision = prec;
        o.fp64_polish = mode;
        v.prec = v.family == kVarWave ? L1LS_FP32 : prec;
        v.wmax = v.family == kVarMfma && v.KB == 2 ? 8 : 4;
        g_tune_cache[tune_key(dev, n, l, o)] = v;
    }
    fclose(f);
}

void tune_store_locked(const std::string &key, const IterVariant &v)
{
    const std::string path = tune_path();
    if (path.empty()) return;
    // create the directory chain of the file, then append one line
    for (size_t k = 1; k < path.size(); ++k)
        if (path[k] == '/') mkdir(path.substr(0, k).c_str(), 0755);
    FILE *f = fopen(path.c_str(), "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %d %d\n", key.c_str(), v.family, v.T, v.KB, v.alds, v.waves, v.nc);
    fclose(f);
}

// Time one solve of a synthetic stack of this shape with the given tiling.
double time_variant(int n, int l, int64_t p, const l1ls_options &opt, int choice, int alt, void *A, void *B,
                    void *lam, void *X, void *ws, size_t ws_bytes, hipStream_t s)
{
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    // one warm-up, then the timed run
    double best = 1e30;
    for (int rep = 0; rep < 2; ++rep) {
        hipEventRecord(e0, s);
        l1ls_status st = solve_stack(n, l, p, (const l1ls_c32 *)A, (const l1ls_c32 *)B, (const float *)lam, 1,
                                     &opt, (l1ls_c32 *)X, nullptr, ws, ws_bytes, s, choice, 0, nullptr, alt);
        hipEventRecord(e1, s);
        hipEventSynchronize(e1);
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        if (st != L1LS_OK) ms = 1e30f;
        if (rep == 1) best = ms;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return best;
}

// Synthetic TomoSAR-like stack for tuning: unit-modulus A with a smooth phase
// ramp, two scatterers plus noise per pixel.
IterVariant autotune(int n, int l, const l1ls_options &opt, int dev)
{
    const std::string key = tune_key(device_tag(dev), n, l, opt);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tune_load_locked();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    // the candidates that exist for this shape
    std::vector<std::pair<int, int>> cands;  // (choice, alt)
    IterVariant probe;
    for (int alt = 0; alt < 3; ++alt)
        if (mfma_supports(n, l) && iter_variant(n, l, opt.precision, kMfma, alt, &probe))
            cands.push_back({kMfma, alt});
    // the streamed tile (either precision)
    if (iter_variant(n, l, opt.precision, kStream, 0, &probe)) cands.push_back({kStream, 0});
    if (opt.precision == L1LS_FP32) cands.push_back({kWave, 0});  // the wave kernel is FP32 only
    IterVariant best_v;
    iter_variant(n, l, opt.precision, cands[0].first, cands[0].second, &best_v);
    if (cands.size() > 1) {
        const int64_t p = 4096;
        std::vector<float> hA(2 * (size_t)n * l), hB(2 * (size_t)p * n), hl(p);
        uint64_t st = 0x9e3779b97f4a7c15ull;
        auto rnd = [&]() {
            st ^= st << 13;
            st ^= st >> 7;
            st ^= st << 17;
            return (double)(st >> 11) / 9007199254740992.0;
        };
        std::vector<double> xi(n);
        for (int i = 0; i < n; ++i) xi[i] = (rnd() - 0.5) * 0.05;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < l; ++j) {
                const double sv = -50.0 + 100.0 * j / (l > 1 ? l - 1 : 1);
                const double ph = -2.0 * 3.14159265358979 * xi[i] * sv;
                hA[2 * ((size_t)i * l + j)] = (float)cos(ph);
                hA[2 * ((size_t)i * l + j) + 1] = (float)sin(ph);
            }
        for (int64_t q = 0; q < p; ++q) {
            const int j1 = (int)(rnd() * l), j2 = (int)(rnd() * l);
            for (int i = 0; i < n; ++i) {
                const float *a1 = &hA[2 * ((size_t)i * l + j1)], *a2 = &hA[2 * ((size_t)i * l + j2)];
                hB[2 * ((size_t)q * n + i)] = a1[0] + 0.7f * a2[0] + 0.3f * (float)(rnd() - 0.5);
                hB[2 * ((size_t)q * n + i) + 1] = a1[1] + 0.7f * a2[1] + 0.3f * (float)(rnd() - 0.5);
            }
            hl[q] = 0.3f * sqrtf(2.0f * n * logf((float)l + 1.0f));
        }
        l1ls_options o = opt;
        o.warm_start = 0;
        const size_t wsb = stack_workspace_bytes(n, l, p, true);
        void *dA = nullptr, *dB = nullptr, *dl = nullptr, *dX = nullptr, *dws = nullptr;
        if (hipMalloc(&dA, hA.size() * 4) == hipSuccess && hipMalloc(&dB, hB.size() * 4) == hipSuccess &&
            hipMalloc(&dl, hl.size() * 4) == hipSuccess && hipMalloc(&dX, (size_t)p * l * 8) == hipSuccess &&
            hipMalloc(&dws, wsb) == hipSuccess) {
            hipStream_t s;
            hipStreamCreate(&s);
            hipMemcpyAsync(dA, hA.data(), hA.size() * 4, hipMemcpyHostToDevice, s);
            hipMemcpyAsync(dB, hB.data(), hB.size() * 4, hipMemcpyHostToDevice, s);
            hipMemcpyAsync(dl, hl.data(), hl.size() * 4, hipMemcpyHostToDevice, s);
            double tbest = 1e30;
            for (auto &c : cands) {
                const double tm = time_variant(n, l, p, o, c.first, c.second, dA, dB, dl, dX, dws, wsb, s);
                if (tm < tbest) {
                    tbest = tm;
                    iter_variant(n, l, opt.precision, c.first, c.second, &best_v);
                }
            }
            hipStreamSynchronize(s);
            hipStreamDestroy(s);
        }
        hipFree(dA);
        hipFree(dB);
        hipFree(dl);
        hipFree(dX);
        hipFree(dws);
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = best_v;
    tune_store_locked(key, best_v);
    return best_v;
}

}  // namespace

extern "C" {

l1ls_status l1ls_plan_create(const l1ls_stack *stacks, int32_t count, const l1ls_options *opt,
                             l1ls_plan **out)
{
    if (!out) return set_error(L1LS_ERR_INVALID_ARG, "out pointer is NULL");
    *out = nullptr;
    if (!opt) return set_error(L1LS_ERR_INVALID_ARG, "options pointer is NULL");
    if (count < 0 || (count > 0 && !stacks)) return set_error(L1LS_ERR_INVALID_ARG, "bad stack list");
    size_t probe = 0;
    for (int i = 0; i < count; ++i) {
        l1ls_status st = l1ls_workspace_size(stacks[i].n, stacks[i].l, stacks[i].p, opt, &probe);
        if (st != L1LS_OK) return st;
    }
    l1ls_plan *pl = new l1ls_plan();
    pl->opt = *opt;
    hipGetDevice(&pl->device);
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        l1ls_plan::Item it;
        it.n = stacks[i].n;
        it.l = stacks[i].l;
        it.p = stacks[i].p;
        if (opt->iteration_kernel != L1LS_ITER_AUTO) {
            // the kernel the options name (l1ls_workspace_size has checked that it takes the shape)
            iter_variant(it.n, it.l, opt->precision, options_choice(opt), 0, &it.var);
        } else if (it.p > 0) {
            it.var = autotune(it.n, it.l, *opt, pl->device);
        } else {
            iter_variant(it.n, it.l, opt->precision, kAuto, 0, &it.var);
        }
        it.ws_bytes = stack_workspace_bytes(it.n, it.l, it.p, it.var.family == kVarStream);
        it.ws_off = off;
        off += (it.ws_bytes + 255) / 256 * 256;
        it.cost = (double)it.p * it.n * it.l;
        pl->items.push_back(it);
    }
    pl->ws_total = off;
    pl->order.resize(count);
    std::iota(pl->order.begin(), pl->order.end(), 0);
    std::stable_sort(pl->order.begin(), pl->order.end(),
                     [&](int a, int b) { return pl->items[a].cost > pl->items[b].cost; });
    *out = pl;
    return L1LS_OK;
}

l1ls_status l1ls_plan_workspace_size(const l1ls_plan *plan, size_t *bytes)
{
    if (!plan || !bytes) return set_error(L1LS_ERR_INVALID_ARG, "NULL argument");
    *bytes = plan->ws_total;
    return L1LS_OK;
}

l1ls_status l1ls_plan_execute(l1ls_plan *plan, const l1ls_stack *stacks, void *workspace,
                              size_t ws_bytes, hipStream_t stream)
{
    if (!plan) return set_error(L1LS_ERR_INVALID_ARG, "plan is NULL");
    const int count = (int)plan->items.size();
    if (count > 0 && !stacks) return set_error(L1LS_ERR_INVALID_ARG, "stacks is NULL");
    for (int i = 0; i < count; ++i) {
        const auto &it = plan->items[i];
        if (stacks[i].n != it.n || stacks[i].l != it.l || stacks[i].p != it.p)
            return set_error(L1LS_ERR_INVALID_ARG, "stack %d does not match the plan's shape", i);
    }
    if (plan->ws_total > 0 && (!workspace || ws_bytes < plan->ws_total))
        return set_error(L1LS_ERR_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, plan->ws_total);
    if (workspace && ((uintptr_t)workspace % 256) != 0)
        return set_error(L1LS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    // every stack's arguments are checked before anything is queued
    std::vector<StackDesc> descs;
    std::vector<IterVariant> vars;
    for (int idx : plan->order) {
        const auto &it = plan->items[idx];
        if (it.p == 0) continue;
        const l1ls_stack &sk = stacks[idx];
        char *ws = (char *)workspace + it.ws_off;
        const l1ls_status st = check_stack(it.n, it.l, it.p, sk.A, sk.B, sk.lambda, sk.lambda_stride, sk.X, ws,
                                           it.ws_bytes, it.var.family == kVarStream);
        if (st != L1LS_OK) return st;
        descs.push_back(stack_desc(it.n, it.l, it.p, sk.A, sk.B, sk.lambda, sk.lambda_stride, sk.X, &sk.diag, ws,
                                   it.var));
        vars.push_back(it.var);
    }
    if (descs.empty()) return L1LS_OK;
    return run_stacks(descs.data(), vars.data(), (int)descs.size(), &plan->opt, stream);
}

void l1ls_plan_destroy(l1ls_plan *plan) { delete plan; }

int32_t l1ls_plan_describe(const l1ls_plan *plan, char *buf, int32_t buf_len)
{
    if (!plan) return 0;
    std::string s;
    char line[200];
    for (size_t i = 0; i < plan->items.size(); ++i) {
        const auto &it = plan->items[i];
        const IterVariant &v = it.var;
        if (v.family == kVarWave)
            snprintf(line, sizeof line, "stack %zu: n=%d l=%d p=%lld kernel=wave chunks=%d\n", i, it.n, it.l,
                     (long long)it.p, v.nc);
        else if (v.family == kVarStream)
            snprintf(line, sizeof line, "stack %zu: n=%d l=%d p=%lld kernel=stream T=%d waves=%d\n", i, it.n,
                     it.l, (long long)it.p, v.T, v.waves);
        else
            snprintf(line, sizeof line, "stack %zu: n=%d l=%d p=%lld kernel=%s T=%d KB=%d waves=%d A=%s\n", i, it.n,
                     it.l, (long long)it.p, "mfma", v.T, v.KB, v.waves,
                     v.alds ? "lds" : "l2");
        s += line;
    }
    if (buf && buf_len > 0) {
        const size_t k = std::min<size_t>(s.size(), (size_t)buf_len - 1);
        memcpy(buf, s.data(), k);
        buf[k] = 0;
    }
    return (int32_t)s.size() + 1;
}

}  // extern "C"
