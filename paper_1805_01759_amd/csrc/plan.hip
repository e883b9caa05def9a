// Batched stacks of uneven shape: a plan assigns each stack an iteration
// kernel (register-resident MFMA tiles or the wave-per-pixel form), chosen by
// timing both on a synthetic problem of the stack's (N, L) class when the plan
// is built, and lays out one workspace slice per stack.  Execution forks the
// caller's stream into branch streams (longest stacks first, round robin), so
// that a captured HIP graph runs small stacks side by side; it only enqueues
// work (no allocation, no host synchronisation), hence it can be captured.
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

#include "l1ls_internal.h"

using namespace l1ls;

struct l1ls_plan {
    struct Item {
        int32_t n, l;
        int64_t p;
        int choice;
        size_t ws_off, ws_bytes;
        int branch;
        double cost;
    };
    std::vector<Item> items;
    l1ls_options opt;
    size_t ws_total = 0;
    std::vector<hipStream_t> branches;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    int device = 0;
};

namespace {

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tune_cache;  // (n, l, precision) -> choice

// Time one solve of a synthetic stack of this shape with the given kernel.
double time_choice(int n, int l, int64_t p, const l1ls_options &opt, int choice, void *A, void *B,
                   void *lam, void *X, void *ws, size_t ws_bytes, hipStream_t s)
{
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    // one warm-up, then the timed run
    double best = 1e30;
    for (int rep = 0; rep < 2; ++rep) {
        hipEventRecord(e0, s);
        l1ls_status st = solve_stack(n, l, p, (const l1ls_c32 *)A, (const l1ls_c32 *)B,
                                     (const float *)lam, 1, &opt, (l1ls_c32 *)X, nullptr, ws,
                                     ws_bytes, s, choice);
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
int autotune(int n, int l, const l1ls_options &opt)
{
    const auto key = std::make_tuple(n, l, opt.precision);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    if (!mfma_supports(n, l)) return kWave;
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
            const double s = -50.0 + 100.0 * j / (l > 1 ? l - 1 : 1);
            const double ph = -2.0 * 3.14159265358979 * xi[i] * s;
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
    size_t wsb = stack_workspace_layout(n, l, p).total;
    void *dA = nullptr, *dB = nullptr, *dl = nullptr, *dX = nullptr, *dws = nullptr;
    int choice = kMfma;
    if (hipMalloc(&dA, hA.size() * 4) == hipSuccess && hipMalloc(&dB, hB.size() * 4) == hipSuccess &&
        hipMalloc(&dl, hl.size() * 4) == hipSuccess &&
        hipMalloc(&dX, (size_t)p * l * 8) == hipSuccess && hipMalloc(&dws, wsb) == hipSuccess) {
        hipStream_t s;
        hipStreamCreate(&s);
        hipMemcpyAsync(dA, hA.data(), hA.size() * 4, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(dB, hB.data(), hB.size() * 4, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(dl, hl.data(), hl.size() * 4, hipMemcpyHostToDevice, s);
        const double tm = time_choice(n, l, p, opt, kMfma, dA, dB, dl, dX, dws, wsb, s);
        const double tw = time_choice(n, l, p, opt, kWave, dA, dB, dl, dX, dws, wsb, s);
        choice = tm <= tw ? kMfma : kWave;
        hipStreamSynchronize(s);
        hipStreamDestroy(s);
    }
    hipFree(dA);
    hipFree(dB);
    hipFree(dl);
    hipFree(dX);
    hipFree(dws);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = choice;
    return choice;
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
        it.choice = it.p > 0 ? autotune(it.n, it.l, *opt) : kAuto;
        l1ls_workspace_size(it.n, it.l, it.p, opt, &it.ws_bytes);
        it.ws_off = off;
        off += (it.ws_bytes + 255) / 256 * 256;
        it.cost = (double)it.p * it.n * it.l;
        it.branch = 0;
        pl->items.push_back(it);
    }
    pl->ws_total = off;
    // longest stacks first, dealt round robin to the branches
    const int nb = std::max(1, std::min<int>(count, 8));
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return pl->items[a].cost > pl->items[b].cost; });
    for (int r = 0; r < count; ++r) pl->items[order[r]].branch = r % nb;
    for (int b = 0; b < nb; ++b) {
        hipStream_t s;
        hipEvent_t e;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            l1ls_plan_destroy(pl);
            return set_error(L1LS_ERR_HIP, "stream/event creation failed");
        }
        pl->branches.push_back(s);
        pl->joins.push_back(e);
    }
    if (hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming) != hipSuccess) {
        l1ls_plan_destroy(pl);
        return set_error(L1LS_ERR_HIP, "event creation failed");
    }
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
    if (count == 0) return L1LS_OK;
    hipError_t e = hipEventRecord(plan->fork, stream);
    for (size_t b = 0; e == hipSuccess && b < plan->branches.size(); ++b)
        e = hipStreamWaitEvent(plan->branches[b], plan->fork, 0);
    if (e != hipSuccess) return set_error(L1LS_ERR_HIP, "fork: %s", hipGetErrorString(e));
    // launch in cost order within each branch
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return plan->items[a].cost > plan->items[b].cost; });
    l1ls_status result = L1LS_OK;
    for (int idx : order) {
        const auto &it = plan->items[idx];
        if (it.p == 0) continue;
        const l1ls_stack &sk = stacks[idx];
        l1ls_status st = solve_stack(it.n, it.l, it.p, sk.A, sk.B, sk.lambda, sk.lambda_stride,
                                     &plan->opt, sk.X, &sk.diag, (char *)workspace + it.ws_off,
                                     it.ws_bytes, plan->branches[it.branch], it.choice);
        if (st != L1LS_OK && result == L1LS_OK) result = st;
    }
    // join every branch back into the caller's stream
    for (size_t b = 0; b < plan->branches.size(); ++b) {
        hipEventRecord(plan->joins[b], plan->branches[b]);
        hipStreamWaitEvent(stream, plan->joins[b], 0);
    }
    return result;
}

void l1ls_plan_destroy(l1ls_plan *plan)
{
    if (!plan) return;
    for (auto s : plan->branches) hipStreamDestroy(s);
    for (auto e : plan->joins) hipEventDestroy(e);
    if (plan->fork) hipEventDestroy(plan->fork);
    delete plan;
}

int32_t l1ls_plan_describe(const l1ls_plan *plan, char *buf, int32_t buf_len)
{
    if (!plan) return 0;
    std::string s;
    char line[160];
    for (size_t i = 0; i < plan->items.size(); ++i) {
        const auto &it = plan->items[i];
        snprintf(line, sizeof line, "stack %zu: n=%d l=%d p=%lld kernel=%s branch=%d\n", i, it.n, it.l,
                 (long long)it.p, it.choice == kMfma ? "mfma" : (it.choice == kWave ? "wave" : "none"),
                 it.branch);
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
