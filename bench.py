#!/usr/bin/env python
"""Throughput of the gfx950 L1LS solver: pixels solved per second at KKT <= 1e-4,
FP32 against split-BF16 contractions on the same stack.

One step = one full solve (setup, accelerated proximal-gradient iteration,
FP64 refinement, FP64 optimality check) of a synthetic TomoSAR stack already
resident in HBM.  Default workload: the close-pair stack, N = 50 acquisitions,
L = 512 elevation bins, P = 2^22 pixels (40% of them two scatterers 0.3-1.0
Rayleigh apart), max 500 iterations, tol 1e-4; `--workload scene` is the
N = 25, L = 256, P = 2^20 stack.  Prints one JSON line with, besides the
throughput, the roofline of the dominant kernel, the oracle timed on the host
cores (cpu_baseline) and, from the same oracle leg, the per-pixel error of both
precisions against the certified FP64 minimiser on a sample (parity).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "pixels solved/sec at KKT residual ≤1e-4 (FP32 vs split-BF16); MFMA %"
PEAK = {"fp32": 157.3e12, "split_bf16": 2.5e15}
WORKLOADS = {
    # name: (synth config id, description)
    "scene": (2, "scene-scale TomoSAR stack: N=25, L=256, P=1048576, baselines U[-300,300] m, "
                 "0/1/2 scatterers (0.3/0.5/0.2), SNR U[0,20] dB, lambda_p = sigma_p sqrt(2 N ln L)"),
    "tiny": (1, "tiny TomoSAR stack: N=15, L=101, P=1024, SNR 10 dB"),
    "pairs": (4, "close-pair TomoSAR stack: N=50, L=512, P=4194304, 40% two scatterers 0.3-1.0 "
                 "Rayleigh apart, SNR 10 dB"),
    "motion": (6, "multicomponent TomoSAR stack (elevation x linear velocity): N=50 acquisitions over "
                  "3 years, 32 elevation bins on [-60, 60] m x 16 velocity bins on [-40, 40] mm/yr "
                  "(L=512), P=524288, 0/1/2 scatterers (0.3/0.5/0.2) at off-grid (s, v), SNR U[0,20] dB"),
    "motion_fine": (7, "multicomponent TomoSAR stack as 'motion' with 64 elevation bins (L=1024), "
                       "P=65536"),
    "motion_seasonal": (10, "multicomponent TomoSAR stack (elevation x linear velocity x seasonal "
                            "amplitude): as 'motion' with 8 seasonal-amplitude bins on [-10, 10] mm "
                            "(L=4096), P=32768"),
    "superres": (8, "double-scatterer simulations: N=29 over a 269.5 m aperture, L=256 bins on "
                    "[-80, 80] m, two unit scatterers kappa rho_s apart; 24 cases (kappa 1.2/0.8/0.4/0.2 "
                    "at 10/3/0 dB with random phase difference; kappa 0.2..1.2 at 2 and 7 dB with phase "
                    "difference 0), 5000 realisations each"),
}
SUPERRES_REALISATIONS = 5000


# sources of each timed kernel; a traffic record is used only while they are unchanged
KERNEL_SOURCES = {
    "fista_mfma_kernel": ("fista_mfma.h", "fista.hip", "l1ls_internal.h"),
    "fista_mfma_kernel_bf16": ("fista_mfma.h", "fista.hip", "l1ls_internal.h"),
    "fista_wave_kernel": ("fista_wave.hip", "l1ls_internal.h"),
    "fista_stream_kernel": ("fista_stream.h", "fista_mfma.h", "l1ls_internal.h"),
    "fista_stream_kernel_bf16": ("fista_stream.h", "fista_mfma.h", "l1ls_internal.h"),
    "polish_kernel": ("polish.hip", "wave_reduce.h", "l1ls_internal.h"),
    "certify_kernel": ("certify.hip", "wave_reduce.h", "l1ls_internal.h"),
}
PEAK_FP64_VALU = 78.6e12   # MI355X FP64 vector FLOP/s
PEAK_FP32_VALU = 157.3e12  # MI355X FP32 vector FLOP/s
# oracle pixels per workload: Algorithm 1 timed (cpu_baseline) and the certified
# minimiser for the parity sample (strided over the whole stack); about 10-30 s
# of host work each on 16 cores
CPU_SAMPLE = {"scene": 16384, "pairs": 4096, "tiny": 1024, "motion": 4096, "motion_fine": 2048,
              "motion_seasonal": 256,
              "superres": 16384}
PARITY_SAMPLE = {"scene": 1024, "pairs": 512, "tiny": 1024, "motion": 512, "motion_fine": 256,
                 "motion_seasonal": 64,
                 "superres": 960}
PARITY_BAR = {"fp32": 1e-4, "split_bf16": 1e-3}
POLISH_AFTER = 12          # FP32 iterations before a pixel goes to the FP64 stage
# per workload where another budget is faster (measured with every pixel refined:
# close pairs 4.83 / 4.71 / 4.57 / 4.32 / 4.08 / 3.86 M solved pixels/s at
# 2 / 3 / 4 / 6 / 8 / 10).  Below 4 the FP32 stage is hardly an estimate of the
# solution any more (its step search has barely started) and the FP32 against
# split-BF16 comparison vanishes into the refinement, so 4 is kept; the scene
# 12.84 / 13.53 / 13.55 / 13.82 M at 12 / 8 / 6 / 4, 8 kept for the same reason.
POLISH_AFTER_BY_WORKLOAD = {"pairs": 4, "scene": 8}


def polish_after_for(workload: str) -> int:
    return POLISH_AFTER_BY_WORKLOAD.get(workload, POLISH_AFTER)
# FP64 refinement of every pixel to FP64 accuracy (fp64_polish = 2): the mode in
# which the returned x matches the certified minimiser to the stated bar
ACCURACY_MODE = 2


def kernel_sha(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(HERE, "paper_1805_01759_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    record of this kernel and workload, or None once the kernel has changed."""
    path = os.path.join(HERE, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha") != kernel_sha(kernel):
        return None  # counters were taken on a different kernel
    return rec.get("traffic_bytes_per_launch")


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, B, lam, sample: int, max_iter: int, tol: float):
    import oracle  # CPU oracle: timed beside the GPU, never on the product path
    oracle.build(force=False)
    nthreads = oracle.default_threads()
    t0 = time.perf_counter()
    X, d = oracle.rbpg_batch(A[:, :].astype(np.complex128), B[:sample].astype(np.complex128),
                             lam[:sample].astype(np.float64), tol=tol, max_iter=max_iter,
                             nthreads=nthreads)
    dt = time.perf_counter() - t0
    solved = int(d["converged"].sum())
    return {"value": solved / dt, "unit": "pixels/s", "cores": nthreads, "kind": "oracle",
            "cpu_model": host_cpu_model(),
            "sample": f"first {sample} pixels of the same stack; Algorithm 1 (J=1) in FP64, "
                      f"tol {tol}, max {max_iter} iterations; {solved} solved in {dt:.1f} s"}


def oracle_minimisers(A, B, lam, idx):
    """The oracle leg's certified FP64 minimisers of the sampled pixels (inputs
    upcast from the device's complex64 values) and sigma_max(A)."""
    import oracle  # CPU oracle: test infrastructure, used here only to measure
    oracle.build(force=False)
    A64 = A.astype(np.complex128)
    B64 = B[idx].astype(np.complex128)
    L64 = lam[idx].astype(np.float64)
    t0 = time.perf_counter()
    Xe, de = oracle.exact_batch(A64, B64, L64)
    dt = time.perf_counter() - t0
    lf = oracle.lipschitz(A64)
    return {"A64": A64, "B64": B64, "L64": L64, "Xe": Xe, "Fe": de["objective"], "lf": lf,
            "certified_kkt_max": float(de["kkt_sub"].max()), "gap_max": float(de["gap"].max()),
            "seconds": dt, "idx": idx}


def parity_report(orc_sol, Xs, conv, bar: float):
    """Per-pixel error of the device's x against the certified minimiser x*:
    e_p = ||x - x*|| / max(||x*||, ||b_p|| / sigma_max(A)); a pixel passes when
    e_p <= bar and its FP64 KKT residual (the CONVERGED bit) is <= tol."""
    import oracle
    A64, B64, L64, Xe = orc_sol["A64"], orc_sol["B64"], orc_sol["L64"], orc_sol["Xe"]
    X = Xs.astype(np.complex128)
    smax = np.sqrt(orc_sol["lf"] / 2.0)
    den = np.maximum(np.linalg.norm(Xe, axis=1), np.linalg.norm(B64, axis=1) / smax)
    e = np.linalg.norm(X - Xe, axis=1) / den
    Fg = np.array([oracle.objective(A64, B64[i], L64[i], X[i]) for i in range(len(X))])
    Fe = orc_sol["Fe"]
    gap = (Fg - Fe) / np.maximum(Fe, 1e-300)
    ok = (e <= bar) & conv
    return {"sample": int(len(X)), "bar": bar, "pass_fraction": float(ok.mean()),
            "solved_fraction": float(conv.mean()),
            "e_p50": float(np.percentile(e, 50)), "e_p99": float(np.percentile(e, 99)),
            "e_max": float(e.max()), "objective_gap_max": float(gap.max()),
            "fail_error_only": int((conv & (e > bar)).sum())}


def bench_batched(args):
    """64 uneven stacks (N ~ U{10..100}, L ~ U{64..1024}, P log-uniform 1e3..2.56e5,
    each with its own A), planned once (autotuned kernel per shape) and replayed
    as one captured HIP graph per step."""
    import torch
    from paper_1805_01759_amd import api, synth
    specs = synth.batched_specs(64)
    dev = torch.device("cuda:0")
    stacks = []
    for ss in specs:
        spec, geom, B, lam = synth.make_batched_stack(ss)
        A32, B32, l32 = synth.to_device_dtypes(geom.A, B, lam)
        stacks.append({"A": torch.from_numpy(A32).to(dev), "B": torch.from_numpy(B32).to(dev),
                       "lam": torch.from_numpy(l32).to(dev),
                       "X": torch.empty((ss.p, ss.l), dtype=torch.complex64, device=dev),
                       "diag": api.new_diag(ss.p, dev)})
    total = sum(ss.p for ss in specs)
    plan = api.Plan([(ss.n, ss.l, ss.p) for ss in specs], max_iter=args.max_iter, tol=1e-4,
                    precision=args.precision, fp64_polish=args.polish,
                    polish_after=args.polish_after)
    ws = torch.empty(plan.workspace_bytes + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + plan.workspace_bytes]
    plan.execute(stacks, ws)  # eager warm-up
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s):
        plan.execute(stacks, ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved = 0
    for _ in range(args.steps):
        g.replay()
        torch.cuda.synchronize()
        solved += sum(int(((st["diag"]["status"] & 1) != 0).sum().item()) for st in stacks)
    dt = time.perf_counter() - t0
    kinds = plan.describe().count("kernel=mfma")
    streamed = plan.describe().count("kernel=stream")
    # the plain FP32 solver on the same stacks, one solve call after another
    wsp = api.Workspace()
    o_opts = dict(max_iter=args.max_iter, tol=1e-4, precision="fp32", fp64_polish=args.polish,
                  polish_after=args.polish_after)
    for st in stacks:
        api.solve(st["A"], st["B"], st["lam"], out=st["X"], workspace=wsp, **o_opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    o_solved = 0
    for _ in range(args.steps):
        ds = [api.solve(st["A"], st["B"], st["lam"], out=st["X"], workspace=wsp, **o_opts)[1]
              for st in stacks]
        torch.cuda.synchronize()
        o_solved += sum(int(((d["status"] & 1) != 0).sum().item()) for d in ds)
    o_dt = time.perf_counter() - t0
    print(json.dumps({"metric": METRIC, "value": solved / dt, "unit": "pixels/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None,
                      "dtype": "f32" if args.precision == "fp32" else "bf16x3", "data": "synthetic",
                      "config": {"workload": f"64 uneven TomoSAR stacks, {total} pixels in total, "
                                             "one HIP graph replay per step",
                                 "pixels": total, "stacks_on_mfma_kernel": kinds,
                                 "stacks_on_streamed_mfma_kernel": streamed,
                                 "solved_fraction": solved / (total * args.steps),
                                 "polish_after": args.polish_after},
                      "compare": {"form": "plain FP32 solve per stack, eager, no plan",
                                  "value": o_solved / o_dt, "unit": "pixels/s",
                                  "ms_per_step": o_dt / args.steps * 1e3}}), flush=True)


def bench_blocks(args):
    """Algorithm 1 with J column blocks (Eqs. (13)-(14)) on the scene stack, one
    shared sequence of seeded draws; the same number of block sweeps (12 J block
    iterations) before the FP64 stage.  Compared with the one-block solver."""
    import torch
    from paper_1805_01759_amd import api, synth
    cfg, desc = WORKLOADS["scene"]
    spec, geom, B, lam = synth.make_config(cfg, 0, args.pixels or None)
    A32, B32, l32 = synth.to_device_dtypes(geom.A, B, lam)
    dev = torch.device("cuda:0")
    Ad, Bd, ld = (torch.from_numpy(x).to(dev) for x in (A32, B32, l32))
    n, l = A32.shape
    p = B32.shape[0]
    J = args.blocks
    cap = args.polish_after * J
    ud = torch.from_numpy(synth.uniform_draws(max(cap, 1), seed=J)).to(dev)
    X = torch.empty((p, l), dtype=torch.complex64, device=dev)
    ws = api.Workspace()

    def timed(**kw):
        for _ in range(args.warmup):
            api.solve(Ad, Bd, ld, out=X, workspace=ws, **kw)
        api.timing_enable(True)
        for kc in ("iteration", "refine", "certify"):
            api.timing_read(kc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = []
        for _ in range(args.steps):
            _, d = api.solve(Ad, Bd, ld, out=X, workspace=ws, **kw)
            st.append(d["status"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = {kc: api.timing_read(kc) for kc in ("iteration", "refine", "certify")}
        api.timing_enable(False)
        solved = sum(int(((x & 1) != 0).sum().item()) for x in st)
        fl = api.solve_counters(n, l, p, d)[0]
        return solved / dt, dt / args.steps * 1e3, solved / (p * args.steps), \
            {kc: ms / max(c, 1) for kc, (ms, c) in kt.items()}, fl

    base = dict(max_iter=args.max_iter, tol=1e-4, fp64_polish=args.polish)
    v, ms, sf, kms, fl = timed(blocks=J, draws=ud, polish_after=cap, **base)
    v1, ms1, sf1, kms1, _ = timed(blocks=1, draws=ud, polish_after=args.polish_after, **base)
    vm, msm, sfm, kmsm, _ = timed(polish_after=args.polish_after, **base)
    it_s = kms["iteration"] / 1e3
    print(json.dumps({
        "metric": METRIC, "value": v, "unit": "pixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc + f"; Algorithm 1 with J={J} column blocks", "blocks": J,
                   "block_iterations_before_fp64": cap, "solved_fraction": sf, "kernel_ms": kms,
                   "iteration_tflops": fl / it_s / 1e12 if it_s > 0 else None},
        "compare": {"one_block_same_kernel": {"value": v1, "ms_per_step": ms1, "solved_fraction": sf1,
                                              "kernel_ms": kms1},
                    "one_block_mfma_solver": {"value": vm, "ms_per_step": msm, "solved_fraction": sfm,
                                              "kernel_ms": kmsm}}}), flush=True)


def bench_unrolled(args):
    """Differentiation through K = 200 unrolled fixed-step iterations (N=25, L=256,
    P=2^18, checkpoints every 20): forward + hand-written adjoint per step."""
    import torch
    from paper_1805_01759_amd import synth
    from paper_1805_01759_amd.unrolled import unrolled
    p = args.pixels or (1 << 18)
    spec, geom, B, lam, meta = synth.make_config(5, 0, p, with_meta=True)
    Xt = synth.xtrue(spec, geom, meta)
    A = geom.A
    alpha = 1.0 / (2 * np.linalg.eigvalsh(A @ A.conj().T).max())
    dev = torch.device("cuda:0")
    Bd = torch.from_numpy(B.astype(np.complex64)).to(dev)
    Xtd = torch.from_numpy(Xt.astype(np.complex64)).to(dev)
    xi = torch.tensor(geom.xi, dtype=torch.float32, device=dev)
    s = torch.tensor(geom.s, dtype=torch.float32, device=dev)
    lam_t = torch.tensor(float(lam[0]), dtype=torch.float32, device=dev)

    def step():
        b = Bd.clone().requires_grad_(True)
        lt = lam_t.clone().requires_grad_(True)
        xg = xi.clone().requires_grad_(True)
        X = unrolled(b, lt, xg, s, alpha, 200, 20)
        loss = (X - Xtd).abs().pow(2).sum()
        loss.backward()
        return xg.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the plain FP32 solver on the same stack (tol 1e-4, FP64 refinement)
    from paper_1805_01759_amd import api
    Ad = torch.from_numpy(A.astype(np.complex64)).to(dev)
    ld = torch.full((p,), float(lam[0]), dtype=torch.float32, device=dev)
    Xs = torch.empty((p, A.shape[1]), dtype=torch.complex64, device=dev)
    wsp = api.Workspace()
    api.solve(Ad, Bd, ld, out=Xs, workspace=wsp, polish_after=args.polish_after)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        _, d = api.solve(Ad, Bd, ld, out=Xs, workspace=wsp, polish_after=args.polish_after)
    torch.cuda.synchronize()
    o_dt = time.perf_counter() - t1
    o_solved = int(((d["status"] & 1) != 0).sum().item())
    n, l = A.shape
    flops = 200 * 64.0 * n * l * p  # forward 16NL + recompute 16NL + reverse 32NL per iteration
    print(json.dumps({"metric": "pixel-gradients/s through 200 unrolled iterations",
                      "value": p * args.steps / dt, "unit": "pixels/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": f"unrolled map N={n}, L={l}, P={p}, K=200, ckpt 20",
                                 "useful_tflops": flops * args.steps / dt / 1e12},
                      "compare": {"form": "plain FP32 solve of the same stack to KKT 1e-4",
                                  "value": p * args.steps / o_dt, "unit": "pixels/s",
                                  "solved_fraction": o_solved / p,
                                  "ms_per_step": o_dt / args.steps * 1e3}}), flush=True)


def run_precision(api, Ad, Bd, ld, X, ws, n, l, p, prec, steps, warmup, args, sample_idx,
                  keep_x=False):
    """Time `steps` solves at one contraction precision; returns the throughput,
    event-timed kernel averages, the kernels' counters and the sampled rows of
    the last solve (x and the CONVERGED bit) for the parity report."""
    import torch
    opts = dict(max_iter=args.max_iter, tol=1e-4, precision=prec, fp64_polish=args.polish,
                polish_after=args.polish_after, fp64_continue=args.fp64_continue,
                iteration_kernel=("auto" if prec != "fp32" and args.iteration_kernel == "wave"
                                  else args.iteration_kernel))
    for _ in range(warmup):
        api.solve(Ad, Bd, ld, out=X, workspace=ws, **opts)
    torch.cuda.synchronize()
    api.timing_enable(True)
    for kc in ("iteration", "refine", "certify"):
        api.timing_read(kc)
    statuses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, d = api.solve(Ad, Bd, ld, out=X, workspace=ws, **opts)
        statuses.append(d["status"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = {kc: api.timing_read(kc) for kc in ("iteration", "refine", "certify")}
    api.timing_enable(False)
    solved = sum(int(((st & 1) != 0).sum().item()) for st in statuses)
    cnt = api.solve_counters(n, l, p, d)
    fwd, adj, npol, f64 = cnt[:4]
    f32 = cnt[4] if len(cnt) > 4 else 0
    avg_s = {kc: (ms / max(c, 1)) / 1e3 for kc, (ms, c) in kt.items()}
    ti = torch.from_numpy(sample_idx).to(X.device)
    xs = X[ti].cpu().numpy()
    x_host = X.cpu().numpy() if keep_x else None
    conv = ((d["status"][ti] & 1) != 0).cpu().numpy()
    return {"value": solved / dt, "ms_per_step": dt / steps * 1e3,
            "solved_fraction": solved / (p * steps), "avg_s": avg_s,
            "fwd": fwd, "adj": adj, "npol": npol, "f64": f64, "f32": f32, "xs": xs, "conv": conv,
            "X_host": x_host}


def algorithm1_only(api, Ad, Bd, ld, X, n, l, args):
    """One FP32 solve by Algorithm 1 alone (fp64_polish = 0, max_iter iterations)."""
    import torch
    p = Bd.shape[0]
    ws = api.Workspace()
    opts = dict(max_iter=args.max_iter, tol=1e-4, precision="fp32", fp64_polish=0, polish_after=0)
    api.timing_enable(True)
    for kc in ("iteration", "refine", "certify"):
        api.timing_read(kc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, d = api.solve(Ad, Bd.contiguous(), ld.contiguous(), out=X, workspace=ws, **opts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    it_ms, _ = api.timing_read("iteration")
    api.timing_enable(False)
    solved = int(((d["status"] & 1) != 0).sum().item())
    iters = d["iters"].float()
    return {"pixels": p, "value": solved / dt, "unit": "pixels/s", "solved_fraction": solved / p,
            "ms": dt * 1e3, "iteration_ms": it_ms, "mean_iterations": float(iters.mean().item()),
            "max_iter": args.max_iter,
            "note": "Algorithm 1 in FP32 on the MFMA kernel, no FP64 refinement; FP64 certificate"}


def rooflines(r, n, l, prec, workload, polish, kernel="auto"):
    """Roofline objects of the iteration and refinement kernels of one run."""
    avg_s = r["avg_s"]
    if prec != "fp32":
        # split-BF16: the automatic choice as in FP32 (the streamed tile beyond 384 bins)
        stream = kernel == "stream" or (kernel != "mfma" and not (n <= 64 and l <= 384))
        it_kernel = "fista_stream_kernel_bf16" if stream else "fista_mfma_kernel_bf16"
    elif kernel != "auto":
        it_kernel = f"fista_{kernel}_kernel"
    elif n <= 64 and l <= 384:
        it_kernel = "fista_mfma_kernel"
    else:
        # the automatic FP32 choice beyond 384 bins: the streamed MFMA tile
        it_kernel = "fista_stream_kernel"
    # iteration kernel: algorithmic flops = (forward + adjoint products) x 8 N L
    it_flops = (r["fwd"] + r["adj"]) * 8.0 * n * l
    it_ach = it_flops / avg_s["iteration"]
    peak = PEAK[prec] if it_kernel != "fista_wave_kernel" else PEAK_FP32_VALU
    roof_it = {"bound": "mfma" if it_kernel != "fista_wave_kernel" else "alu",
               "achieved": it_ach / 1e12, "peak": peak / 1e12,
               "unit": "TFLOP/s", "frac": it_ach / peak,
               "traffic": load_traffic(it_kernel, workload), "kernel": it_kernel,
               "kernel_ms": avg_s["iteration"] * 1e3, "flops_per_launch": it_flops}
    roof_rf = None
    if polish and avg_s["refine"] > 0:
        # FP64 refinement: plain vector arithmetic, FP64 and (mode 1's round-end
        # gradient) FP32 flops counted by the kernel; the peak is the rate at which
        # this mix would run with each part at its own vector peak
        fl = float(r["f64"] + r["f32"])
        t_peak = r["f64"] / PEAK_FP64_VALU + r["f32"] / PEAK_FP32_VALU
        mix_peak = fl / t_peak if t_peak > 0 else PEAK_FP64_VALU
        rf_ach = fl / avg_s["refine"]
        roof_rf = {"bound": "alu", "achieved": rf_ach / 1e12, "peak": mix_peak / 1e12,
                   "unit": "TFLOP/s", "frac": rf_ach / mix_peak,
                   "traffic": load_traffic("polish_kernel", workload), "kernel": "polish_kernel",
                   "kernel_ms": avg_s["refine"] * 1e3, "flops_per_launch": fl,
                   "fp64_flops_per_launch": float(r["f64"]), "fp32_flops_per_launch": float(r["f32"])}
    return roof_it, roof_rf


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="pairs", choices=sorted(WORKLOADS) + ["unrolled", "batched", "blocks"])
    ap.add_argument("--blocks", type=int, default=4, help="J for --workload blocks")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "split_bf16"],
                    help="the precision reported as value; the other one is timed beside it")
    ap.add_argument("--compare-steps", type=int, default=5,
                    help="timed steps of the other precision (at most --steps)")
    ap.add_argument("--max-iter", type=int, default=500)
    ap.add_argument("--polish-after", type=int, default=0,
                    help="FP32 iterations before the FP64 stage (0: the workload's default)")
    ap.add_argument("--polish", type=int, default=ACCURACY_MODE,
                    help="fp64_polish: 1 refine pixels above tol, 2 every pixel to FP64 accuracy")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle pixels timed for cpu_baseline (0: the workload's default)")
    ap.add_argument("--parity-sample", type=int, default=-1,
                    help="pixels of the parity report (-1: the workload's default, 0: none)")
    ap.add_argument("--pixels", type=int, default=0, help="override the pixel count (tests only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iteration-kernel", default="auto", choices=["auto", "mfma", "wave", "stream"],
                    help="kernel of the FP32 iterations (auto: the register tile where it exists, "
                         "else the streamed tile)")
    ap.add_argument("--no-fp64-continue", dest="fp64_continue", action="store_false",
                    help="return the pixels the 32-slot refinement leaves above tol unsolved instead of "
                         "continuing Algorithm 1 in FP64")
    ap.add_argument("--alg1-pixels", type=int, default=1 << 20,
                    help="pixels of the Algorithm-1-only leg (0: skip it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.polish_after <= 0:
        args.polish_after = polish_after_for(args.workload)
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path (pixels are "
              "independent problems, so a stack would shard by pixel range with a copy of A "
              "on every GPU). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4}))
        return
    from paper_1805_01759_amd import api, synth

    if args.workload == "unrolled":
        return bench_unrolled(args)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "blocks":
        return bench_blocks(args)
    cfg, desc = WORKLOADS[args.workload]
    sr_meta = None
    if args.workload == "superres":
        reps = args.pixels // len(synth.SUPERRES_CASES) if args.pixels else SUPERRES_REALISATIONS
        geom, B, lam, sr_meta = synth.make_superres(max(reps, 1))
    elif cfg in synth.MOTION_SPECS:
        spec, geom, B, lam = synth.make_motion_config(cfg, 0, args.pixels or None)
    else:
        spec, geom, B, lam = synth.make_config(cfg, 0, args.pixels or None)
    A32, B32, l32 = synth.to_device_dtypes(geom.A, B, lam)
    del B
    dev = torch.device("cuda:0")
    Ad = torch.from_numpy(A32).to(dev)
    Bd = torch.from_numpy(B32).to(dev)
    ld = torch.from_numpy(l32).to(dev)
    n, l = A32.shape
    p = B32.shape[0]
    X = torch.empty((p, l), dtype=torch.complex64, device=dev)
    ws = api.Workspace()
    ps = PARITY_SAMPLE.get(args.workload, 512) if args.parity_sample < 0 else args.parity_sample
    ps = min(ps, p)
    sample_idx = (np.arange(ps, dtype=np.int64) * p) // max(ps, 1) + (p // max(ps, 1)) // 2 \
        if ps else np.zeros(0, np.int64)
    other = "split_bf16" if args.precision == "fp32" else "fp32"
    if args.precision == "split_bf16" and args.iteration_kernel == "wave":
        sys.exit("split-BF16 runs on the MFMA tiles only (not the wave-per-pixel kernel)")
    runs = {args.precision: run_precision(api, Ad, Bd, ld, X, ws, n, l, p, args.precision,
                                          args.steps, args.warmup, args, sample_idx,
                                          keep_x=sr_meta is not None)}
    if other:
        runs[other] = run_precision(api, Ad, Bd, ld, X, ws, n, l, p, other,
                                    max(1, min(args.steps, args.compare_steps)),
                                    min(args.warmup, 1), args, sample_idx)
    r = runs[args.precision]
    roof_it, roof_rf = rooflines(r, n, l, args.precision, args.workload, args.polish, args.iteration_kernel)
    # the dominant kernel by event-timed duration
    roof = roof_rf if roof_rf is not None and r["avg_s"]["refine"] > r["avg_s"]["iteration"] else roof_it
    rec = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": desc if not args.pixels else desc + f" (first {p} pixels)", "n": n, "l": l,
                   "pixels": p, "max_iter": args.max_iter, "tol": 1e-4, "precision": args.precision,
                   "polish_after": args.polish_after, "fp64_polish": args.polish,
                   "fp64_continue": int(args.fp64_continue),
                   "iteration_kernel": args.iteration_kernel,
                   "solved_fraction": r["solved_fraction"], "pixels_refined_fp64": r["npol"],
                   "kernel_ms": {kc: v * 1e3 for kc, v in r["avg_s"].items()}},
        "roofline": roof,
    }
    rec["roofline_iteration" if roof is not roof_it else "roofline_refine"] = \
        roof_it if roof is not roof_it else roof_rf
    if sr_meta is not None:
        # detection rate of the pair per case, from the primary precision's last solve
        from paper_1805_01759_amd import detect
        Xh = runs[args.precision]["X_host"]
        rates = []
        for c, (kind, kappa, snr) in enumerate(synth.SUPERRES_CASES):
            sl = sr_meta["case"] == c
            rates.append({"set": kind, "kappa": kappa, "snr_db": snr,
                          "detection_rate": detect.detection_rate(Xh[sl], geom.s, sr_meta["s1"][sl],
                                                                  sr_meta["s2"][sl], geom.rayleigh)})
        rec["config"]["detection"] = {"rule": "two clusters of adjacent nonzero bins, one each side of "
                                              "the pair's midpoint, within rho_s/2 of the truth, the "
                                              "lighter >= 10% of the heavier (the package's own rule)",
                                      "cases": rates}
    if other:
        o = runs[other]
        o_it, o_rf = rooflines(o, n, l, other, args.workload, args.polish,
                               "auto" if other != "fp32" and args.iteration_kernel == "wave"
                               else args.iteration_kernel)
        rec["compare"] = {"precision": other, "value": o["value"], "unit": "pixels/s",
                          "steps": max(1, min(args.steps, args.compare_steps)),
                          "ms_per_step": o["ms_per_step"], "solved_fraction": o["solved_fraction"],
                          "kernel_ms": {kc: v * 1e3 for kc, v in o["avg_s"].items()},
                          "roofline_iteration": o_it, "roofline_refine": o_rf}
    else:
        rec["compare"] = {"precision": "split_bf16", "value": None,
                          "note": f"not available at n = {n}, l = {l}: split-BF16 runs in the MFMA "
                                  f"kernels only (n <= 64, l <= 512)"}
    # Algorithm 1 alone (FP32, up to max_iter iterations, no FP64 refinement; the
    # certificate still decides "solved") on the first pixels, for context: the
    # value above comes from a short Algorithm 1 stage plus the FP64 refinement
    if args.alg1_pixels > 0:
        p1 = min(p, args.alg1_pixels)
        rec["algorithm1_only"] = algorithm1_only(api, Ad[:], Bd[:p1], ld[:p1], X[:p1], n, l, args)
    # the oracle leg (after all GPU timing): Algorithm 1 timed on the host cores,
    # and the certified minimisers of the parity sample
    if not args.no_cpu_baseline:
        sample = args.cpu_sample if args.cpu_sample else CPU_SAMPLE.get(args.workload, 1024)
        rec["cpu_baseline"] = cpu_baseline(A32, B32, l32, min(sample, p), args.max_iter, 1e-4)
    if ps:
        sol = oracle_minimisers(A32, B32, l32, sample_idx)
        rec["parity"] = {prec: parity_report(sol, runs[prec]["xs"], runs[prec]["conv"],
                                             PARITY_BAR[prec]) for prec in runs}
        rec["parity"]["metric"] = ("e_p = ||x - x*|| / max(||x*||, ||b||/sigma_max) against "
                                   "the certified FP64 minimiser; pass = e_p <= bar and FP64 "
                                   "KKT <= 1e-4; pixels strided over the whole stack")
        rec["parity"]["oracle_certificate"] = {"kkt_sub_max": sol["certified_kkt_max"],
                                               "gap_max": sol["gap_max"],
                                               "seconds": sol["seconds"]}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
