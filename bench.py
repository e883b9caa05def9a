#!/usr/bin/env python
"""Throughput of the gfx950 L1LS solver: pixels solved per second at KKT <= 1e-4.

One step = one full solve (setup, accelerated proximal-gradient iteration,
FP64 refinement, FP64 optimality check) of a synthetic scene-scale TomoSAR
stack already resident in HBM: N = 25 acquisitions, L = 256 elevation bins,
P = 2^20 pixels, max 500 iterations, tol 1e-4.  Prints one JSON line.
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
}


# sources of each timed kernel; a traffic record is used only while they are unchanged
KERNEL_SOURCES = {
    "fista_mfma_kernel": ("fista_mfma.h", "fista.hip"),
    "fista_mfma_kernel_bf16": ("fista_mfma.h", "fista.hip"),
    "fista_kernel": ("fista_impl.h", "fista.hip"),
    "polish_kernel": ("polish.hip", "wave_reduce.h"),
    "certify_kernel": ("certify.hip", "wave_reduce.h"),
}
PEAK_FP64_VALU = 78.6e12   # MI355X FP64 vector FLOP/s
POLISH_AFTER = 12          # FP32 iterations before a pixel goes to the FP64 stage


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
            "sample": f"first {sample} pixels of the same stack; Algorithm 1 (J=1) in FP64, "
                      f"tol {tol}, max {max_iter} iterations; {solved} solved in {dt:.1f} s"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scene", choices=sorted(WORKLOADS) + ["unrolled", "batched", "blocks"])
    ap.add_argument("--blocks", type=int, default=4, help="J for --workload blocks")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "split_bf16"])
    ap.add_argument("--max-iter", type=int, default=500)
    ap.add_argument("--polish-after", type=int, default=POLISH_AFTER)
    ap.add_argument("--polish", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle pixels timed for cpu_baseline (0: 16384 at N L = 25 x 256, scaled by 1/(N L))")
    ap.add_argument("--pixels", type=int, default=0, help="override the pixel count (tests only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path (pixels are "
              "independent; see the sharding note in DESIGN.md). Run with --gpus 1.",
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
    if cfg in synth.MOTION_SPECS:
        spec, geom, B, lam = synth.make_motion_config(cfg, 0, args.pixels or None)
    else:
        spec, geom, B, lam = synth.make_config(cfg, 0, args.pixels or None)
    A32, B32, l32 = synth.to_device_dtypes(geom.A, B, lam)
    dev = torch.device("cuda:0")
    Ad = torch.from_numpy(A32).to(dev)
    Bd = torch.from_numpy(B32).to(dev)
    ld = torch.from_numpy(l32).to(dev)
    n, l = A32.shape
    p = B32.shape[0]
    opts = dict(max_iter=args.max_iter, tol=1e-4, precision=args.precision,
                fp64_polish=args.polish, polish_after=args.polish_after)
    X = torch.empty((p, l), dtype=torch.complex64, device=dev)
    ws = api.Workspace()
    for _ in range(args.warmup):
        api.solve(Ad, Bd, ld, out=X, workspace=ws, **opts)
    torch.cuda.synchronize()
    api.timing_enable(True)
    for kc in ("iteration", "refine", "certify"):
        api.timing_read(kc)
    diags = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, d = api.solve(Ad, Bd, ld, out=X, workspace=ws, **opts)
        diags.append(d["status"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = {kc: api.timing_read(kc) for kc in ("iteration", "refine", "certify")}
    api.timing_enable(False)
    solved = sum(int(((s & 1) != 0).sum().item()) for s in diags)
    fwd, adj, npol, pflops = api.solve_counters(n, l, p, d)
    avg_s = {kc: (ms / max(c, 1)) / 1e3 for kc, (ms, c) in kt.items()}
    # iteration kernel: algorithmic flops = (forward + adjoint products) x 8 N L
    if n <= 64 and l <= 512:
        it_kernel = "fista_mfma_kernel" if args.precision == "fp32" else "fista_mfma_kernel_bf16"
    else:
        it_kernel = "fista_wave_kernel"
    it_flops = (fwd + adj) * 8.0 * n * l
    it_ach = it_flops / avg_s["iteration"]
    roof_it = {"bound": "mfma", "achieved": it_ach / 1e12, "peak": PEAK[args.precision] / 1e12,
               "unit": "TFLOP/s", "frac": it_ach / PEAK[args.precision],
               "traffic": load_traffic(it_kernel, args.workload), "kernel": it_kernel,
               "kernel_ms": avg_s["iteration"] * 1e3, "flops_per_launch": it_flops}
    roof = roof_it
    if args.polish and avg_s["refine"] > 0:
        # FP64 refinement: plain FP64 VALU arithmetic, flops counted by the kernel
        rf_ach = pflops / avg_s["refine"]
        roof_rf = {"bound": "alu", "achieved": rf_ach / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                   "unit": "TFLOP/s", "frac": rf_ach / PEAK_FP64_VALU,
                   "traffic": load_traffic("polish_kernel", args.workload), "kernel": "polish_kernel",
                   "kernel_ms": avg_s["refine"] * 1e3, "flops_per_launch": float(pflops)}
        if avg_s["refine"] > avg_s["iteration"]:
            roof = roof_rf
    rec = {
        "metric": METRIC,
        "value": solved / dt,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": desc if not args.pixels else desc + f" (first {p} pixels)", "n": n, "l": l, "pixels": p, "max_iter": args.max_iter,
                   "tol": 1e-4, "precision": args.precision, "polish_after": args.polish_after,
                   "solved_fraction": solved / (p * args.steps), "pixels_refined_fp64": npol,
                   "kernel_ms": {kc: avg_s[kc] * 1e3 for kc in avg_s}},
        # dominant kernel by event-timed duration
        "roofline": roof,
    }
    if roof is not roof_it:
        rec["roofline_iteration"] = roof_it
    elif args.polish and avg_s["refine"] > 0:
        rec["roofline_refine"] = roof_rf
    # the metric compares the two contraction precisions: time the other one on the
    # same stack and steps
    other = "split_bf16" if args.precision == "fp32" else "fp32"
    o_opts = dict(opts, precision=other)
    for _ in range(args.warmup):
        api.solve(Ad, Bd, ld, out=X, workspace=ws, **o_opts)
    api.timing_enable(True)
    for kc in ("iteration", "refine", "certify"):
        api.timing_read(kc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    o_diags = []
    for _ in range(args.steps):
        _, d2 = api.solve(Ad, Bd, ld, out=X, workspace=ws, **o_opts)
        o_diags.append(d2["status"])
    torch.cuda.synchronize()
    o_dt = time.perf_counter() - t0
    o_kt = {kc: api.timing_read(kc) for kc in ("iteration", "refine", "certify")}
    api.timing_enable(False)
    o_solved = sum(int(((st & 1) != 0).sum().item()) for st in o_diags)
    rec["compare"] = {"precision": other, "value": o_solved / o_dt, "unit": "pixels/s",
                      "ms_per_step": o_dt / args.steps * 1e3,
                      "solved_fraction": o_solved / (p * args.steps),
                      "kernel_ms": {kc: (ms / max(c, 1)) for kc, (ms, c) in o_kt.items()}}
    if not args.no_cpu_baseline:
        # about 10-30 s of oracle work: fewer pixels where a pixel costs more
        sample = args.cpu_sample if args.cpu_sample else max(1024, (16384 * 25 * 256) // (n * l))
        rec["cpu_baseline"] = cpu_baseline(A32, B32, l32, min(sample, p), args.max_iter, 1e-4)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
