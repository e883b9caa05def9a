"""Batched uneven stacks (plan + HIP graph), and the streamed MFMA tile and the
wave-per-pixel kernel for shapes beyond the register-resident MFMA tiles, against
the FP64 oracle."""
import numpy as np
import pytest
import torch

from paper_1805_01759_amd import _lib, api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch.device("cuda:0")


def _stack(ss):
    spec, geom, B, lam = synth.make_batched_stack(ss)
    return synth.to_device_dtypes(geom.A, B, lam)


@pytest.mark.parametrize("kernel,precision", [("auto", "fp32"), ("wave", "fp32"), ("auto", "split_bf16")])
@pytest.mark.parametrize("n,l,p", [(100, 1024, 24), (80, 300, 40), (128, 64, 20), (11, 700, 33)])
def test_large_shapes(dev, orc, n, l, p, kernel, precision):
    ss = synth.StackSpec(90 + n % 7, n, l, p)
    A, B, lam = _stack(ss)
    Ad, Bd, ld = (torch.from_numpy(x).to(dev) for x in (A, B, lam))
    X, d = api.solve(Ad, Bd, ld, fp64_polish=2, polish_after=100, iteration_kernel=kernel, precision=precision)
    A64, B64, L64 = A.astype(complex), B.astype(complex), lam.astype(float)
    Xe, de = orc.exact_batch(A64, B64, L64)
    Xg = X.cpu().numpy().astype(complex)
    Fg = np.array([orc.objective(A64, B64[i], L64[i], Xg[i]) for i in range(p)])
    gap = (Fg - de["objective"]) / np.maximum(de["objective"], 1.0)
    conv = (d["status"].cpu().numpy() & _lib.PX_CONVERGED) != 0
    assert conv.all() and gap.max() <= 1e-9, (conv.mean(), gap.max())


def _plan_inputs(dev, specs):
    stacks = []
    for ss in specs:
        A, B, lam = _stack(ss)
        stacks.append({"A": torch.from_numpy(A).to(dev), "B": torch.from_numpy(B).to(dev),
                       "lam": torch.from_numpy(lam).to(dev),
                       "X": torch.zeros((ss.p, ss.l), dtype=torch.complex64, device=dev),
                       "diag": api.new_diag(ss.p, dev), "np": (A, B, lam)})
    return stacks


def _run_plan(dev, specs, stacks, **opts):
    plan = api.Plan([(s.n, s.l, s.p) for s in specs], **opts)
    ws = torch.empty(plan.workspace_bytes + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + plan.workspace_bytes]
    plan.execute(stacks, ws)
    torch.cuda.synchronize()
    return plan, ws


def test_plan_matches_single_solves_and_graph_replay(dev, orc):
    """Twelve uneven stacks through one plan (one setup launch, one persistent iteration
    launch per tiling class, the refinement and the certificate over all stacks): every
    stack equals a plan of that stack alone bit for bit (same tiling: the autotuner's
    choice is cached), its sampled pixels match the oracle's minimiser, and graph replays
    reproduce the eager result."""
    specs = [s for s in synth.batched_specs(64, scale=0.01)][:12]
    opts = dict(fp64_polish=2, polish_after=12)
    stacks = _plan_inputs(dev, specs)
    plan, ws = _run_plan(dev, specs, stacks, **opts)
    desc = plan.describe()
    print(desc)
    eager = [st["X"].clone() for st in stacks]
    diag_eager = [{k: v.clone() for k, v in st["diag"].items()} for st in stacks]
    for i, (st, ss) in enumerate(zip(stacks, specs)):
        one = _plan_inputs(dev, [ss])
        p1, _ = _run_plan(dev, [ss], one, **opts)
        assert p1.describe().split(":", 1)[1].strip() == desc.splitlines()[i].split(":", 1)[1].strip()
        assert torch.equal(one[0]["X"], st["X"]), f"stack {i} differs from its own plan"
        for k in ("status", "iters", "kkt", "nnz"):
            assert torch.equal(one[0]["diag"][k], st["diag"][k]), (i, k)
        conv = (st["diag"]["status"].cpu().numpy() & _lib.PX_CONVERGED) != 0
        assert conv.mean() >= 0.99
        A, B, lam = st["np"]
        idx = np.unique(np.array([0, ss.p // 2, ss.p - 1]))
        A64 = A.astype(np.complex128)
        Xe, de = orc.exact_batch(A64, B[idx].astype(np.complex128), lam[idx].astype(np.float64))
        Xg = st["X"].cpu().numpy()[idx].astype(np.complex128)
        Fg = np.array([orc.objective(A64, B[k].astype(np.complex128), float(lam[k]), Xg[j])
                       for j, k in enumerate(idx)])
        gap = (Fg - de["objective"]) / np.maximum(de["objective"], 1.0)
        assert gap.max() <= 1e-9, (i, gap.max())
    # capture into a graph; replay several times with eager work in between
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for st in stacks:
            st["X"].zero_()
        with torch.cuda.graph(g, stream=s):
            plan.execute(stacks, ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for st in stacks:
            st["X"].fill_(7.0)
            st["diag"]["status"].fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device=dev).sum()  # unrelated eager work
        for st, ref, dref in zip(stacks, eager, diag_eager):
            assert torch.equal(st["X"], ref), f"replay {rep} differs"
            assert torch.equal(st["diag"]["status"], dref["status"])


TUNE_SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
from paper_1805_01759_amd import api
plan = api.Plan([(20, 200, 64), (40, 500, 64), (90, 700, 64)], fp64_polish=1)
print(plan.describe())
"""


def test_plan_tuning_cache_file(dev, tmp_path):
    """The autotuner's choices go to the cache file (one line per shape, device, precision
    and refinement mode) and a second process takes them from there."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, L1LS_TUNE_CACHE=str(cache))
    code = TUNE_SCRIPT.format(root=root)
    r1 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert r1.returncode == 0, r1.stderr
    lines = cache.read_text().split("\n")
    lines = [ln for ln in lines if ln.strip()]
    assert len(lines) == 3
    for ln, (n, l) in zip(lines, [(20, 200), (40, 500), (90, 700)]):
        f = ln.split()
        assert len(f) == 11 and (int(f[1]), int(f[2])) == (n, l) and f[4] == "1"
        assert f[5] in ("1", "2", "3")
    assert lines[2].split()[5] in ("2", "3")  # n = 90 > 64: the streamed tile or the wave kernel
    r2 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert r2.returncode == 0, r2.stderr
    assert r2.stdout == r1.stdout
    assert len([ln for ln in cache.read_text().split("\n") if ln.strip()]) == 3
