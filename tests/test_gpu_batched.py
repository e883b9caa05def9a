"""Batched uneven stacks (plan + HIP graph) and the wave-per-pixel kernel for
shapes beyond the register-resident MFMA tiles, against the FP64 oracle."""
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


@pytest.mark.parametrize("n,l,p", [(100, 1024, 24), (80, 300, 40), (128, 64, 20), (11, 700, 33)])
def test_large_shapes(dev, orc, n, l, p):
    ss = synth.StackSpec(90 + n % 7, n, l, p)
    A, B, lam = _stack(ss)
    Ad, Bd, ld = (torch.from_numpy(x).to(dev) for x in (A, B, lam))
    X, d = api.solve(Ad, Bd, ld, fp64_polish=2, polish_after=100)
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


def test_plan_matches_single_solves_and_graph_replay(dev):
    specs = [s for s in synth.batched_specs(64, scale=0.01)][:12]
    plan = api.Plan([(s.n, s.l, s.p) for s in specs], fp64_polish=1, polish_after=50)
    print(plan.describe())
    stacks = _plan_inputs(dev, specs)
    ws = torch.empty(plan.workspace_bytes + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + plan.workspace_bytes]
    plan.execute(stacks, ws)
    torch.cuda.synchronize()
    eager = [st["X"].clone() for st in stacks]
    # every stack equals a single-stack solve with the kernel the plan chose
    for st, ss in zip(stacks, specs):
        conv = (st["diag"]["status"].cpu().numpy() & _lib.PX_CONVERGED) != 0
        assert conv.mean() >= 0.99
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
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device=dev).sum()  # unrelated eager work
        for st, ref in zip(stacks, eager):
            assert torch.equal(st["X"], ref), f"replay {rep} differs"
