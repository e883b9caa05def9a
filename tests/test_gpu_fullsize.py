"""Parity at the benchmark's full sizes and launch configurations, on sampled
outputs the oracle computes one by one.

Scene (2^20 pixels) and close pairs (2^22 pixels) are solved exactly as bench.py
times them (FP64 stage after bench.POLISH_AFTER FP32 iterations), in both
contraction precisions; the 64 uneven stacks through one plan; the unrolled
map at 2^18 pixels, K = 200, checkpoints every 20.  Each sampled pixel is
checked against the certified minimiser (solves: its KKT certificate and
objective, the unique parts of a result whose x is any point with KKT <= tol)
or the FP64 reference map and its gradient (unrolled: per-pixel outputs depend
on that pixel alone); the pixel-summed gradients are checked through their
additivity over a split of the pixel set.
"""
import numpy as np
import pytest
import torch

import bench
from paper_1805_01759_amd import _lib, api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch.device("cuda:0")


def _rel_err(X, Xe, B, Lf):
    den = np.maximum(np.linalg.norm(Xe, axis=1), np.linalg.norm(B, axis=1) / np.sqrt(Lf / 2))
    return np.linalg.norm(X - Xe, axis=1) / den


def _check_sampled(orc, A32, B32, l32, X, d, idx, bar, min_solved=0.9999, median_e=1e-5,
                   pass_floor=None):
    """What is unique in the result is checked exactly: the certified KKT residual
    of the returned x (device vs oracle) and its objective against the minimiser's
    (relative gap within bar, never below the minimum beyond rounding).  The
    distance to the minimiser, e_p = ||x - x*|| / max(||x*||, ||b|| / sigma_max),
    is reported and its pass fraction (e_p <= bar and solved) held to
    `pass_floor`: for near-adjacent bins the minimiser is ill-conditioned, so a
    KKT residual at tol does not bound e_p; the solves here refine every pixel to
    FP64 accuracy (the benchmark's mode), which does for all but a few pixels."""
    A64 = A32.astype(np.complex128)
    Lf = orc.lipschitz(A64)
    Bs = B32[idx].astype(np.complex128)
    ls = l32[idx].astype(np.float64)
    Xe, de = orc.exact_batch(A64, Bs, ls)
    it = torch.from_numpy(idx).to(X.device)
    Xg = X[it].cpu().numpy().astype(np.complex128)
    kg = d["kkt"][it].cpu().numpy()
    ko = np.array([orc.kkt_nat(A64, Bs[k], ls[k], Xg[k], Lf) for k in range(len(idx))])
    Fg = np.array([orc.objective(A64, Bs[k], ls[k], Xg[k]) for k in range(len(idx))])
    Fe = np.array([orc.objective(A64, Bs[k], ls[k], Xe[k]) for k in range(len(idx))])
    gap = (Fg - Fe) / np.maximum(Fe, 1e-30)
    e = _rel_err(Xg, Xe, Bs, Lf)
    st = d["status"].cpu().numpy()
    conv = (st & _lib.PX_CONVERGED) != 0
    passed = conv[idx] & (e <= bar)
    print(f"solved {conv.mean():.6f}; sampled objective gap max {gap.max():.1e}; kkt max {ko.max():.1e}; "
          f"x vs minimiser: e p50 {np.median(e):.1e}, p99 {np.percentile(e, 99):.1e}, max {e.max():.1e}; "
          f"parity pass {passed.mean():.4f} at bar {bar:g}")
    assert conv.mean() >= min_solved
    assert np.allclose(kg, ko, rtol=1e-5, atol=1e-9)
    assert (ko[conv[idx]] <= 1e-4 * (1 + 1e-5)).all()
    assert gap.min() >= -1e-12 and gap.max() <= bar
    if median_e is not None:
        assert np.median(e) <= median_e
    if pass_floor is not None:
        assert passed.mean() >= pass_floor
    return e, passed


# pass-fraction floors of e_p <= bar (and solved) on the sampled pixels, in the
# benchmark's configuration; measured: scene 0.98 / 0.99, close pairs 0.98 / 0.996
@pytest.mark.parametrize("prec,bar,floor", [("fp32", 1e-4, 0.95), ("split_bf16", 1e-3, 0.95)])
def test_scene_full_size(dev, orc, prec, bar, floor):
    spec, geom, B, lam = synth.make_config(2)
    A32, B32, l32 = synth.to_device_dtypes(geom.A, B, lam)
    Ad, Bd, ld = (torch.from_numpy(x).to(dev) for x in (A32, B32, l32))
    X, d = api.solve(Ad, Bd, ld, tol=1e-4, max_iter=500, precision=prec, fp64_polish=bench.ACCURACY_MODE,
                     polish_after=bench.POLISH_AFTER)
    p = B32.shape[0]
    idx = np.arange(7, p, p // 256)
    _check_sampled(orc, A32, B32, l32, X, d, idx, bar, pass_floor=floor)


@pytest.mark.parametrize("prec,bar,floor", [("fp32", 1e-4, 0.95), ("split_bf16", 1e-3, 0.95)])
def test_close_pairs_full_size(dev, orc, prec, bar, floor):
    spec, geom, B, lam = synth.make_config(4)
    A32, B32, l32 = synth.to_device_dtypes(geom.A, B, lam)
    del B
    Ad, Bd, ld = (torch.from_numpy(x).to(dev) for x in (A32, B32, l32))
    X, d = api.solve(Ad, Bd, ld, tol=1e-4, max_iter=500, precision=prec, fp64_polish=bench.ACCURACY_MODE,
                     polish_after=bench.polish_after_for("pairs"))
    p = B32.shape[0]
    idx = np.arange(11, p, p // 192)
    _check_sampled(orc, A32, B32, l32, X, d, idx, bar, pass_floor=floor)


def test_batched_full_size(dev, orc):
    specs = synth.batched_specs(64)
    stacks, host = [], []
    for ss in specs:
        spec, geom, B, lam = synth.make_batched_stack(ss)
        A32, B32, l32 = synth.to_device_dtypes(geom.A, B, lam)
        host.append((A32, B32, l32))
        stacks.append({"A": torch.from_numpy(A32).to(dev), "B": torch.from_numpy(B32).to(dev),
                       "lam": torch.from_numpy(l32).to(dev),
                       "X": torch.empty((ss.p, ss.l), dtype=torch.complex64, device=dev),
                       "diag": api.new_diag(ss.p, dev)})
    plan = api.Plan([(ss.n, ss.l, ss.p) for ss in specs], max_iter=500, tol=1e-4,
                    fp64_polish=bench.ACCURACY_MODE, polish_after=bench.POLISH_AFTER)
    ws = torch.empty(plan.workspace_bytes + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    plan.execute(stacks, ws[off:off + plan.workspace_bytes])
    torch.cuda.synchronize()
    all_pass = []
    for (A32, B32, l32), st in zip(host, stacks):
        p = B32.shape[0]
        idx = np.unique(np.array([0, p // 3, (2 * p) // 3, p - 1]))
        # grids of up to 1024 bins over 100 m: the minimiser's distance is not
        # bounded by the certificate (reported, not asserted)
        _, passed = _check_sampled(orc, A32, B32, l32, st["X"], st["diag"], idx, 1e-4, min_solved=0.999,
                                   median_e=None)
        all_pass.append(passed)
    passed = np.concatenate(all_pass)
    print(f"batched: parity pass over {len(passed)} sampled pixels of 64 stacks: {passed.mean():.4f}")
    assert passed.mean() >= 0.9


def test_unrolled_full_size(dev, orc):
    from oracle import unrolled_ref
    from paper_1805_01759_amd.unrolled import unrolled
    p, K = 1 << 18, 200
    spec, geom, B, lam, meta = synth.make_config(5, 0, p, with_meta=True)
    Xt = synth.xtrue(spec, geom, meta)
    A = geom.A
    alpha = 1.0 / (2 * np.linalg.eigvalsh(A @ A.conj().T).max())
    lam0 = float(np.float32(lam[0]))
    B64 = B.astype(np.complex64).astype(np.complex128)
    xi = torch.tensor(geom.xi, dtype=torch.float32)
    s = torch.tensor(geom.s, dtype=torch.float32)

    def run(rows):
        Bd = torch.from_numpy(B64[rows].astype(np.complex64)).to(dev).requires_grad_(True)
        lt = torch.tensor(lam0, dtype=torch.float32, device=dev, requires_grad=True)
        xg = xi.to(dev).requires_grad_(True)
        X = unrolled(Bd, lt, xg, s.to(dev), alpha, K, 20)
        Xtd = torch.from_numpy(Xt[rows].astype(np.complex64)).to(dev)
        (X - Xtd).abs().pow(2).sum().backward()
        return X.detach(), Bd.grad, lt.grad.item(), xg.grad.double().cpu().numpy()

    X, gB, glam, gxi = run(slice(0, p))
    idx = np.arange(5, p, p // 16)
    # per-pixel outputs against the FP64 references on the sampled pixels alone
    A64 = np.exp(-2j * np.pi * np.outer(xi.double().numpy(), s.double().numpy()))
    Xo = orc.unrolled_batch(A64, B64[idx], lam0, alpha, K)
    Xg = X[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.complex128)
    e = np.linalg.norm(Xg - Xo, axis=1) / np.maximum(np.linalg.norm(Xo, axis=1), 1e-3)
    _, _, dB, _, _ = unrolled_ref.loss_and_grads(xi.double(), s.double(), torch.from_numpy(B64[idx]),
                                                 lam0, alpha, K, torch.from_numpy(Xt[idx]))
    gBs = gB[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.complex128)
    eB = np.linalg.norm(gBs - dB.numpy(), axis=1) / np.maximum(np.linalg.norm(dB.numpy(), axis=1), 1e-6)
    # the pixel-summed gradients are additive over a split of the pixels
    h = p // 2
    _, _, gl1, gx1 = run(slice(0, h))
    _, _, gl2, gx2 = run(slice(h, p))
    el = abs(gl1 + gl2 - glam) / abs(glam)
    ex = np.linalg.norm(gx1 + gx2 - gxi) / np.linalg.norm(gxi)
    print(f"unrolled full size: X e max {e.max():.1e}; dB e max {eB.max():.1e}; "
          f"additivity dlambda {el:.1e} dxi {ex:.1e}")
    assert e.max() < 1e-4
    assert eB.max() < 1e-4
    assert el < 1e-4 and ex < 1e-4
