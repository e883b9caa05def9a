"""The streamed MFMA tile (iteration_kernel="stream": the register tile's FP32 or
split-BF16 contractions with each 16-pixel tile's iterates kept in the workspace),
through the C ABI: bit-identical to the register-resident tile where both exist
(384 < L <= 512, where the two split the unknowns over their four waves alike), in
both precisions; the first iterations of Algorithm 1 against the FP64 oracle at
shapes beyond the register tile (cold and warm, FP32 and split-BF16); the
hand-derived golden trajectories; and full solves with more tiles than persistent
workgroups (each workgroup's state slot reused tile after tile)."""
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


def _t(dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _stack(n, l, p, seed_cfg=9):
    # elevations over [-50, 50] m, widened beyond 1,024 bins so that the bin spacing
    # stays at the 0.1 m of the L = 1,024 grid
    half = 50.0 * max(1.0, l / 1024.0)
    geom = synth.make_geometry(seed_cfg, n, l, 250.0, -half, half)
    spec = synth.Spec(seed_cfg, n, l, p, 250.0, -half, half, "c1", 10.0)
    B, lam = synth.make_pixels(spec, geom)
    return synth.to_device_dtypes(geom.A, B, lam)


def _rel_err(X, Xe, B, Lf):
    den = np.maximum(np.linalg.norm(Xe, axis=1), np.linalg.norm(B, axis=1) / np.sqrt(Lf / 2))
    return np.linalg.norm(X - Xe, axis=1) / den


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("n,l,p", [(50, 512, 200), (40, 450, 77), (64, 400, 33), (17, 385, 50)])
@pytest.mark.parametrize("mode", ["iterations", "default", "warm"])
def test_stream_bitwise_equals_register_tile(dev, n, l, p, mode, precision):
    """Same inputs, same options: X and every diagnostic agree bit for bit."""
    A32, B32, l32 = _stack(n, l, p)
    Ad, Bd, ld = _t(dev, A32), _t(dev, B32), _t(dev, l32)
    if mode == "iterations":
        opts = dict(max_iter=40, tol=1e-30, fp64_polish=0)
    elif mode == "default":
        opts = dict(polish_after=12)
    else:
        opts = dict(max_iter=30, fp64_polish=1, warm_start=True)
    rng = np.random.default_rng(3)
    X0 = (0.1 * (rng.standard_normal((p, l)) + 1j * rng.standard_normal((p, l)))
          * (rng.random((p, l)) < 0.05)).astype(np.complex64)
    outs = []
    for kern in ("mfma", "stream"):
        X = _t(dev, X0) if mode == "warm" else None
        X, d = api.solve(Ad, Bd, ld, out=X, iteration_kernel=kern, precision=precision, **opts)
        torch.cuda.synchronize()
        outs.append((X.clone(), {k: v.clone() for k, v in d.items() if not k.startswith("_")}))
    (Xm, dm), (Xs, ds) = outs
    assert torch.equal(Xm, Xs)
    for k in ("iters", "kkt", "objective", "status", "nnz"):
        assert torch.equal(dm[k], ds[k]), k


# beyond the register tile: up to 8 row blocks, up to 1,024 bins, ragged N, L and P
BEYOND = [(100, 1024, 24), (80, 300, 40), (128, 64, 20), (11, 700, 33), (70, 1000, 17), (65, 1, 5),
          (1, 1024, 19), (120, 513, 31), (50, 2048, 24), (40, 4096, 16), (128, 3000, 9)]


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("n,l,p", BEYOND)
def test_stream_trajectory_vs_oracle(dev, orc, n, l, p, precision):
    """Five iterations of Algorithm 1 from 0: streamed tile vs FP64 oracle (split-BF16
    products carry about 2^-16 relative error each: three bf16 passes)."""
    A32, B32, l32 = _stack(n, l, p)
    l32 = np.maximum(l32, 0.5).astype(np.float32)
    X, d = api.solve(_t(dev, A32), _t(dev, B32), _t(dev, l32), max_iter=5, tol=1e-30, fp64_polish=0,
                     iteration_kernel="stream", precision=precision)
    A64, B64, L64 = A32.astype(np.complex128), B32.astype(np.complex128), l32.astype(np.float64)
    Xo, do = orc.rbpg_batch(A64, B64, L64, tol=1e-30, max_iter=5)
    e = _rel_err(X.cpu().numpy().astype(np.complex128), Xo, B64, orc.lipschitz(A64))
    med, bar = (1e-6, 1e-4) if precision == "fp32" else (3e-5, 1e-3)
    assert np.median(e) < med
    assert (e <= bar).mean() >= 0.95
    # iterations performed agree, except where the oracle's FP64 iterate lands exactly
    # on the minimiser, which its tol = 1e-30 test then reports (one of the five
    # pixels at L = 1, where one step of length 1/L_f solves the problem)
    di = d["iters"].cpu().numpy()
    differ = di != do["iters"]
    assert (do["converged"][differ] & (do["iters"][differ] < di[differ])).all()
    assert np.mean(~differ) >= (0.95 if p >= 20 else 0.8)


@pytest.mark.parametrize("n,l,p", [(100, 1024, 24), (70, 300, 40)])
def test_stream_warm_trajectory_vs_oracle(dev, orc, n, l, p):
    """Five iterations from x^(0) = the oracle's third iterate from 0 (complex64)."""
    A32, B32, l32 = _stack(n, l, p)
    A64, B64, L64 = A32.astype(np.complex128), B32.astype(np.complex128), l32.astype(np.float64)
    X3, _ = orc.rbpg_batch(A64, B64, L64, tol=1e-30, max_iter=3)
    X0 = X3.astype(np.complex64)
    X = _t(dev, X0)
    _, d = api.solve(_t(dev, A32), _t(dev, B32), _t(dev, l32), out=X, warm_start=True, max_iter=5, tol=1e-30,
                     fp64_polish=0, iteration_kernel="stream")
    Xo, do = orc.rbpg_batch(A64, B64, L64, tol=1e-30, max_iter=5, X0=X0.astype(np.complex128))
    e = _rel_err(X.cpu().numpy().astype(np.complex128), Xo, B64, orc.lipschitz(A64))
    assert np.median(e) < 1e-6
    assert (e <= 1e-4).mean() >= 0.95
    assert np.mean(d["iters"].cpu().numpy() == do["iters"]) >= 0.95


def test_stream_golden_trajectories(dev):
    """The hand-derived golden trajectories (cold and warm start) on the streamed tile."""
    from test_oracle_trajectory import A_G, B_G, LAM_G, golden_rows, warm_rows
    p = 64
    rot = np.exp(1j * np.linspace(-3.0, 3.0, p))
    Ad = _t(dev, A_G.astype(np.complex64))
    Bd = _t(dev, (B_G[None, :] * rot[:, None]).astype(np.complex64))
    ld = _t(dev, np.full(p, LAM_G, np.float32))
    for rows, warm in ((golden_rows(), False), (warm_rows(), True)):
        start = rows[0] if warm else None
        X0 = (np.array([float(v) for v in start["x"]])[None, :] * rot[:, None]).astype(np.complex64) if warm \
            else None
        for r in rows[1:] if warm else rows:
            X = _t(dev, X0) if warm else None
            X, d = api.solve(Ad, Bd, ld, out=X, warm_start=warm, max_iter=r["k"], tol=1e-30, fp64_polish=0,
                             iteration_kernel="stream")
            want = np.array([float(v) for v in r["x"]])[None, :] * rot[:, None]
            Xg = X.cpu().numpy().astype(np.complex128)
            assert np.abs(Xg - want).max() <= 2e-6 * max(np.abs(want).max(), 1e-30), (warm, r["k"])
            assert (d["iters"].cpu().numpy() == r["k"]).all()


@pytest.mark.parametrize("n,l,p", [(100, 1024, 512 * 16 + 5), (90, 700, 20000)])
def test_stream_more_tiles_than_workgroups(dev, orc, n, l, p):
    """More 16-pixel tiles than persistent workgroups (each workgroup's state slot is
    reused tile after tile): twelve iterations on sampled pixels follow the oracle's
    Algorithm 1, and the default solve (FP64 stage on, tol 1e-4) certifies every pixel
    with its objective within the tolerance's bar of the minimum, as the wave-per-pixel
    kernel's solve does."""
    A32, B32, l32 = _stack(n, l, p)
    Ad, Bd, ld = _t(dev, A32), _t(dev, B32), _t(dev, l32)
    idx = np.unique(np.linspace(0, p - 1, 24).astype(int))
    A64 = A32.astype(np.complex128)
    B64, L64 = B32[idx].astype(np.complex128), l32[idx].astype(np.float64)
    Lf = orc.lipschitz(A64)
    X, d = api.solve(Ad, Bd, ld, max_iter=12, tol=1e-30, fp64_polish=0, iteration_kernel="stream")
    Xo, do = orc.rbpg_batch(A64, B64, L64, tol=1e-30, max_iter=12)
    e = _rel_err(X.cpu().numpy()[idx].astype(np.complex128), Xo, B64, Lf)
    assert np.median(e) < 1e-5 and (e <= 1e-3).mean() >= 0.9, (np.median(e), e.max())
    assert np.mean(d["iters"].cpu().numpy()[idx] == do["iters"]) >= 0.9
    Xe, de = orc.exact_batch(A64, B64, L64)
    objs = []
    for kern in ("stream", "wave"):
        X, d = api.solve(Ad, Bd, ld, polish_after=12, iteration_kernel=kern)
        conv = (d["status"].cpu().numpy() & _lib.PX_CONVERGED) != 0
        assert conv.mean() >= 0.999, kern
        Xg = X.cpu().numpy()[idx].astype(np.complex128)
        Fg = np.array([orc.objective(A64, B64[j], L64[j], Xg[j]) for j in range(len(idx))])
        ko = np.array([orc.kkt_nat(A64, B64[j], L64[j], Xg[j], Lf) for j in range(len(idx))])
        gap = (Fg - de["objective"]) / np.maximum(de["objective"], 1.0)
        assert gap.min() >= -1e-12 and gap[conv[idx]].max() <= 1e-4, (kern, gap.max())
        assert (ko[conv[idx]] <= 1e-4 * (1 + 1e-5)).all(), kern
        objs.append(Fg)
    assert np.abs(objs[0] - objs[1]).max() <= 1e-4 * max(np.abs(objs[1]).max(), 1.0)


@pytest.mark.parametrize("n,l,p", [(50, 2048, 40), (40, 4096, 20), (128, 3000, 17)])
def test_grids_beyond_1024_bins_reach_the_minimiser(dev, orc, n, l, p):
    """Beyond 1,024 bins (the streamed tile, the refinement with its bin Gram, the
    certificate): with every pixel refined to FP64 accuracy each pixel is certified
    and its objective is the oracle's minimum."""
    A32, B32, l32 = _stack(n, l, p)
    X, d = api.solve(_t(dev, A32), _t(dev, B32), _t(dev, l32), fp64_polish=2, polish_after=12)
    A64, B64, L64 = A32.astype(np.complex128), B32.astype(np.complex128), l32.astype(np.float64)
    Xe, de = orc.exact_batch(A64, B64, L64)
    Xg = X.cpu().numpy().astype(np.complex128)
    Fg = np.array([orc.objective(A64, B64[i], L64[i], Xg[i]) for i in range(p)])
    gap = (Fg - de["objective"]) / np.maximum(de["objective"], 1.0)
    conv = (d["status"].cpu().numpy() & _lib.PX_CONVERGED) != 0
    assert conv.all() and gap.max() <= 1e-9, (conv.mean(), gap.max())
