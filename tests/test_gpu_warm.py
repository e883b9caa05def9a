"""Algorithm 1 from a given initial point (warm_start: X holds x^(0) on entry,
the Init of Algorithm 1) through the C ABI, against the oracle started from the
same point: the hand-derived warm trajectory, the first iterations on the MFMA
and the wave-per-pixel kernels, the fixed point at the minimiser, and full
solves from perturbed minimisers."""
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
    geom = synth.make_geometry(seed_cfg, n, l, 250.0, -50.0, 50.0)
    spec = synth.Spec(seed_cfg, n, l, p, 250.0, -50.0, 50.0, "c1", 10.0)
    B, lam = synth.make_pixels(spec, geom)
    return synth.to_device_dtypes(geom.A, B, lam)


@pytest.mark.parametrize("precision,rtol", [("fp32", 2e-6), ("split_bf16", 2e-4)])
def test_golden_warm_trajectory_on_device(dev, precision, rtol):
    """tests/golden/algorithm1_warm_start.txt for 64 pixels whose b and x^(0) are the
    golden ones rotated by a per-pixel phase (A is real, so every iterate rotates)."""
    from test_oracle_trajectory import A_G, B_G, LAM_G, warm_rows
    rows = warm_rows()
    p = 64
    rot = np.exp(1j * np.linspace(-3.0, 3.0, p))
    x0 = np.array([float(v) for v in rows[0]["x"]])
    Ad = _t(dev, A_G.astype(np.complex64))
    Bd = _t(dev, (B_G[None, :] * rot[:, None]).astype(np.complex64))
    ld = _t(dev, np.full(p, LAM_G, np.float32))
    X0 = (x0[None, :] * rot[:, None]).astype(np.complex64)
    for r in rows[1:]:
        X = _t(dev, X0)
        _, d = api.solve(Ad, Bd, ld, out=X, warm_start=True, max_iter=r["k"], tol=1e-30, fp64_polish=0,
                         precision=precision)
        want = np.array([float(v) for v in r["x"]])[None, :] * rot[:, None]
        Xg = X.cpu().numpy().astype(np.complex128)
        assert np.abs(Xg - want).max() <= rtol * np.abs(want).max(), r["k"]
        assert (d["iters"].cpu().numpy() == r["k"]).all()


@pytest.mark.parametrize("n,l,p,precision", [(15, 101, 512, "fp32"), (25, 256, 256, "fp32"), (70, 300, 96, "fp32"),
                                             (25, 256, 256, "split_bf16"), (40, 200, 128, "split_bf16"),
                                             (50, 512, 128, "split_bf16")])
def test_warm_trajectory_parity(dev, orc, n, l, p, precision):
    """Five iterations from x^(0) = the oracle's third iterate from 0 (complex64): device
    (MFMA kernel for n <= 64, wave kernel above; split-BF16 with A's planes in LDS or
    read from L2) against the oracle from the same x^(0)."""
    A32, B32, l32 = _stack(n, l, p)
    A64, B64, L64 = A32.astype(np.complex128), B32.astype(np.complex128), l32.astype(np.float64)
    X3, _ = orc.rbpg_batch(A64, B64, L64, tol=1e-30, max_iter=3)
    X0 = X3.astype(np.complex64)
    print(f"warm trajectory n={n} l={l} p={p}", flush=True)
    X = _t(dev, X0)
    _, d = api.solve(_t(dev, A32), _t(dev, B32), _t(dev, l32), out=X, warm_start=True, max_iter=5,
                     tol=1e-30, fp64_polish=0, precision=precision)
    Xo, do = orc.rbpg_batch(A64, B64, L64, tol=1e-30, max_iter=5, X0=X0.astype(np.complex128))
    Xg = X.cpu().numpy().astype(np.complex128)
    Lf = orc.lipschitz(A64)
    den = np.maximum(np.linalg.norm(Xo, axis=1), np.linalg.norm(B64, axis=1) / np.sqrt(Lf / 2))
    e = np.linalg.norm(Xg - Xo, axis=1) / den
    # the cold start from 0 reaches a different point after five iterations
    Xc, _ = orc.rbpg_batch(A64, B64, L64, tol=1e-30, max_iter=5)
    ec = np.linalg.norm(Xc - Xo, axis=1) / den
    print(f"  e median {np.median(e):.1e}, e <= 1e-4 {np.mean(e <= 1e-4):.3f}; cold differs {np.median(ec):.1e}")
    # split-BF16 products carry about 2^-16 relative error each (three bf16 passes)
    med, bar = (1e-6, 1e-4) if precision == "fp32" else (3e-5, 1e-3)
    assert np.median(e) < med
    assert (e <= bar).mean() >= 0.98
    assert np.median(ec) > 1e-3
    # iterations performed agree (an FP32 iterate can land exactly on its fixed point,
    # which the tol = 1e-30 test then reports converged a step early)
    assert np.mean(d["iters"].cpu().numpy() == do["iters"]) >= 0.99


@pytest.mark.parametrize("n,l,p", [(25, 256, 256), (70, 300, 64)])
def test_warm_start_at_the_minimiser(dev, orc, n, l, p):
    """From the certified minimiser the first KKT test passes: no iteration, x unchanged."""
    A32, B32, l32 = _stack(n, l, p)
    Xe, _ = orc.exact_batch(A32.astype(np.complex128), B32.astype(np.complex128), l32.astype(np.float64))
    X0 = Xe.astype(np.complex64)
    X = _t(dev, X0)
    _, d = api.solve(_t(dev, A32), _t(dev, B32), _t(dev, l32), out=X, warm_start=True, fp64_polish=0)
    assert (d["iters"].cpu().numpy() == 0).all()
    assert np.array_equal(X.cpu().numpy(), X0)
    assert ((d["status"].cpu().numpy() & _lib.PX_CONVERGED) != 0).all()


@pytest.mark.parametrize("n,l,p", [(25, 256, 512), (70, 300, 96)])
def test_warm_solve_from_perturbed_minimiser(dev, orc, n, l, p):
    """A full solve (FP64 stage on) from a perturbed minimiser certifies every pixel and
    reaches the minimum (objective within the FP32 bar); it needs fewer iterations than
    the cold start."""
    A32, B32, l32 = _stack(n, l, p)
    A64, B64, L64 = A32.astype(np.complex128), B32.astype(np.complex128), l32.astype(np.float64)
    Xe, de = orc.exact_batch(A64, B64, L64)
    rng = np.random.default_rng(5)
    pert = 0.05 * (rng.standard_normal(Xe.shape) + 1j * rng.standard_normal(Xe.shape)) * (Xe != 0)
    X0 = (Xe + pert).astype(np.complex64)
    Ad, Bd, ld = _t(dev, A32), _t(dev, B32), _t(dev, l32)
    X = _t(dev, X0)
    _, d = api.solve(Ad, Bd, ld, out=X, warm_start=True, fp64_polish=1, polish_after=100)
    Xg = X.cpu().numpy().astype(np.complex128)
    Fg = np.array([orc.objective(A64, B64[i], L64[i], Xg[i]) for i in range(p)])
    gap = (Fg - de["objective"]) / np.maximum(de["objective"], 1.0)
    assert ((d["status"].cpu().numpy() & _lib.PX_CONVERGED) != 0).all()
    assert gap.min() >= -1e-12 and gap.max() <= 1e-4
    _, dc = api.solve(Ad, Bd, ld, fp64_polish=1, polish_after=100)
    assert d["iters"].float().mean().item() < dc["iters"].float().mean().item()


def test_warm_start_needs_out(dev):
    A32, B32, l32 = _stack(20, 400, 8)
    with pytest.raises(ValueError):
        api.solve(_t(dev, A32), _t(dev, B32), _t(dev, l32), warm_start=True)
