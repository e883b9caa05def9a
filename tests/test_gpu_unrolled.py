"""GPU unrolled map and its hand-written adjoint against the FP64 references.

Forward: the C FP64 loop (oracle.unrolled_batch).  Gradients: PyTorch autograd
of the complex128 CPU loop (oracle.unrolled_ref), itself pinned by central
finite differences in the CPU tests.  Tolerances come from FP32 rounding
carried through K fixed-step iterations (measured, not assumed: reported in
the assertion messages).
"""
import numpy as np
import pytest
import torch

from paper_1805_01759_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch.device("cuda:0")


def _problem(p, K=200):
    spec, geom, B, lam, meta = synth.make_config(5, 0, p, with_meta=True)
    Xt = synth.xtrue(spec, geom, meta)
    A = geom.A
    Lf = 2 * np.linalg.eigvalsh(A @ A.conj().T).max()
    alpha = 1.0 / Lf
    return geom, B.astype(np.complex64), float(np.float32(lam[0])), alpha, Xt


def test_forward_matches_fp64(dev, orc):
    from paper_1805_01759_amd.unrolled import unrolled
    geom, B, lam, alpha, Xt = _problem(1024)
    xi = torch.tensor(geom.xi, dtype=torch.float32)
    s = torch.tensor(geom.s, dtype=torch.float32)
    X = unrolled(torch.from_numpy(B).to(dev), lam, xi.to(dev), s.to(dev), alpha, 200, 20)
    # the oracle builds A from the same float32 xi and s, in FP64
    A64 = np.exp(-2j * np.pi * np.outer(xi.double().numpy(), s.double().numpy()))
    Xo = orc.unrolled_batch(A64, B.astype(np.complex128), lam, alpha, 200)
    Xg = X.cpu().numpy().astype(np.complex128)
    e = np.linalg.norm(Xg - Xo, axis=1) / np.maximum(np.linalg.norm(Xo, axis=1), 1e-3)
    print(f"unrolled forward: e p50 {np.median(e):.1e} p99 {np.percentile(e, 99):.1e} max {e.max():.1e}")
    assert e.max() < 1e-4


def test_gradients_match_fp64_autograd(dev):
    from oracle import unrolled_ref
    from paper_1805_01759_amd.unrolled import unrolled
    geom, B, lam, alpha, Xt = _problem(256, K=200)
    xi = torch.tensor(geom.xi, dtype=torch.float32)
    s = torch.tensor(geom.s, dtype=torch.float32)
    Bd = torch.from_numpy(B).to(dev).requires_grad_(True)
    lam_t = torch.tensor(lam, dtype=torch.float32, device=dev, requires_grad=True)
    xid = xi.to(dev).requires_grad_(True)
    X = unrolled(Bd, lam_t, xid, s.to(dev), alpha, 200, 20)
    Xt_d = torch.from_numpy(Xt.astype(np.complex64)).to(dev)
    loss = (X - Xt_d).abs().pow(2).sum()
    loss.backward()
    lref, Xref, dB, dlam, dxi = unrolled_ref.loss_and_grads(
        xi.double(), s.double(), torch.from_numpy(B.astype(np.complex128)), lam, alpha, 200,
        torch.from_numpy(Xt))
    gB = Bd.grad.cpu().numpy().astype(np.complex128)
    eB = np.linalg.norm(gB - dB.numpy()) / np.linalg.norm(dB.numpy())
    el = abs(lam_t.grad.item() - dlam.item()) / abs(dlam.item())
    ex = np.linalg.norm(xid.grad.cpu().double().numpy() - dxi.numpy()) / np.linalg.norm(dxi.numpy())
    print(f"unrolled grads: rel err dB {eB:.2e} dlambda {el:.2e} dxi {ex:.2e}")
    assert eB < 1e-4 and el < 1e-4 and ex < 1e-4, (eB, el, ex)


def test_checkpoint_spacing_does_not_change_gradients(dev):
    from paper_1805_01759_amd.unrolled import unrolled
    geom, B, lam, alpha, Xt = _problem(64, K=40)
    xi = torch.tensor(geom.xi, dtype=torch.float32, device=dev)
    s = torch.tensor(geom.s, dtype=torch.float32, device=dev)
    grads = []
    for ck in (1, 4, 40):
        Bd = torch.from_numpy(B).to(dev).requires_grad_(True)
        xid = xi.clone().requires_grad_(True)
        X = unrolled(Bd, lam, xid, s, alpha, 40, ck)
        (X.abs() ** 2).sum().backward()
        grads.append((Bd.grad.clone(), xid.grad.clone()))
    for g in grads[1:]:
        assert torch.equal(g[0], grads[0][0]) and torch.equal(g[1], grads[0][1])


def test_wave_kernels_outside_the_tile_shapes(dev, orc):
    """N = 40, L = 300 falls outside the matrix-core tile (N <= 32, L <= 256): the
    wave-per-pixel kernels run; forward and gradients against the FP64 references."""
    from oracle import unrolled_ref
    from paper_1805_01759_amd.unrolled import unrolled
    geom = synth.make_geometry(5, 40, 300, 300.0, -60.0, 60.0, stack=7)
    rng = np.random.default_rng(1805)
    p, K = 32, 40
    B = (rng.standard_normal((p, 40)) + 1j * rng.standard_normal((p, 40))).astype(np.complex64)
    lam = 4.0
    xi = torch.tensor(geom.xi, dtype=torch.float32)
    s = torch.tensor(geom.s, dtype=torch.float32)
    A64 = np.exp(-2j * np.pi * np.outer(xi.double().numpy(), s.double().numpy()))
    alpha = 1.0 / (2 * np.linalg.eigvalsh(A64 @ A64.conj().T).max())
    Bd = torch.from_numpy(B).to(dev).requires_grad_(True)
    xid = xi.to(dev).requires_grad_(True)
    X = unrolled(Bd, lam, xid, s.to(dev), alpha, K, 10)
    Xo = orc.unrolled_batch(A64, B.astype(np.complex128), lam, alpha, K)
    e = np.linalg.norm(X.detach().cpu().numpy() - Xo, axis=1) / np.maximum(np.linalg.norm(Xo, axis=1), 1e-3)
    assert e.max() < 1e-4, e.max()
    Xt = np.zeros((p, 300), np.complex128)
    (X.abs() ** 2).sum().backward()
    lref, Xref, dB, dlam, dxi = unrolled_ref.loss_and_grads(
        xi.double(), s.double(), torch.from_numpy(B.astype(np.complex128)), lam, alpha, K,
        torch.from_numpy(Xt))
    eB = np.linalg.norm(Bd.grad.cpu().numpy() - dB.numpy()) / np.linalg.norm(dB.numpy())
    ex = np.linalg.norm(xid.grad.cpu().double().numpy() - dxi.numpy()) / np.linalg.norm(dxi.numpy())
    print(f"wave kernels: forward e max {e.max():.1e}, grads dB {eB:.2e} dxi {ex:.2e}")
    assert eB < 1e-4 and ex < 1e-4, (eB, ex)
