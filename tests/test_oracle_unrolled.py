"""Pins of the unrolled fixed-step reference (Eqs. (11)-(12), constant step).

Two independent FP64 implementations (C loop, PyTorch loop) must agree, and
the autograd gradients of the PyTorch loop must agree with central finite
differences of the C forward map.  The complex soft threshold's VJP is checked
against finite differences away from its kink.
"""
import numpy as np
import pytest
import torch

from paper_1805_01759_amd import synth


def _problem(p=6, n=6, l=16, K=12, seed=0):
    rng = np.random.default_rng(seed)
    b = rng.uniform(-250, 250, n)
    xi = 2 * b / (synth.WAVELENGTH * synth.RANGE)
    s = np.linspace(-30, 30, l)
    A = np.exp(-2j * np.pi * np.outer(xi, s))
    X = np.zeros((p, l), complex)
    for i in range(p):
        X[i, rng.integers(0, l, 2)] = rng.standard_normal(2) + 1j * rng.standard_normal(2)
    B = X @ A.T + 0.1 * (rng.standard_normal((p, n)) + 1j * rng.standard_normal((p, n)))
    lam = 0.8
    Lf = 2 * np.linalg.eigvalsh(A @ A.conj().T).max()
    return xi, s, A, B, X, lam, 1.0 / Lf, K


def test_c_and_torch_forward_agree(orc):
    from oracle import unrolled_ref
    xi, s, A, B, X, lam, alpha, K = _problem()
    Xc = orc.unrolled_batch(A, B, lam, alpha, K)
    Xt = unrolled_ref.unrolled(torch.tensor(xi), torch.tensor(s), torch.tensor(B),
                               torch.tensor(lam, dtype=torch.float64), alpha, K).numpy()
    assert np.abs(Xc - Xt).max() <= 1e-12 * max(1.0, np.abs(Xc).max())


def _fd_loss(orc, xi, s, B, lam, alpha, K, Xtrue):
    A = np.exp(-2j * np.pi * np.outer(xi, s))
    Xk = orc.unrolled_batch(A, B, lam, alpha, K)
    return float(np.sum(np.abs(Xk - Xtrue) ** 2))


def test_autograd_matches_finite_differences(orc):
    from oracle import unrolled_ref
    xi, s, A, B, Xtrue, lam, alpha, K = _problem(seed=3)
    loss, Xk, dB, dlam, dxi = unrolled_ref.loss_and_grads(
        torch.tensor(xi), torch.tensor(s), torch.tensor(B), lam, alpha, K, torch.tensor(Xtrue))
    f = lambda xi_, B_, lam_: _fd_loss(orc, xi_, s, B_, lam_, alpha, K, Xtrue)
    # xi: perturb through the baseline, 1e-3 m (dxi = 2 h / (lambda_w r))
    hx = 2e-3 / (synth.WAVELENGTH * synth.RANGE)
    for nidx in range(len(xi)):
        e = np.zeros_like(xi)
        e[nidx] = hx
        fd = (f(xi + e, B, lam) - f(xi - e, B, lam)) / (2 * hx)
        assert fd == pytest.approx(dxi[nidx].item(), rel=1e-5, abs=1e-6 * abs(dxi).max().item())
    hl = 1e-6 * lam
    fd = (f(xi, B, lam + hl) - f(xi, B, lam - hl)) / (2 * hl)
    assert fd == pytest.approx(dlam.item(), rel=1e-5)
    rng = np.random.default_rng(1)
    for _ in range(4):
        D = rng.standard_normal(B.shape) + 1j * rng.standard_normal(B.shape)
        h = 1e-6
        fd = (f(xi, B + h * D, lam) - f(xi, B - h * D, lam)) / (2 * h)
        an = float(np.sum((dB.numpy().conj() * D).real))
        assert fd == pytest.approx(an, rel=1e-5, abs=1e-8)


def test_prox_vjp_matches_fd():
    """VJP of S_tau (complex) vs central differences, away from |v| = tau."""
    from oracle import unrolled_ref
    rng = np.random.default_rng(5)
    v = torch.tensor(rng.standard_normal(64) + 1j * rng.standard_normal(64))
    tau = torch.tensor(0.7, dtype=torch.float64)
    keep = (v.abs() - tau).abs() > 1e-3
    v = v[keep]
    w = torch.tensor(rng.standard_normal(v.shape[0]) + 1j * rng.standard_normal(v.shape[0]))
    vv = v.clone().requires_grad_(True)
    tt = tau.clone().requires_grad_(True)
    out = unrolled_ref.prox(vv, tt)
    (out.conj() * w).real.sum().backward()
    h = 1e-7
    def L(v_, t_):
        return float((unrolled_ref.prox(v_, t_).conj() * w).real.sum())
    for i in range(v.shape[0]):
        for d in (1.0, 1j):
            e = torch.zeros_like(v)
            e[i] = d * h
            fd = (L(v + e, tau) - L(v - e, tau)) / (2 * h)
            an = vv.grad[i].real.item() if d == 1.0 else vv.grad[i].imag.item()
            assert fd == pytest.approx(an, abs=1e-7)
    fd = (L(v, tau + h) - L(v, tau - h)) / (2 * h)
    assert fd == pytest.approx(tt.grad.item(), abs=1e-6)
