"""Gap-safe column screening (oracle.gap_screen, not in the paper): every bin it
declares zero is zero in the certified minimiser, at any point x; at the exact
minimiser of an orthonormal-column problem (closed form) it declares zero exactly
the bins with 2|a_l^H b| < lambda; and it screens more as x approaches x*."""
import numpy as np
import pytest

from paper_1805_01759_amd import synth


def _pixels(cfg, p):
    spec, geom, B, lam = synth.make_config(cfg, 0, p)
    A32, B32, l32 = synth.to_device_dtypes(geom.A, B, lam)
    return A32.astype(np.complex128), B32.astype(np.complex128), l32.astype(np.float64)


@pytest.mark.parametrize("cfg,p", [(1, 96), (2, 48), (4, 24)])
def test_screen_never_removes_a_support_bin(orc, cfg, p):
    A, B, L = _pixels(cfg, p)
    Xe, de = orc.exact_batch(A, B, L)
    assert de["kkt_sub"].max() <= 1e-10
    fracs = []
    for k in (3, 30, 300):
        Xk, _ = orc.rbpg_batch(A, B, L, tol=1e-30, max_iter=k)
        for i in range(p):
            mask, gap = orc.gap_screen(A, B[i], L[i], Xk[i])
            assert gap >= -1e-9 * max(1.0, de["objective"][i])
            assert not np.any(mask & (Xe[i] != 0)), (cfg, k, i)
            fracs.append((k, mask.mean()))
    for i in range(p):
        mask, gap = orc.gap_screen(A, B[i], L[i], Xe[i])
        assert not np.any(mask & (Xe[i] != 0))
        fracs.append((10 ** 9, mask.mean()))
    by_k = {k: np.mean([f for kk, f in fracs if kk == k]) for k in (3, 30, 300, 10 ** 9)}
    print(cfg, by_k)
    # closer points screen more; at the minimiser most off-support bins go
    assert by_k[3] <= by_k[300] + 1e-12 and by_k[300] <= by_k[10 ** 9] + 1e-12
    assert by_k[10 ** 9] >= 0.5


def test_screen_closed_form_orthonormal(orc):
    rng = np.random.default_rng(3)
    n, l = 12, 8
    Q, _ = np.linalg.qr(rng.standard_normal((n, l)) + 1j * rng.standard_normal((n, l)))
    for trial in range(20):
        b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        c = Q.conj().T @ b
        lam = float(np.sort(2 * np.abs(c))[trial % l]) * 0.999 + 1e-3
        # x* = S_{lambda/2}(A^H b) for orthonormal columns
        mag = np.abs(c)
        xs = np.where(mag > lam / 2, c * (1 - lam / 2 / np.maximum(mag, 1e-300)), 0)
        mask, gap = orc.gap_screen(Q, b, lam, xs)
        assert abs(gap) <= 1e-10 * max(1.0, np.linalg.norm(b) ** 2)
        # at x*, s = 1 and the radius is ~0: exactly the bins with 2|a_l^H b| < lambda
        want = 2 * mag < lam * (1 - 1e-9)
        assert np.array_equal(mask[want], np.ones(want.sum(), bool))
        assert not np.any(mask[2 * mag > lam * (1 + 1e-9)])
        # at x = 0 only bins far inside the dual ball go
        m0, g0 = orc.gap_screen(Q, b, lam, np.zeros(l, complex))
        assert not np.any(m0 & (xs != 0))


@pytest.mark.parametrize("b,x,gap,screened", [
    # hand-derived, N = L = 1, A = [1], lambda = 1 (F(x) = (x - b)^2 + |x|, x* = S_{1/2}(b)):
    # b = 0.6 (x* = 0.1), x = 0.3: r = -0.3, g = -0.6, s = 1, nu = -0.6, F = 0.39,
    #   D = -0.09 + 0.36 = 0.27, gap = 0.12; 0.6 + 2 sqrt(0.12) = 1.293 > 1: kept
    #   (with a radius of sqrt(gap) instead, 0.946 < 1 would drop a nonzero of x*)
    (0.6, 0.3, 0.12, False),
    # b = 0.1 (x* = 0), x = 0.2: g = 0.2, nu = 0.2, F = 0.21, D = -0.01 - 0.02, gap = 0.24;
    #   0.2 + 2 sqrt(0.24) = 1.18 > 1: kept
    (0.1, 0.2, 0.24, False),
    # b = 0.1, x = 0: g = -0.2, nu = -0.2, F = 0.01, D = -0.01 + 0.02 = 0.01, gap = 0: dropped
    (0.1, 0.0, 0.0, True),
    # b = 0.6, x = 0: g = -1.2, s = 1/1.2, nu = -1, F = 0.36, D = -0.25 + 0.6, gap = 0.01;
    #   s |g| = 1: kept
    (0.6, 0.0, 0.01, False),
])
def test_screen_scalar_closed_form(orc, b, x, gap, screened):
    A = np.array([[1.0 + 0j]])
    mask, g = orc.gap_screen(A, np.array([b + 0j]), 1.0, np.array([x + 0j]))
    assert abs(g - gap) <= 1e-12
    assert bool(mask[0]) == screened
