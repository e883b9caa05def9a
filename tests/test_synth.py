"""Seeded synthetic inputs: shapes, reproducibility, pixel-subset independence."""
import math

import numpy as np

from paper_1805_01759_amd import synth


def test_shapes_and_lambda():
    spec, geom, B, lam = synth.make_config(1)
    assert B.shape == (1024, 15) and geom.A.shape == (15, 101)
    assert np.allclose(np.abs(geom.A), 1.0)
    sigma = math.sqrt(0.1)
    assert np.allclose(lam, sigma * math.sqrt(2 * 15 * math.log(101)))
    assert abs(lam[0] - 3.72) < 0.01


def test_subset_reproducible():
    _, _, B, lam = synth.make_config(2, 0, 10000)
    _, _, B2, lam2 = synth.make_config(2, 4000, 9000)
    assert np.array_equal(B[4000:9000], B2) and np.array_equal(lam[4000:9000], lam2)
    _, _, B3, _ = synth.make_config(2, 0, 10000)
    assert np.array_equal(B, B3)


def test_scatterer_mix_and_snr():
    _, geom, B, lam, meta = synth.make_config(2, 0, 20000, with_meta=True)
    frac = np.bincount(meta["k"], minlength=3) / 20000
    assert np.allclose(frac, [0.3, 0.5, 0.2], atol=0.02)
    assert meta["snr_db"].min() >= 0 and meta["snr_db"].max() <= 20
    assert 1.6 < lam.min() and lam.max() < 16.7
    # noise-only pixels: mean power per acquisition equals sigma^2
    z = meta["k"] == 0
    sig2 = 10 ** (-meta["snr_db"][z] / 10)
    ratio = (np.abs(B[z]) ** 2).mean(1) / sig2
    assert abs(ratio.mean() - 1) < 0.05


def test_close_pairs_config4():
    _, geom, B, lam, meta = synth.make_config(4, 0, 8192, with_meta=True)
    ds = np.abs(meta["elev"][:, 1] - meta["elev"][:, 0])
    kappa = ds / geom.rayleigh
    pairs = (meta["k"] == 2) & (kappa <= 1.0) & (kappa >= 0.3)
    assert pairs.mean() > 0.35
    assert (meta["elev"] >= -60).all() and (meta["elev"] <= 60).all()


def test_rayleigh_uses_half_aperture_reading():
    g = synth.make_geometry(1, 15, 101, 250.0, -50.0, 50.0)
    span = g.baselines.max() - g.baselines.min()
    assert np.isclose(g.rayleigh, 0.031 * 7e5 / (2 * span))
    xi_span = g.xi.max() - g.xi.min()
    assert np.isclose(g.rayleigh, 1 / xi_span)


def test_batched_specs():
    ss = synth.batched_specs()
    assert len(ss) == 64
    assert all(10 <= s.n <= 100 and 64 <= s.l <= 1024 and 1000 <= s.p <= 256000 for s in ss)


def test_config5_on_grid_truth():
    spec, geom, B, lam, meta = synth.make_config(5, 0, 512, with_meta=True)
    X = synth.xtrue(spec, geom, meta)
    resid = B - X @ geom.A.T
    assert np.abs(resid).std() < 0.5  # only noise remains


def test_motion_matrix_is_kronecker_of_steering():
    """Eqs. (3)-(4): column i + Ls j of A is the elevation steering vector of s_i
    times the velocity one of v_j (unit modulus)."""
    spec, geom, B, lam = synth.make_motion_config(6, 0, 64)
    assert geom.A.shape == (50, 512) and B.shape == (64, 50)
    Es = np.exp(-2j * np.pi * np.outer(geom.xi, geom.s))
    Ev = np.exp(-2j * np.pi * np.outer(geom.eta, geom.v))
    want = (Es[:, None, :] * Ev[:, :, None]).reshape(50, -1)
    assert np.allclose(geom.A, want, atol=1e-12)
    assert np.allclose(np.abs(geom.A), 1.0)
    assert np.all(np.diff(geom.times) >= 0) and geom.times.max() <= 3.0
    assert np.allclose(lam, np.sqrt(10 ** (-_motion_snr(0, 64) / 10)) * math.sqrt(2 * 50 * math.log(512)))


def _motion_snr(p0, p1):
    return synth.make_motion_config(6, p0, p1, with_meta=True)[4]["snr_db"]


def test_motion_subset_reproducible():
    _, _, B, lam = synth.make_motion_config(6, 0, 9000)
    _, _, B2, lam2 = synth.make_motion_config(6, 4000, 9000)
    assert np.array_equal(B[4000:9000], B2) and np.array_equal(lam[4000:9000], lam2)


def test_motion_pixels_follow_the_model():
    """A noiseless-limit check: B minus the scatterers' steering vectors is the
    noise, whose power matches the drawn SNR."""
    spec, geom, B, lam, meta = synth.make_motion_config(6, 0, 8000, with_meta=True)
    sig = np.einsum("pk,pkn->pn", meta["amp"], synth.motion_steering(geom, meta["elev"], meta["vel"]))
    noise = B - sig
    ratio = np.mean(np.abs(noise) ** 2, axis=1) / 10 ** (-meta["snr_db"] / 10)
    assert abs(np.mean(ratio) - 1.0) < 0.02
    frac = np.bincount(meta["k"], minlength=3) / 8000
    assert np.allclose(frac, [0.3, 0.5, 0.2], atol=0.02)


def test_superres_cases():
    """Double-scatterer stacks: N = 29 over the full 269.5 m aperture, rho_s from it,
    the pair at +-kappa rho_s / 2, unit amplitudes, phase difference 0 in the
    detection set, noise at the per-scatterer SNR, ranges regenerate alone."""
    R = 400
    geom, B, lam, meta = synth.make_superres(R)
    ncase = len(synth.SUPERRES_CASES)
    assert B.shape == (ncase * R, 29) and geom.A.shape == (29, 256)
    assert math.isclose(geom.baselines.max() - geom.baselines.min(), 269.5)
    assert math.isclose(geom.rayleigh, 0.031 * 7e5 / (2 * 269.5))
    for c, (kind, kappa, snr) in enumerate(synth.SUPERRES_CASES):
        sl = slice(c * R, (c + 1) * R)
        assert np.all(meta["case"][sl] == c) and np.all(meta["kappa"][sl] == kappa)
        assert np.allclose(meta["s2"][sl] - meta["s1"][sl], kappa * geom.rayleigh)
        assert np.allclose(meta["s1"][sl] + meta["s2"][sl], 0.0)
        a1 = synth.steering(geom.xi, meta["s1"][sl][:1])[0]
        a2 = synth.steering(geom.xi, meta["s2"][sl][:1])[0]
        sig = a1[None, :] + np.exp(1j * meta["dphi"][sl])[:, None] * a2[None, :]
        noise = B[sl] - sig
        sigma2 = 10 ** (-snr / 10)
        assert abs((np.abs(noise) ** 2).mean() / sigma2 - 1) < 0.05
        assert np.allclose(lam[sl], math.sqrt(sigma2) * math.sqrt(2 * 29 * math.log(256)))
        if kind == "detection":
            assert np.all(meta["dphi"][sl] == 0.0)
        else:
            assert meta["dphi"][sl].min() >= 0 and meta["dphi"][sl].max() < 2 * math.pi
            assert meta["dphi"][sl].std() > 1.5
    _, B2, _, meta2 = synth.make_superres(100, r0=250)
    for c in range(ncase):
        assert np.array_equal(B2[c * 100:(c + 1) * 100], B[c * R + 250:c * R + 350])


def test_seasonal_motion_matrix_is_kronecker_of_three_steerings():
    """Eq. (4) with a seasonal component (base function sin(2 pi t)): column
    i + Ls j + Ls Lv k of A is the product of the elevation, velocity and seasonal
    steering vectors of (s_i, v_j, a_k), and the pixels follow the model."""
    spec, geom, B, lam, meta = synth.make_motion_config(10, 0, 4000, with_meta=True)
    assert geom.A.shape == (50, 4096) and spec.l == 4096 and B.shape == (4000, 50)
    Es = np.exp(-2j * np.pi * np.outer(geom.xi, geom.s))
    Ev = np.exp(-2j * np.pi * np.outer(geom.eta, geom.v))
    Ea = np.exp(-2j * np.pi * np.outer(geom.zeta, geom.a))
    want = (Es[:, None, None, :] * Ev[:, None, :, None] * Ea[:, :, None, None]).reshape(50, -1)
    assert np.allclose(geom.A, want, atol=1e-12)
    assert np.allclose(geom.zeta, 2 * np.sin(2 * np.pi * geom.times) / 0.031)
    sig = np.einsum("pk,pkn->pn", meta["amp"],
                    synth.motion_steering(geom, meta["elev"], meta["vel"], meta["seas"]))
    ratio = np.mean(np.abs(B - sig) ** 2, axis=1) / 10 ** (-meta["snr_db"] / 10)
    assert abs(np.mean(ratio) - 1.0) < 0.03
    assert meta["seas"].min() >= -0.01 and meta["seas"].max() <= 0.01
    assert np.allclose(lam, np.sqrt(10 ** (-meta["snr_db"] / 10)) * math.sqrt(2 * 50 * math.log(4096)))
