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
