"""The double-scatterer detection rule (paper_1805_01759_amd.detect) on
constructed profiles, and the paper's qualitative super-resolution statements
on the oracle's minimisers of the double-scatterer stacks.

The rule itself is this package's (the paper's detection step belongs to the
SL1MMER model selection, which the paper does not define), so its counts are
pinned only by these constructed cases.  The statements from the simulation
section are weak pins of the minimiser on this workload: at SNR 10 dB the
minimiser separates the pair down to kappa = 0.4, both at 3 dB and 10 dB it
separates kappa = 1.2, and at kappa = 0.2, 3 dB the pair is lost.
"""
import numpy as np
import pytest

from paper_1805_01759_amd import detect, synth

S = np.linspace(-80.0, 80.0, 256)
RHO = 40.26


def _profile(entries):
    x = np.zeros(256, np.complex128)
    for m, v in entries:
        x[m] = v
    return x


def test_clusters_weights_and_positions():
    x = _profile([(100, 1.0), (101, 3.0), (150, 1j), (200, 0.05)])
    w, p = detect.clusters(x, S)
    assert np.allclose(w, [4.0, 1.0, 0.05])
    assert np.isclose(p[0], (S[100] * 1 + S[101] * 3) / 4)
    assert np.isclose(p[1], S[150])


def test_pair_rule_cases():
    s1, s2 = -8.0, 8.0
    m1, m2 = np.argmin(abs(S - s1)), np.argmin(abs(S - s2))
    assert detect.detects_pair(_profile([(m1, 1.0), (m2, 0.8)]), S, s1, s2, RHO)
    # one cluster only (merged)
    assert not detect.detects_pair(_profile([(127, 1.0), (128, 1.0)]), S, s1, s2, RHO)
    # second peak lighter than 10 % of the first: dropped
    assert not detect.detects_pair(_profile([(m1, 1.0), (m2, 0.05)]), S, s1, s2, RHO)
    # both peaks on one side of the midpoint
    assert not detect.detects_pair(_profile([(m2 - 3, 1.0), (m2 + 3, 1.0)]), S, s1, s2, RHO)
    # a peak beyond half a resolution cell from its scatterer
    far = np.argmin(abs(S - (s2 + 0.6 * RHO)))
    assert not detect.detects_pair(_profile([(m1, 1.0), (far, 1.0)]), S, s1, s2, RHO)
    # a light third cluster does not matter; the heaviest two decide
    assert detect.detects_pair(_profile([(m1, 1.0), (m2, 0.9), (10, 0.3)]), S, s1, s2, RHO)


def _rates(orc, cases, R):
    geom, B, lam, meta = synth.make_superres(R, cases=cases)
    A32, B32, l32 = synth.to_device_dtypes(geom.A, B, lam)
    X, d = orc.exact_batch(A32.astype(np.complex128), B32.astype(np.complex128), l32.astype(np.float64))
    assert d["kkt_sub"].max() <= 1e-10
    out = []
    for c in range(len(cases)):
        sl = slice(c * R, (c + 1) * R)
        out.append(detect.detection_rate(X[sl], geom.s, meta["s1"][sl], meta["s2"][sl], geom.rayleigh))
    return out


def test_superresolution_statements_on_the_minimiser(orc):
    cases = [("profiles", 0.4, 10.0), ("profiles", 1.2, 10.0), ("profiles", 1.2, 3.0),
             ("profiles", 0.2, 3.0)]
    r = _rates(orc, cases, 60)
    print("detection rates", r)
    assert r[0] >= 0.8      # kappa 0.4, 10 dB: two separated peaks
    assert r[1] >= 0.95 and r[2] >= 0.95
    assert r[3] <= 0.5      # kappa 0.2, 3 dB: the pair is lost
