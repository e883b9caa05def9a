"""GPU parity on the double-scatterer simulations (N = 29, L = 256, 24 cases of
separation kappa and SNR, 100 realisations each), solved as bench.py solves
them, against the oracle's certified minimiser of every realisation: the
certified KKT residual (device vs oracle), the objective gap, the distance to
the minimiser e_p, and the double-scatterer detections of the package's rule
on the device's x against those on the minimiser."""
import numpy as np
import pytest
import torch

import bench
from paper_1805_01759_amd import _lib, api, detect, synth

pytestmark = pytest.mark.gpu

R = 100


@pytest.fixture(scope="module")
def case(orc):
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    geom, B, lam, meta = synth.make_superres(R)
    A32, B32, l32 = synth.to_device_dtypes(geom.A, B, lam)
    A64, B64, L64 = A32.astype(np.complex128), B32.astype(np.complex128), l32.astype(np.float64)
    Xe, de = orc.exact_batch(A64, B64, L64)
    return dict(geom=geom, meta=meta, A32=A32, B32=B32, l32=l32, A64=A64, B64=B64, L64=L64, Xe=Xe,
                de=de, Lf=orc.lipschitz(A64))


# pass-fraction floors (e_p <= bar and solved); measured 0.966 (FP32 bar) and 0.997
# (split-BF16 bar): on this grid (64 bins per resolution cell, N = 29) the
# minimiser of a few percent of the realisations is determined to worse than
# 1e-4 even at FP64 KKT residuals of 1e-10
@pytest.mark.parametrize("prec,bar,floor", [("fp32", 1e-4, 0.95), ("split_bf16", 1e-3, 0.99)])
def test_superres_parity_and_detections(case, orc, prec, bar, floor):
    dev = torch.device("cuda:0")
    print(f"superres {prec}: {case['B32'].shape[0]} pixels", flush=True)
    Ad, Bd, ld = (torch.from_numpy(x).to(dev) for x in (case["A32"], case["B32"], case["l32"]))
    X, d = api.solve(Ad, Bd, ld, tol=1e-4, max_iter=500, precision=prec, fp64_polish=bench.ACCURACY_MODE,
                     polish_after=bench.POLISH_AFTER)
    Xg = X.cpu().numpy().astype(np.complex128)
    conv = (d["status"].cpu().numpy() & _lib.PX_CONVERGED) != 0
    kg = d["kkt"].cpu().numpy()
    A64, B64, L64, Xe = case["A64"], case["B64"], case["L64"], case["Xe"]
    ko = np.array([orc.kkt_nat(A64, B64[i], L64[i], Xg[i], case["Lf"]) for i in range(len(Xg))])
    Fg = np.array([orc.objective(A64, B64[i], L64[i], Xg[i]) for i in range(len(Xg))])
    gap = (Fg - case["de"]["objective"]) / case["de"]["objective"]
    smax = np.sqrt(case["Lf"] / 2)
    e = np.linalg.norm(Xg - Xe, axis=1) / np.maximum(np.linalg.norm(Xe, axis=1),
                                                     np.linalg.norm(B64, axis=1) / smax)
    passed = conv & (e <= bar)
    geom, meta = case["geom"], case["meta"]
    dg = np.array([detect.detects_pair(Xg[i], geom.s, meta["s1"][i], meta["s2"][i], geom.rayleigh)
                   for i in range(len(Xg))])
    do = np.array([detect.detects_pair(Xe[i], geom.s, meta["s1"][i], meta["s2"][i], geom.rayleigh)
                   for i in range(len(Xe))])
    print(f"solved {conv.mean():.4f}; parity pass {passed.mean():.4f} (e p50 {np.median(e):.1e}, "
          f"p99 {np.percentile(e, 99):.1e}, max {e.max():.1e}); gap max {gap.max():.1e}; "
          f"detections agree {np.mean(dg == do):.4f}")
    assert conv.mean() >= 0.999
    assert np.allclose(kg, ko, rtol=1e-5, atol=1e-9)
    assert (ko[conv] <= 1e-4 * (1 + 1e-5)).all()
    assert gap.min() >= -1e-12 and gap[conv].max() <= bar
    assert passed.mean() >= floor
    assert np.mean(dg == do) >= 0.97
    # the paper's statement at kappa 0.4, 10 dB on the device's profiles
    c04 = [c for c, cs in enumerate(synth.SUPERRES_CASES) if cs == ("profiles", 0.4, 10.0)][0]
    assert dg[meta["case"] == c04].mean() >= 0.8
