"""Counting double-scatterer detections in reconstructed elevation profiles.

The paper reports detection rates of two close scatterers (simulation with
N = 29, phase difference 0, per-scatterer SNR 2 dB and 7 dB) but the model
selection that decides "detected" belongs to the surrounding SL1MMER
framework and is not defined in the paper.  The rule here is this package's
own, stated so that it can be checked: a profile's support splits into
clusters (maximal runs of adjacent nonzero bins: a scatterer between two grid
points occupies both); a cluster's weight is the sum of |x| over it and its
position the |x|-weighted mean elevation; clusters lighter than 10% of the
heaviest are dropped; the pair counts as detected when two clusters remain
and the two heaviest lie on opposite sides of the midpoint of the true pair,
each within half a resolution cell (rho_s / 2) of its true elevation.  (The
L1 minimiser places resolved close peaks slightly apart from the truth, so
the positions are not held to a tighter window.)
"""
from __future__ import annotations

import numpy as np

MIN_WEIGHT = 0.1


def clusters(x: np.ndarray, s: np.ndarray):
    """(weights, positions) of the runs of adjacent nonzero bins of x, heaviest first."""
    mag = np.abs(np.asarray(x))
    nz = mag > 0
    out_w, out_p = [], []
    m, L = 0, len(mag)
    while m < L:
        if not nz[m]:
            m += 1
            continue
        e = m
        while e < L and nz[e]:
            e += 1
        w = float(mag[m:e].sum())
        out_w.append(w)
        out_p.append(float((mag[m:e] * s[m:e]).sum() / w))
        m = e
    order = np.argsort(out_w)[::-1]
    return np.array(out_w)[order], np.array(out_p)[order]


def detects_pair(x: np.ndarray, s: np.ndarray, s1: float, s2: float, rho: float) -> bool:
    w, p = clusters(x, s)
    if len(w) < 2:
        return False
    keep = w >= MIN_WEIGHT * w[0]
    w, p = w[keep], p[keep]
    if len(w) < 2:
        return False
    lo, hi = sorted(p[:2])
    t1, t2 = sorted((s1, s2))
    mid = 0.5 * (t1 + t2)
    return lo < mid < hi and abs(lo - t1) <= rho / 2.0 and abs(hi - t2) <= rho / 2.0


def detection_rate(X: np.ndarray, s: np.ndarray, s1, s2, rho: float) -> float:
    X = np.asarray(X)
    s1 = np.broadcast_to(s1, (len(X),))
    s2 = np.broadcast_to(s2, (len(X),))
    return float(np.mean([detects_pair(X[i], s, s1[i], s2[i], rho) for i in range(len(X))]))
