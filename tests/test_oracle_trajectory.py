"""Pin of the oracle's Algorithm 1 step sequence against a hand-derived trajectory.

tests/golden/algorithm1_trajectory.txt holds six iterations of Algorithm 1 (one
block) on a 2 x 2 real problem, derived by hand in exact rational arithmetic:
the extrapolation weights of Eqs. (11)-(12), the carried and shrunk step of
Eq. (15) with its 1/L_f floor, and one monotone reject.  The oracle's one-block
algorithm and its J-block form with J = 1 must reproduce every iterate, step
and objective; a reading that differs in any of these (another beta sequence,
a step restarted from alpha_0 every iteration, no reject) changes an iterate.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

A_G = np.array([[-2.0, -2.0], [-2.0, 1.0]], dtype=np.complex128)
B_G = np.array([6.0, -3.0], dtype=np.complex128)
LAM_G = 2.0
LF_G = 18.0


def golden_rows():
    path = os.path.join(os.path.dirname(__file__), "golden", "algorithm1_trajectory.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, beta, alpha, shr, acc, x1, x2, F = line.split()
        rows.append(dict(k=int(k), beta=Fraction(beta), alpha=Fraction(alpha), shrinks=int(shr),
                         accepted=bool(int(acc)), x=(Fraction(x1), Fraction(x2)), F=Fraction(F)))
    return rows


def test_golden_constants(orc):
    """The stated L_f, alpha_0 and minimiser of the golden problem."""
    assert abs(orc.lipschitz(A_G) - LF_G) < 1e-12
    assert np.allclose((np.abs(A_G) ** 2).sum(0), [8.0, 5.0])
    x, info = orc.rbpg(A_G, B_G, LAM_G, tol=1e-13, max_iter=2000, Lf=LF_G)
    assert np.allclose(x, [0.0, -14.0 / 5.0], atol=1e-10)
    assert abs(info["objective"] - 29.0 / 5.0) < 1e-10


def test_golden_self_consistent():
    """Each data row agrees with its own columns: beta_k = max(0, (k-2)/(k+1)), F = f + lambda |x|_1
    for the stated iterate, the objective never increases, and a reject repeats the iterate."""
    rows = golden_rows()
    assert [r["k"] for r in rows] == list(range(1, 7))
    prevF, prevx = Fraction(45), (Fraction(0), Fraction(0))
    A = [[Fraction(-2), Fraction(-2)], [Fraction(-2), Fraction(1)]]
    b = (Fraction(6), Fraction(-3))
    for r in rows:
        assert r["beta"] == max(Fraction(0), Fraction(r["k"] - 2, r["k"] + 1))
        x = r["x"]
        res = [A[i][0] * x[0] + A[i][1] * x[1] - b[i] for i in range(2)]
        F = res[0] ** 2 + res[1] ** 2 + 2 * (abs(x[0]) + abs(x[1]))
        assert F == r["F"]
        assert F <= prevF
        if not r["accepted"]:
            assert x == prevx
        prevF, prevx = F, x
    assert any(not r["accepted"] for r in rows)
    assert any(r["shrinks"] > 0 for r in rows)


def _check_against_golden(run):
    backtracks = 0
    for r in golden_rows():
        x, info = run(r["k"])
        backtracks += r["shrinks"]
        assert np.abs(x.imag).max() == 0.0, r["k"]
        assert np.allclose(x.real, [float(v) for v in r["x"]], rtol=1e-13, atol=1e-15), (r["k"], x)
        assert abs(info["alpha"] - float(r["alpha"])) <= 1e-15, (r["k"], info["alpha"])
        assert info["backtracks"] == backtracks, (r["k"], info["backtracks"])
        assert abs(info["objective"] - float(r["F"])) <= 1e-13 * float(r["F"]), r["k"]


def test_rbpg_matches_golden_trajectory(orc):
    """Algorithm 1 (J = 1) stopped after k iterations equals the hand-derived x^k."""
    _check_against_golden(lambda k: orc.rbpg(A_G, B_G, LAM_G, tol=1e-300, max_iter=k, Lf=LF_G))


def test_rbpg_blocks_j1_matches_golden_trajectory(orc):
    """The J-block form with J = 1 follows the same hand-derived trajectory."""
    u = np.full(8, 0.5)
    _check_against_golden(lambda k: orc.rbpg_blocks(A_G, B_G, LAM_G, 1, u, tol=1e-300, max_iter=k,
                                                    Lf=LF_G))


@pytest.mark.parametrize("phi", [0.7, -2.1])
def test_rbpg_golden_phase_equivariance(orc, phi):
    """A real: b -> e^{j phi} b rotates every iterate by e^{j phi} (complex prox of Eq. (10))."""
    rot = np.exp(1j * phi)
    for r in golden_rows():
        x, info = orc.rbpg(A_G, B_G * rot, LAM_G, tol=1e-300, max_iter=r["k"], Lf=LF_G)
        want = np.array([float(v) for v in r["x"]]) * rot
        assert np.allclose(x, want, rtol=1e-12, atol=1e-14), (r["k"], x, want)
        assert abs(info["objective"] - float(r["F"])) <= 1e-12 * float(r["F"])


def warm_rows():
    path = os.path.join(os.path.dirname(__file__), "golden", "algorithm1_warm_start.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, beta, alpha, shr, acc, x1, x2, F = line.split()
        rows.append(dict(k=int(k), alpha=Fraction(alpha), x=(Fraction(x1), Fraction(x2)), F=Fraction(F)))
    return rows


def test_rbpg_warm_start_matches_golden(orc):
    """Algorithm 1 from a given x^(0): the hand-derived first two iterates, steps and objectives
    (tests/golden/algorithm1_warm_start.txt); from the minimiser it stops at once, unchanged."""
    rows = warm_rows()
    x0 = np.array([float(v) for v in rows[0]["x"]], dtype=np.complex128)
    for r in rows[1:]:
        x, info = orc.rbpg(A_G, B_G, LAM_G, tol=1e-300, max_iter=r["k"], Lf=LF_G, x0=x0)
        assert np.allclose(x.real, [float(v) for v in r["x"]], rtol=1e-13, atol=1e-15), (r["k"], x)
        assert np.abs(x.imag).max() == 0.0
        assert abs(info["alpha"] - float(r["alpha"])) <= 1e-15
        assert abs(info["objective"] - float(r["F"])) <= 1e-13 * float(r["F"])
    xs = np.array([0.0, -14.0 / 5.0], dtype=np.complex128)
    x, info = orc.rbpg(A_G, B_G, LAM_G, tol=1e-8, max_iter=50, Lf=LF_G, x0=xs)
    assert info["iters"] == 0 and np.array_equal(x, xs)
    # the batch form reads its X0 rows the same way
    X, d = orc.rbpg_batch(A_G, np.stack([B_G, B_G]), LAM_G, tol=1e-300, max_iter=2,
                          X0=np.stack([x0, x0]))
    assert np.allclose(X.real, [[float(v) for v in rows[2]["x"]]] * 2, rtol=1e-13, atol=1e-15)
