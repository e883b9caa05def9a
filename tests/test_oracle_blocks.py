"""Pins of the oracle's Algorithm 1 with J blocks (Eqs. (13)-(14)).

Each pin is fixed by something other than the oracle's own code: J = 1 is the
one-block algorithm (already pinned elsewhere) bit for bit; the block Lipschitz
constants are numpy's eigenvalues of the block Gram; the block draw follows the
distribution of Eq. (14) (exact boundaries, and frequencies over many draws);
with orthonormal columns and one column per block the minimiser is the closed
form; on small problems the iterates reach the certified minimiser, and the
objective never increases (the monotone step of Algorithm 1).
"""
import numpy as np
import pytest

import oracle
from paper_1805_01759_amd import synth


@pytest.fixture(scope="module")
def tiny():
    spec, geom, B, lam = synth.make_config(1, 0, 24)
    return geom.A, B, lam


def test_one_block_is_algorithm_1(tiny):
    A, B, lam = tiny
    u = np.random.default_rng(5).random(600)
    for p in range(6):
        x1, i1 = oracle.rbpg(A, B[p], lam[p], max_iter=600)
        x2, i2 = oracle.rbpg_blocks(A, B[p], lam[p], 1, u, max_iter=600)
        assert np.array_equal(x1, x2) and i1["iters"] == i2["iters"]


@pytest.mark.parametrize("J", [1, 2, 3, 5, 7])
def test_block_lipschitz_against_eigvalsh(tiny, J):
    A = tiny[0]
    l = A.shape[1]
    w = -(-l // J)
    Lb = oracle.block_lipschitz(A, J)
    for j in range(J):
        Aj = A[:, j * w:min(l, (j + 1) * w)]
        want = 2 * np.linalg.eigvalsh(Aj @ Aj.conj().T).max() if Aj.shape[1] else 0.0
        assert abs(Lb[j] - want) <= 1e-10 * want


def test_block_draw_distribution():
    Lb = np.array([3.0, 1.0, 4.0, 2.0])
    c = np.cumsum(Lb) / Lb.sum()
    # exact boundaries: u at a cumulative boundary selects the next block
    assert oracle.block_pick(Lb, 0.0) == 0
    assert [oracle.block_pick(Lb, v) for v in c[:-1]] == [1, 2, 3]
    assert [oracle.block_pick(Lb, np.nextafter(v, 0)) for v in c[:-1]] == [0, 1, 2]
    assert oracle.block_pick(Lb, np.nextafter(1.0, 0)) == 3
    u = np.random.default_rng(11).random(200000)
    f = np.bincount([oracle.block_pick(Lb, v) for v in u[:40000]], minlength=4) / 40000
    assert np.allclose(f, Lb / Lb.sum(), atol=0.01)


def test_orthonormal_one_column_blocks():
    rng = np.random.default_rng(7)
    n, l = 12, 8
    Q, _ = np.linalg.qr(rng.standard_normal((n, l)) + 1j * rng.standard_normal((n, l)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lam = 0.9
    v = Q.conj().T @ b
    want = np.where(np.abs(v) > lam / 2, v * (1 - (lam / 2) / np.maximum(np.abs(v), 1e-300)), 0)
    u = rng.random(4000)
    x, info = oracle.rbpg_blocks(Q, b, lam, l, u, tol=1e-12, max_iter=4000)
    assert info["converged"]
    assert np.abs(x - want).max() <= 1e-9


@pytest.mark.parametrize("J", [2, 3, 5])
def test_reaches_the_certified_minimiser(tiny, J):
    A, B, lam = tiny
    u = np.random.default_rng(13).random(30000)
    X, d = oracle.rbpg_blocks_batch(A, B[:8], lam[:8], J, u, tol=1e-7, max_iter=30000)
    Xe, de = oracle.exact_batch(A, B[:8], lam[:8])
    F = np.array([oracle.objective(A, B[p], lam[p], X[p]) for p in range(8)])
    assert d["converged"].all()
    assert ((F - de["objective"]) / np.maximum(de["objective"], 1.0)).max() <= 1e-8


def test_objective_never_increases(tiny):
    A, B, lam = tiny
    u = np.random.default_rng(17).random(200)
    for p in range(3):
        F = []
        for k in range(1, 60):
            x, _ = oracle.rbpg_blocks(A, B[p], lam[p], 4, u, tol=1e-30, max_iter=k)
            F.append(oracle.objective(A, B[p], lam[p], x))
        assert all(F[i + 1] <= F[i] * (1 + 1e-14) for i in range(len(F) - 1))
