"""GPU checks at the configurations' full sizes, in the launch configuration the benchmark times
(default options: tile 128, persistent DAG scheduler).  The oracle cannot solve these sizes
within a test, so the checks are properties that hold at any size, evaluated by the oracle where
it can: exact (long double) residual rows on a seeded sample of rows, the invariants of the robust
method (finite, bounded by Omega, alpha < 1 on growth inputs), and the device eq. (9).
"""
import numpy as np
import pytest

import oracle
import trsyl_workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
OMEGA = 2.0 ** 1022


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1905_10574_amd as T
    T.lib()
    return T


def _sampled_rows_check(A, B, Y, e, C, nrows=24, seed=0, tol=1e-13):
    """Per-row eq. (9) on sampled rows, in long double by the oracle, with Y and alpha scaled by
    the power of two at or above max |Y|."""
    m, n = Y.shape
    ymax = np.abs(Y).max()
    shift = int(np.frexp(ymax)[1]) if ymax > 0 else 0
    rows = np.sort(np.random.default_rng(seed).choice(m, size=min(nrows, m), replace=False))
    rr, yy, cc = oracle.residual_rows(A, B, Y, e, C, rows, shift)
    nA = np.linalg.norm(np.triu(A, -1))
    nB = np.linalg.norm(np.triu(B, -1))
    q = np.sqrt(rr) / ((nA + nB) * np.sqrt(yy) + np.sqrt(cc))
    assert q <= tol, q


def test_separated_8192(T):
    A, B, C = W.config_separated(0)
    Y, e, info = T.solve(A, B, C)
    assert info == 0 and e == 0
    assert T.residual(A, B, Y, e, C) <= 1e-13
    Yn = Y.cpu().numpy()
    assert np.all(np.isfinite(Yn))
    _sampled_rows_check(A, B, Yn, e, C)


@pytest.mark.parametrize("tile", [256, 128])
def test_growth_4096(T, tile):
    A, B, C = W.config_growth(0)
    Y, e, info = T.solve(A, B, C, tile=tile)
    assert info in (0, 1) and e > 0
    Yn = Y.cpu().numpy()
    assert np.all(np.isfinite(Yn)) and np.abs(Yn).max() <= OMEGA
    # every tile's infinity norm within Omega (row sums of each tile)
    t = tile
    for r0 in range(0, Yn.shape[0], t):
        for c0 in range(0, Yn.shape[1], 4 * t):
            blk = np.abs(Yn[r0:r0 + t + 1, c0:c0 + 4 * t])
            assert np.all(blk.sum(axis=1) <= 4 * OMEGA)
    assert T.residual(A, B, Y, e, C) <= 1e-13
    _sampled_rows_check(A, B, Yn, e, C)


def test_batched_256(T):
    probs = W.config_batched(0)
    As = [p[1] for p in probs]
    Bs = [p[2] for p in probs]
    Cs = [p[3] for p in probs]
    out = T.solve_batched(As, Bs, Cs)
    for (kind, A, B, C), (Y, e, info) in zip(probs, out):
        assert info in (0, 1)
        if kind == "growth" and min(C.shape) >= 512:
            assert e > 0
        if kind == "separated":
            assert e == 0
        assert T.residual(A, B, Y, e, C) <= 1e-13


def test_adjoint_32(T):
    probs = W.config_adjoint(0)
    for i, (A, B, C, Wm) in enumerate(probs):
        G, e, info = T.adjoint(A, B, Wm)
        assert info == 0 and e == 0
        G = G.cpu().numpy()
        R = A.T @ G + G @ B.T - Wm
        q = np.linalg.norm(R) / ((np.linalg.norm(A) + np.linalg.norm(B)) * np.linalg.norm(G) + np.linalg.norm(Wm))
        assert q <= 1e-13, (i, q)
