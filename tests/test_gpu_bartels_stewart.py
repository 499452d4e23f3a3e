"""GPU tests of the Bartels-Stewart driver (Sec. 1): real Schur forms from SciPy (LAPACK dgees),
the transforms and the robust triangular solve on the device through the C ABI, compared with
SciPy's dense Sylvester solver (an independent library routine) and by the residual of
A X + X B = 2^-e C; sizes span several 64-tiles with ragged tails."""
import numpy as np
import pytest
import scipy.linalg as sla

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_10574_amd as T
    T.lib()
    return T


def _dense(rng, n, shift):
    # eigenvalues near shift (+- about 1), complex pairs included
    return rng.standard_normal((n, n)) / np.sqrt(n) + shift * np.eye(n)


@pytest.mark.parametrize("m,n", [(150, 133), (64, 200), (1, 37)])
def test_bartels_stewart_matches_dense_solver(T, m, n):
    rng = np.random.default_rng(m * 1000 + n)
    A, B = _dense(rng, m, 3.0), _dense(rng, n, 2.0)
    C = rng.standard_normal((m, n))
    At, U = sla.schur(A, output="real")
    Bt, V = sla.schur(B, output="real")
    print(f"  gpu bartels_stewart m={m} n={n} tile=64", flush=True)
    X, e, info = T.bartels_stewart(U, At, V, Bt, C, tile=64)
    X = X.cpu().numpy()
    assert info == 0 and e == 0
    Xr = sla.solve_sylvester(A, B, C)
    assert np.linalg.norm(X - Xr) / np.linalg.norm(Xr) <= 1e-10
    R = A @ X + X @ B - C
    assert np.linalg.norm(R) / (np.linalg.norm(A) + np.linalg.norm(B)) / np.linalg.norm(X) <= 1e-13


def test_bartels_stewart_with_scaling(T):
    """Eigenvalues of A and -B almost meet, so the triangular solve scales: X = 2^e-scaled
    solution, still satisfying A X + X B = 2^-e C to working accuracy."""
    rng = np.random.default_rng(5)
    m = n = 96
    lam = rng.uniform(-1, 1, m) * 1e-150
    At = np.diag(lam) + np.triu(np.ones((m, m)), 1)
    Bt = np.diag(-lam[::-1] + 1e-160) + np.triu(np.ones((n, n)), 1)
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    C = rng.standard_normal((m, n))
    print(f"  gpu bartels_stewart scaling m=n={m} tile=32", flush=True)
    X, e, info = T.bartels_stewart(U, At, V, Bt, C, tile=32)
    X = X.cpu().numpy()
    assert info in (0, 1) and e > 0
    assert np.all(np.isfinite(X)) and np.abs(X).max() <= 2.0 ** 1022
    # residual of the triangular problem, transformed and normalised by 2^-k (|X 2^-k| < 1):
    # Ys = U^T (2^-k X) V solves At Ys + Ys Bt = 2^-(e + k) U^T C V
    k = int(np.frexp(np.abs(X).max())[1])
    Ys = U.T @ np.ldexp(X, -k) @ V
    R = At @ Ys + Ys @ Bt - np.ldexp(U.T @ C @ V, -(e + k))
    den = (np.abs(At).sum(1).max() + np.abs(Bt).sum(0).max()) * np.abs(Ys).sum(1).max()
    assert np.isfinite(den) and den > 0
    assert np.abs(R).sum(1).max() / den <= 1e-13


@pytest.mark.parametrize("m,n", [(0, 4), (5, 0)])
def test_bartels_stewart_empty(T, m, n):
    U, At = np.eye(m), np.eye(m) * 2.0
    V, Bt = np.eye(n), np.eye(n) * 3.0
    X, e, info = T.bartels_stewart(U, At, V, Bt, np.zeros((m, n)))
    assert e == 0 and info == 0 and X.shape == (m, n)


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _oracle_bs(orc, U, At, V, Bt, C, tile):
    """Bartels-Stewart (Sec. 1, eq. (3)) around the oracle's robust triangular solve: Ct = U^T C V,
    At Y + Y Bt = 2^-e Ct by Alg. 4, X = U Y V^T (the orthogonal transforms in plain FP64 NumPy)."""
    Ct = U.T @ C @ V
    Y, e, rc = orc.drsylv(At, Bt, Ct, tile)
    return U @ Y @ V.T, e


def test_bartels_stewart_vs_oracle_separated(T, orc):
    rng = np.random.default_rng(11)
    m, n = 170, 129
    A, B = _dense(rng, m, 3.0), _dense(rng, n, 2.0)
    C = rng.standard_normal((m, n))
    At, U = sla.schur(A, output="real")
    Bt, V = sla.schur(B, output="real")
    print(f"  gpu bartels_stewart vs oracle m={m} n={n}", flush=True)
    X, e, info = T.bartels_stewart(U, At, V, Bt, C, tile=64)
    X = X.cpu().numpy()
    Xo, eo = _oracle_bs(orc, U, At, V, Bt, C, 64)
    assert info == 0 and e == 0 and eo == 0
    assert np.abs(X - Xo).max() <= 1e-10 * np.abs(Xo).max()
    assert np.linalg.norm(X - Xo) <= 1e-10 * np.linalg.norm(Xo)


def test_bartels_stewart_vs_oracle_scaling(T, orc):
    """A case that needs scaling (the eigenvalues of At and -Bt almost meet, strict upper parts of
    ones): both sides return 2^-e times the solution, so the solutions are compared after bringing
    them to the same exponent and normalising by the largest entry."""
    rng = np.random.default_rng(6)
    m, n = 80, 72
    lam = rng.uniform(0.5, 1.0, m) * 1e-3
    At = np.diag(lam) + np.triu(np.ones((m, m)), 1)
    Bt = np.diag(rng.uniform(0.5, 1.0, n) * 1e-3) + np.triu(np.ones((n, n)), 1)
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    C = rng.standard_normal((m, n))
    print(f"  gpu bartels_stewart scaling vs oracle m={m} n={n}", flush=True)
    X, e, info = T.bartels_stewart(U, At, V, Bt, C, tile=32)
    X = X.cpu().numpy()
    Xo, eo = _oracle_bs(orc, U, At, V, Bt, C, 32)
    assert info in (0, 1) and e > 0 and eo > 0
    assert np.all(np.isfinite(X)) and np.all(np.isfinite(Xo))
    # X 2^e and Xo 2^eo represent the same solution: normalise both by the oracle's largest entry
    sg = int(np.frexp(np.abs(X).max())[1])
    so = int(np.frexp(np.abs(Xo).max())[1])
    assert abs((sg + e) - (so + eo)) <= 1
    ng, no = np.ldexp(X, (e - eo) - so), np.ldexp(Xo, -so)
    assert np.linalg.norm(ng - no) / np.linalg.norm(no) <= 1e-8
