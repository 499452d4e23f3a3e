"""GPU tests of the general form op(A) Y + isgn Y op(B) = 2^-e C (trsyl_robust_general) and of
the Lyapunov case A Y + Y A^T = 2^-e C (Sec. 1), all through the C ABI:

  * every combination of op(A), op(B) in {X, X^T} and isgn = +-1 on separated spectra against
    SciPy's dense Bartels-Stewart solver (an independent library routine) to 1e-10, with
    e = 0 and the eq. (9)-style residual of the general equation below 1e-13;
  * the Lyapunov case against SciPy's continuous Lyapunov solver, and Y symmetric for a
    symmetric C;
  * a transposed problem that needs scaling (the paper's test matrices with mu = 1e-3), against
    the oracle on the order-reversed problem (a pure index permutation), normalised, to the
    bound the oracle's own spread between two tile sizes allows.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import trsyl_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_10574_amd as T
    T.lib()
    return T


def _op(X, t):
    return X.T if t == "T" else X


def _resid(A, B, Y, e, C, ta, tb, sg):
    oA, oB = _op(A, ta), _op(B, tb)
    R = oA @ Y + sg * (Y @ oB) - np.ldexp(C, -e)
    den = (np.abs(oA).sum(1).max() + np.abs(oB).sum(0).max()) * np.abs(Y).sum(1).max() + np.abs(np.ldexp(C, -e)).sum(1).max()
    return np.abs(R).sum(1).max() / den


@pytest.mark.parametrize("ta", ["N", "T"])
@pytest.mark.parametrize("tb", ["N", "T"])
@pytest.mark.parametrize("sg", [1, -1])
def test_general_form_matches_dense_solver(T, ta, tb, sg):
    rng = np.random.default_rng(100 + 4 * (ta == "T") + 2 * (tb == "T") + (sg < 0))
    m, n = 150, 133                       # several 64-tiles and ragged tails
    A = W.quasi_triangular(rng, m, p2x2=0.3, upper=("normal", 1.0 / math.sqrt(m)))
    # isgn = -1 takes B with a negative spectrum, so that lambda_A - lambda_B stays away from 0
    diag = ("uniform", 1.0, 10.0) if sg > 0 else ("uniform", -10.0, -1.0)
    B = W.quasi_triangular(rng, n, p2x2=0.3, diag=diag, upper=("normal", 1.0 / math.sqrt(n)))
    C = rng.standard_normal((m, n))
    print(f"  gpu solve_general trana={ta} tranb={tb} isgn={sg} m={m} n={n} tile=64", flush=True)
    Y, e, info = T.solve_general(A, B, C, ta, tb, sg, tile=64)
    Y = Y.cpu().numpy()
    assert info == 0 and e == 0
    X = sla.solve_sylvester(_op(A, ta), sg * _op(B, tb), C)
    assert np.linalg.norm(Y - X) / np.linalg.norm(X) <= 1e-10
    assert _resid(A, B, Y, e, C, ta, tb, sg) <= 1e-13


def test_general_nn_plus_is_the_forward_solve(T):
    A, B, C = W.separated_problem(7, 97, 88)
    Y1, e1, i1 = T.solve(A, B, C, tile=32)
    Y2, e2, i2 = T.solve_general(A, B, C, "N", "N", 1, tile=32)
    assert (e1, i1) == (e2, i2)
    assert np.array_equal(Y1.cpu().numpy(), Y2.cpu().numpy())


def test_lyapunov(T):
    rng = np.random.default_rng(11)
    m = 141
    A = W.quasi_triangular(rng, m, p2x2=0.3, upper=("normal", 1.0 / math.sqrt(m)))
    G = rng.standard_normal((m, m))
    C = G + G.T
    print(f"  gpu lyapunov m={m} tile=64", flush=True)
    Y, e, info = T.lyapunov(A, C, tile=64)
    Y = Y.cpu().numpy()
    assert info == 0 and e == 0
    X = sla.solve_continuous_lyapunov(A, C)
    assert np.linalg.norm(Y - X) / np.linalg.norm(X) <= 1e-10
    assert np.linalg.norm(Y - Y.T) / np.linalg.norm(Y) <= 1e-12
    assert _resid(A, A, Y, e, C, "N", "T", 1) <= 1e-13


def _normalised(Y):
    mx = np.abs(Y).max()
    return np.ldexp(Y, -math.frexp(mx)[1]) if mx else Y.copy()


def test_transposed_problem_with_scaling(T):
    import oracle
    oracle.build(force=False)
    m = n = 200
    A, B, C = W.paper_problem(0, m, n, 1e-3, 1e-2, p2x2=0.1)
    # op(A) = A^T: solve A^T Y + Y B = 2^-e C
    print(f"  gpu solve_general trana=T paper mu=1e-3 nu=1e-2 m=n={m} tile=64", flush=True)
    Y, e, info = T.solve_general(A, B, C, "T", "N", 1, tile=64)
    Y = Y.cpu().numpy()
    assert info == 0 and e > 100
    assert np.all(np.isfinite(Y)) and np.abs(Y).max() <= 2.0 ** 1022
    # the order-reversed problem (P A^T P) (P Y) + (P Y) B = 2^-e P C, solved by the oracle
    Ah = A.T[::-1, ::-1].copy()
    Yh, eo, _ = oracle.drsylv(Ah, B, C[::-1, :].copy(), 64)
    Yh2, _, _ = oracle.drsylv(Ah, B, C[::-1, :].copy(), 32)
    Yo, Yo2 = Yh[::-1, :], Yh2[::-1, :]
    spread = np.linalg.norm(_normalised(Yo2) - _normalised(Yo)) / np.linalg.norm(_normalised(Yo))
    err = np.linalg.norm(_normalised(Y) - _normalised(Yo)) / np.linalg.norm(_normalised(Yo))
    print(f"    e_gpu={e} e_orc={eo} err={err:.2e} oracle spread={spread:.2e}")
    assert err <= max(1e-8, 100 * spread)


@pytest.mark.parametrize("m,n", [(0, 5), (6, 0), (0, 0)])
def test_general_form_empty(T, m, n):
    A = np.eye(m) * 2.0
    B = np.eye(n) * 3.0
    C = np.zeros((m, n))
    Y, e, info = T.solve_general(A, B, C, "T", "T", -1)
    assert e == 0 and info == 0 and Y.shape == (m, n)


def test_general_form_precision_form(T):
    """The general form passes the options through: the FP32-update + FP64-refinement form on a
    transposed, negative-sign problem reaches the dense solver's solution to 1e-10."""
    rng = np.random.default_rng(21)
    m, n = 140, 120
    A = W.quasi_triangular(rng, m, p2x2=0.3, upper=("normal", 1.0 / math.sqrt(m)))
    B = W.quasi_triangular(rng, n, p2x2=0.3, diag=("uniform", -10.0, -1.0), upper=("normal", 1.0 / math.sqrt(n)))
    C = rng.standard_normal((m, n))
    print(f"  gpu solve_general fp32_refine trana=T tranb=N isgn=-1 m={m} n={n}", flush=True)
    Y, e, info = T.solve_general(A, B, C, "T", "N", -1, tile=64, precision="fp32_refine")
    Y = Y.cpu().numpy()
    assert info == 0 and e == 0
    X = sla.solve_sylvester(A.T, -B, C)
    assert np.linalg.norm(Y - X) / np.linalg.norm(X) <= 1e-10
