"""Pins for the oracle's scalar primitives and structure scan (Sec. 2.1, Sec. 1 eq. (4)).

ProtectUpdate / ProtectDivision are checked against their contracts in exact rational
arithmetic (fractions.Fraction), so a wrong exponent, a dropped term or an off-by-one in either
direction fails here.  The small solve is checked against closed forms (1x1 division, Cramer's
rule) and an independently formed Kronecker system solved by LAPACK.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

OMEGA = Fraction(2) ** 1022
EDGE = [0.0, 2.0 ** -1074, 2.0 ** -1060, 2.0 ** -1022, 1e-300, 0.5, 0.75, 1.0, 1.5, 3.0, 2.0 ** 100,
        1e200, 2.0 ** 511, 2.0 ** 512 * 1.5, 2.0 ** 1000, 2.0 ** 1021, 2.0 ** 1022 * 0.75, 2.0 ** 1022]


def _exact_ok(s, c, a, y):
    return Fraction(1, 2 ** s) * (Fraction(c) + Fraction(a) * Fraction(y)) <= OMEGA


def test_protect_update_contract_and_minimality(orc):
    rng = np.random.default_rng(7)
    vals = list(EDGE) + [float(x) for x in 2.0 ** rng.uniform(-1074, 1022, 40)]
    checked = 0
    for c in vals[::2] + [0.0, 2.0 ** 1022]:
        for a in vals:
            for y in vals[::3] + [2.0 ** 1022]:
                s = orc.protect_update(c, a, y)
                assert s >= 0
                assert _exact_ok(s, c, a, y), (c, a, y, s)
                if s > 0:
                    g = Fraction(c) + Fraction(a) * Fraction(y)
                    # one power of two less would violate the bound, unless g sits in the
                    # documented 2^-51 guard band just below the threshold
                    larger = Fraction(1, 2 ** (s - 1)) * g
                    assert larger > OMEGA or larger * (1 + Fraction(1, 2 ** 51)) > OMEGA
                checked += 1
    assert checked > 1000


def test_protect_update_simple_values(orc):
    assert orc.protect_update(0.0, 0.0, 0.0) == 0
    assert orc.protect_update(1.0, 1.0, 1.0) == 0
    assert orc.protect_update(2.0 ** 1022, 0.0, 5.0) == 0
    # Omega + Omega*1 = 2 Omega -> one halving
    assert orc.protect_update(2.0 ** 1022, 1.0, 2.0 ** 1022) == 1
    # a*y = 2^1022 * 2^1022 = 2^2044 -> need 2^-1022 exactly (plus nothing for c = 0)
    assert orc.protect_update(0.0, 2.0 ** 1022, 2.0 ** 1022) == 1022
    # 3 * 2^1021 > 2^1022 -> s = 1 ; 1.5*2^1021 + tiny: (1.5 2^1021) <= 2^1022 -> s = 0
    assert orc.protect_update(0.0, 3.0, 2.0 ** 1021) == 1
    assert orc.protect_update(0.0, 1.5, 2.0 ** 1021) == 0


def test_protect_division_contract_and_minimality(orc):
    rng = np.random.default_rng(11)
    bs = list(EDGE) + [float(x) for x in 2.0 ** rng.uniform(-1074, 1022, 30)]
    ts = [2.0 ** -1074, 2.0 ** -1073 * 3, 2.0 ** -1022, 1e-300, 1e-20, 0.3, 0.5, 0.999, 1.0, 2.0, 1e300]
    for b in bs:
        for t in ts:
            for sb in (1.0, -1.0):
                for st in (1.0, -1.0):
                    s = orc.protect_division(sb * b, st * t)
                    assert s >= 0
                    lhs = Fraction(1, 2 ** s) * abs(Fraction(b))
                    assert lhs <= abs(Fraction(t)) * OMEGA
                    if s > 0:
                        assert 2 * lhs > abs(Fraction(t)) * OMEGA
                    # the guarded quotient is finite and within Omega after rounding
                    q = math.ldexp(sb * b, -s) / (st * t)
                    assert math.isfinite(q) and abs(q) <= 2.0 ** 1022


def test_block_starts_and_malformed(orc):
    T = np.loadtxt(_golden("paper_example_5x5.txt"))
    assert orc.block_starts(T) == [0, 1, 2, 4]
    bad = np.triu(np.ones((4, 4)))
    bad[1, 0] = 1.0
    bad[2, 1] = 1.0
    with pytest.raises(ValueError):
        orc.block_starts(bad)


def _golden(name):
    import os
    return os.path.join(os.path.dirname(__file__), "golden", name)


def test_paper_example_eigenvalues():
    """Sec. 3: the 5x5 example has eigenvalues mu, mu, mu(1+i), mu(1-i), mu (mu = 1 here);
    the fixture file holds the matrix and the eigenvalues the paper prints."""
    T = np.loadtxt(_golden("paper_example_5x5.txt"))
    ev = np.sort_complex(np.linalg.eigvals(T))
    want = np.sort_complex(np.array([1, 1, 1 + 1j, 1 - 1j, 1]))
    assert np.allclose(ev, want, atol=1e-7)


def test_tile_offsets_never_split_2x2(orc):
    T = np.triu(np.ones((10, 10)))
    # 2x2 block at rows 3,4 : boundary 4 (t=4) must move to 5; 2x2 at 7,8: boundary 8 -> 9
    T[4, 3] = -1.0
    T[8, 7] = -1.0
    assert orc.tile_offsets(T, 4) == [0, 5, 9, 10]
    assert orc.tile_offsets(T, 2) == [0, 2, 5, 6, 9, 10]
    assert orc.tile_offsets(T, 100) == [0, 10]
    # boundary pushed onto n: single tile
    U = np.triu(np.ones((5, 5)))
    U[4, 3] = 2.0
    assert orc.tile_offsets(U, 4) == [0, 5]


def _kron_solve(A11, B11, R):
    r, c = A11.shape[0], B11.shape[0]
    K = np.kron(np.eye(c), A11) + np.kron(B11.T, np.eye(r))
    return np.linalg.solve(K, R.reshape(-1, order="F")).reshape((r, c), order="F")


@pytest.mark.parametrize("r,c", [(1, 1), (2, 1), (1, 2), (2, 2)])
def test_small_solve_matches_kronecker(orc, r, c):
    rng = np.random.default_rng(100 + 10 * r + c)
    for _ in range(50):
        A11 = rng.uniform(1, 10, (r, r))
        B11 = rng.uniform(1, 10, (c, c))
        if r == 2:
            A11 = np.array([[A11[0, 0], 1.3], [-0.7, A11[0, 0]]])
        if c == 2:
            B11 = np.array([[B11[0, 0], -0.9], [1.8, B11[0, 0]]])
        R = rng.standard_normal((r, c))
        Z, sb, pert = orc.small_solve(A11, B11, R)
        assert sb == 0 and pert == 0
        assert np.allclose(Z, _kron_solve(A11, B11, R), rtol=1e-13, atol=1e-15)


def test_small_solve_closed_forms(orc):
    # 1x1: z = r / (a + b)
    Z, sb, _ = orc.small_solve(np.array([[3.0]]), np.array([[5.0]]), np.array([[2.0]]))
    assert sb == 0 and Z[0, 0] == 0.25
    # 2x1: (A + b I) z = r by Cramer's rule
    A11 = np.array([[2.0, 3.0], [-1.0, 2.0]])
    b = 1.5
    rr = np.array([1.0, -2.0])
    M = A11 + b * np.eye(2)
    det = M[0, 0] * M[1, 1] - M[0, 1] * M[1, 0]
    z0 = (rr[0] * M[1, 1] - M[0, 1] * rr[1]) / det
    z1 = (M[0, 0] * rr[1] - rr[0] * M[1, 0]) / det
    Z, sb, _ = orc.small_solve(A11, np.array([[b]]), rr.reshape(2, 1))
    assert np.allclose(Z[:, 0], [z0, z1], rtol=1e-15)
    # 1x2: z (a I + B) = r  (row vector), Cramer on the transposed 2x2
    a = 0.5
    B11 = np.array([[1.0, 2.0], [-3.0, 1.0]])
    M = (a * np.eye(2) + B11).T
    det = M[0, 0] * M[1, 1] - M[0, 1] * M[1, 0]
    rr = np.array([4.0, 1.0])
    z0 = (rr[0] * M[1, 1] - M[0, 1] * rr[1]) / det
    z1 = (M[0, 0] * rr[1] - rr[0] * M[1, 0]) / det
    Z, sb, _ = orc.small_solve(np.array([[a]]), B11, rr.reshape(1, 2))
    assert np.allclose(Z[0], [z0, z1], rtol=1e-15)


def test_small_solve_scales_instead_of_overflowing(orc):
    # |r| = Omega-ish and a + b tiny: the plain quotient overflows, the robust one scales
    big = 2.0 ** 1021
    Z, sb, pert = orc.small_solve(np.array([[1e-300]]), np.array([[1e-300]]), np.array([[big]]))
    assert sb > 0 and np.isfinite(Z).all() and abs(Z[0, 0]) <= 2.0 ** 1022
    beta = Fraction(1, 2 ** sb)
    # (a + b) z == beta r to rounding
    lhs = Fraction(2e-300) * Fraction(Z[0, 0])
    assert abs(lhs - beta * Fraction(big)) <= abs(beta * Fraction(big)) * Fraction(1, 2 ** 50)
    # 2x2 with tiny spectrum sum and large rhs
    A11 = np.array([[1e-200, 1e-200], [-1e-200, 1e-200]])
    B11 = np.array([[3e-200, 1e-200], [-2e-200, 3e-200]])
    R = np.array([[2.0 ** 1020, -2.0 ** 1019], [2.0 ** 1018, 2.0 ** 1021]])
    Z, sb, pert = orc.small_solve(A11, B11, R)
    assert sb > 0 and np.isfinite(Z).all()
    assert np.abs(Z).sum(axis=1).max() <= 2.0 ** 1022
    # scaled back to unit size, the defining equation holds
    Zs = Z * 2.0 ** -900
    Rs = np.ldexp(R, -sb - 900)
    resid = A11 @ Zs + Zs @ B11 - Rs
    assert np.abs(Rs).max() > 0
    assert np.abs(resid).max() <= 1e-14 * np.abs(Rs).max()


def test_small_solve_singular_pair_is_perturbed(orc):
    """Eigenvalues of mu*[[1,1],[-1,1]] are mu(1 +- i) (Sec. 3); with B11 = -A11 they cancel,
    lambda_A + lambda_B = 0, the uniqueness condition of Sec. 1 fails and the pivot floor
    must be applied."""
    mu = 3.0
    A11 = mu * np.array([[1.0, 1.0], [-1.0, 1.0]])
    Z, sb, pert = orc.small_solve(A11, -A11, np.ones((2, 2)), smin=1e-12)
    assert pert == 1 and np.isfinite(Z).all()
    Z, sb, pert = orc.small_solve(A11, A11, np.ones((2, 2)), smin=1e-12)
    assert pert == 0
