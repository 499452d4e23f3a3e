"""Seeded synthetic inputs for the triangular Sylvester solve A Y + Y B = alpha C.

This module only draws random matrices; it holds none of the solver's arithmetic.  Both the
GPU library's tests/benchmark and the CPU oracle's tests take their inputs from here.

All matrices are float64 numpy arrays in column-major (Fortran) order.  A and B are upper
quasi-triangular: the diagonal is a sequence of 1x1 and 2x2 blocks, a 2x2 block being marked
by a nonzero first-subdiagonal entry (the shape of a real Schur form, Sec. 1, eq. (4)).

Draw order for one quasi-triangular matrix of order n (fixed, so a seed fixes the matrix):
  1. u = random(n)              -- block pattern: at row i, a 2x2 block starts if u[i] < p2x2
                                   and i+1 < n (walking down the diagonal), else a 1x1 block
  2. d = diagonal draws (n)      -- 1x1 value, or the common diagonal a of a 2x2 block
  3. bm = uniform(0.5, 2, n)     -- |b| of a 2x2 block [[a, b], [c, a]]
  4. cm = uniform(0.5, 2, n)     -- |c|
  5. sg = random(n) < 0.5        -- sign: b = +|b|, c = -|c| if sg else b = -|b|, c = +|c|
  6. U  = the full n x n strictly-upper draw (only the strict upper triangle is kept)
A 2x2 block [[a, b], [c, a]] with b*c < 0 has the complex pair a +- i*sqrt(|b c|).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "quasi_triangular", "separated_problem", "growth_problem", "paper_problem",
    "config_small", "config_growth", "config_separated", "config_batched",
    "config_adjoint", "block_starts", "flop_count",
]


def flop_count(m: int, n: int) -> float:
    """Nominal flop count m^2 n + m n^2 of one solve (Sec. 1: two backward substitutions)."""
    return float(m) * m * n + float(m) * n * n


def _walk_blocks(u: np.ndarray, p2x2: float) -> list[tuple[int, int]]:
    n = len(u)
    blocks, i = [], 0
    while i < n:
        if i + 1 < n and u[i] < p2x2:
            blocks.append((i, 2))
            i += 2
        else:
            blocks.append((i, 1))
            i += 1
    return blocks


def quasi_triangular(rng: np.random.Generator, n: int, *, p2x2: float,
                     diag=("uniform", 1.0, 10.0), upper=("normal", 1.0)) -> np.ndarray:
    """Random upper quasi-triangular matrix, drawn in the documented order."""
    u = rng.random(n)
    if diag[0] == "uniform":
        d = rng.uniform(diag[1], diag[2], n)
    elif diag[0] == "given":
        d = np.asarray(diag[1], dtype=np.float64)
        assert d.shape == (n,)
    else:
        raise ValueError(diag)
    bm = rng.uniform(0.5, 2.0, n)
    cm = rng.uniform(0.5, 2.0, n)
    sg = rng.random(n) < 0.5
    if upper[0] == "normal":
        U = rng.standard_normal((n, n)) * upper[1]
    elif upper[0] == "uniform":
        U = rng.uniform(-upper[1], upper[1], (n, n))
    elif upper[0] == "ones":
        U = np.ones((n, n))
    else:
        raise ValueError(upper)
    T = np.triu(U, 1)
    for (i, sz) in _walk_blocks(u, p2x2):
        T[i, i] = d[i]
        if sz == 2:
            b = bm[i] if sg[i] else -bm[i]
            c = -cm[i] if sg[i] else cm[i]
            T[i + 1, i + 1] = d[i]
            T[i, i + 1] = b
            T[i + 1, i] = c
    return np.asfortranarray(T)


def block_starts(T: np.ndarray) -> list[int]:
    """Row indices where diagonal blocks start (a nonzero subdiagonal opens a 2x2 block)."""
    n = T.shape[0]
    out, i = [], 0
    while i < n:
        out.append(i)
        i += 2 if (i + 1 < n and T[i + 1, i] != 0.0) else 1
    return out


def separated_problem(seed, m: int, n: int, *, p2x2: float = 0.2, upper_scale: str = "sqrt",
                      c_dist: str = "normal"):
    """Well-separated spectra: diagonals U[1,10] (so |lambda_A + lambda_B| >= 2)."""
    rng = np.random.default_rng(seed)
    sa = 1.0 / np.sqrt(m) if upper_scale == "sqrt" else 1.0
    sb = 1.0 / np.sqrt(n) if upper_scale == "sqrt" else 1.0
    A = quasi_triangular(rng, m, p2x2=p2x2, upper=("normal", sa))
    B = quasi_triangular(rng, n, p2x2=p2x2, upper=("normal", sb))
    if c_dist == "normal":
        C = rng.standard_normal((m, n))
    else:
        C = rng.uniform(-1.0, 1.0, (m, n))
    return A, B, np.asfortranarray(C)


def growth_problem(seed, m: int, n: int):
    """Growth case: all 1x1 blocks, lambda_A ~ U[-1,1]*1e-2, and lambda_B_j = -lambda_A_(j mod m)
    + s_j u_j with s_j = +-1 and u_j ~ U[1e-3, 1e-2], so each paired sum has modulus in
    [1e-3, 1e-2].  Strict upper parts U[-10,10]; C ~ U[-1,1]."""
    rng = np.random.default_rng(seed)
    la = rng.uniform(-1.0, 1.0, m) * 1e-2
    A = quasi_triangular(rng, m, p2x2=0.0, diag=("given", la), upper=("uniform", 10.0))
    uj = rng.uniform(1e-3, 1e-2, n)
    sj = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    lb = -la[np.arange(n) % m] + sj * uj
    B = quasi_triangular(rng, n, p2x2=0.0, diag=("given", lb), upper=("uniform", 10.0))
    C = rng.uniform(-1.0, 1.0, (m, n))
    return A, B, np.asfortranarray(C)


def paper_problem(seed, m: int, n: int, mu: float, nu: float, p2x2: float = 0.0):
    """Sec. 3 test matrices: C and the strict upper parts are ones; diagonal blocks are mu*T
    (resp. nu*T) with T = [1] or [[1, 1], [-1, 1]].  The paper leaves the 1x1/2x2 pattern
    open; here a 2x2 block starts with probability p2x2 while walking down the diagonal."""
    rng = np.random.default_rng(seed)

    def make(k, s):
        u = rng.random(k)
        T = np.triu(np.ones((k, k)), 1)
        for (i, sz) in _walk_blocks(u, p2x2):
            T[i, i] = s
            if sz == 2:
                T[i + 1, i + 1] = s
                T[i, i + 1] = s
                T[i + 1, i] = -s
        return np.asfortranarray(T)

    A = make(m, mu)
    B = make(n, nu)
    return A, B, np.asfortranarray(np.ones((m, n)))


# ---- named workloads -------------------------------------------------------------------

def config_small(seed):
    """m = n = 64, 30% 2x2 blocks, diagonal U[1,10], strict upper N(0,1), C ~ U[-1,1]."""
    return separated_problem(seed, 64, 64, p2x2=0.3, upper_scale="none", c_dist="uniform")


def config_growth(seed, m: int = 4096, n: int = 4096):
    return growth_problem(seed, m, n)


def config_separated(seed, m: int = 8192, n: int = 8192):
    """m = n = 8192 (by default), 20% 2x2 blocks, strict upper N(0,1)/sqrt(order), C ~ N(0,1)."""
    return separated_problem(seed, m, n, p2x2=0.2, upper_scale="sqrt", c_dist="normal")


def config_batched(seed: int = 0, count: int = 256, lo: int = 64, hi: int = 2048):
    """`count` independent problems, m and n log-uniform in [lo, hi] (independently); even
    indices use the separated distribution, odd indices the growth distribution.  Problem i
    draws from the i-th child of SeedSequence(seed)."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(count)
    out = []
    for i, kid in enumerate(kids):
        r = np.random.default_rng(kid)
        m = int(round(np.exp(r.uniform(np.log(lo), np.log(hi)))))
        n = int(round(np.exp(r.uniform(np.log(lo), np.log(hi)))))
        sub = r.integers(0, 2**63 - 1)
        if i % 2 == 0:
            out.append(("separated",) + separated_problem(int(sub), m, n))
        else:
            out.append(("growth",) + growth_problem(int(sub), m, n))
    return out


def config_adjoint(seed: int = 0, count: int = 32, lo: int = 256, hi: int = 1536):
    """`count` separated problems with m, n uniform integers in [lo, hi], plus W ~ N(0,1)."""
    ss = np.random.SeedSequence(seed)
    out = []
    for kid in ss.spawn(count):
        r = np.random.default_rng(kid)
        m = int(r.integers(lo, hi + 1))
        n = int(r.integers(lo, hi + 1))
        sub = int(r.integers(0, 2**63 - 1))
        A, B, C = separated_problem(sub, m, n)
        W = np.asfortranarray(np.random.default_rng(sub + 1).standard_normal((m, n)))
        out.append((A, B, C, W))
    return out
