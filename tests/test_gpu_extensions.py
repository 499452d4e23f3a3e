"""GPU parity of the adjoint solve, the gradient products, the autograd function and the device
eq. (9) residual, each against the CPU oracle (and central finite differences for the gradients).
"""
import numpy as np
import pytest

import oracle
import trsyl_workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1905_10574_amd as T
    T.lib()
    return T


def _problem(seed, m, n, p2=0.3):
    rng = np.random.default_rng(seed)
    A = W.quasi_triangular(rng, m, p2x2=p2)
    B = W.quasi_triangular(rng, n, p2x2=p2)
    Wm = rng.standard_normal((m, n))
    return A, B, Wm


def _pattern(T_):
    """Quasi-triangular pattern: upper triangle plus the subdiagonal entries of 2x2 blocks."""
    n = T_.shape[0]
    P = np.triu(np.ones((n, n), dtype=bool))
    for i in range(n - 1):
        if T_[i + 1, i] != 0.0:
            P[i + 1, i] = True
    return P


@pytest.mark.parametrize("m,n,tile", [(1, 1, 16), (17, 9, 16), (40, 33, 16), (70, 64, 32), (150, 97, 64)])
def test_adjoint_matches_oracle(T, m, n, tile):
    A, B, Wm = _problem(m * 1000 + n, m, n)
    G, e, info = T.adjoint(A, B, Wm, tile=tile)
    Go, eo, rc = oracle.adjoint(A, B, Wm, 32)
    assert info == 0 and rc == 0 and e == 0 and eo == 0
    G = G.cpu().numpy()
    err = np.linalg.norm(G - Go) / np.linalg.norm(Go)
    assert err <= 1e-10, err
    assert np.abs(G - Go).max() <= 1e-10 * np.abs(Go).max()
    # the adjoint equation itself, in long double on the host
    R = A.T @ G + G @ B.T - Wm
    assert np.linalg.norm(R) / (np.linalg.norm(Wm) + (np.linalg.norm(A) + np.linalg.norm(B)) * np.linalg.norm(G)) <= 1e-13


def test_adjoint_tile_norm_precondition(T):
    """The adjoint runs Algorithm 4 on the order-reversed problem, whose tiles carry its data
    requirement (tile infinity norms at most Omega): upper-triangular entries just below 2^1016
    fail 128-wide tiles and pass 64-wide ones, with the oracle's adjoint in the same tiling."""
    rng = np.random.default_rng(6)
    m, n = 128, 4
    A = np.triu(rng.uniform(0.9, 1, (m, m))) * 2.0 ** 1016
    B = np.triu(rng.uniform(0.5, 1, (n, n)))
    Wm = rng.uniform(-1, 1, (m, n))
    assert oracle.adjoint(A, B, Wm, 128)[2] == 3
    _, _, info = T.adjoint(A, B, Wm, tile=128)
    assert info == 3
    Go, eo, rc = oracle.adjoint(A, B, Wm, 64)
    G, e, info = T.adjoint(A, B, Wm, tile=64)
    assert rc == 0 and info == 0 and e == 0 and eo == 0
    G = G.cpu().numpy()
    assert np.abs(G - Go).max() <= 1e-10 * np.abs(Go).max()


def test_adjoint_empty(T):
    A = np.zeros((0, 0))
    B = np.eye(3)
    G, e, info = T.adjoint(A, B, np.zeros((0, 3)))
    assert G.shape == (0, 3) and e == 0 and info == 0


@pytest.mark.parametrize("m,n", [(24, 19), (65, 40)])
def test_grad_products_match_definition(T, m, n):
    """dA = -G~ Y^T on A's pattern, dB = -Y^T G~ on B's pattern, dC = alpha G~, with Y and G
    from the oracle (forward and adjoint)."""
    A, B, Wm = _problem(7 + m, m, n)
    rng = np.random.default_rng(99)
    C = rng.uniform(-1, 1, (m, n))
    Y, eY, _ = oracle.drsylv(A, B, C, 32)
    G, eG, _ = oracle.adjoint(A, B, Wm, 32)
    dA, dB, dC = T.grad(A, B, Y, eY, G, eG)
    torch.cuda.synchronize()
    dA, dB, dC = dA.cpu().numpy(), dB.cpu().numpy(), dC.cpu().numpy()
    Gt = np.ldexp(G, eG)
    eA = np.where(_pattern(A), -Gt @ Y.T, 0.0)
    eB = np.where(_pattern(B), -Y.T @ Gt, 0.0)
    eC = np.ldexp(Gt, -eY)
    for got, want in ((dA, eA), (dB, eB), (dC, eC)):
        assert np.linalg.norm(got - want) <= 1e-12 * max(np.linalg.norm(want), 1e-300)


def test_autograd_matches_finite_differences(T):
    """L = <W, Y>: central differences (h = 1e-6) on a 12 x 9 problem against TrsylFunction."""
    m, n = 12, 9
    A, B, Wm = _problem(5, m, n)
    rng = np.random.default_rng(6)
    C = rng.uniform(-1, 1, (m, n))
    At = torch.tensor(A, dtype=torch.float64, device="cuda", requires_grad=True)
    Bt = torch.tensor(B, dtype=torch.float64, device="cuda", requires_grad=True)
    Ct = torch.tensor(C, dtype=torch.float64, device="cuda", requires_grad=True)
    Wt = torch.tensor(Wm, dtype=torch.float64, device="cuda")
    Y, e = T.trsyl(At, Bt, Ct, 16)
    assert int(e.item()) == 0
    L = (Wt * Y).sum()
    L.backward()

    def loss(A_, B_, C_):
        Yo, eo, _ = oracle.drsylv(A_, B_, C_, 8)
        assert eo == 0
        return float((Wm * Yo).sum())

    h = 1e-6
    PA, PB = _pattern(A), _pattern(B)
    for (M, Pm, g) in ((A, PA, At.grad), (B, PB, Bt.grad), (C, np.ones_like(C, dtype=bool), Ct.grad)):
        g = g.cpu().numpy()
        idx = np.argwhere(Pm)
        sel = idx[np.random.default_rng(1).choice(len(idx), size=min(12, len(idx)), replace=False)]
        for (i, j) in sel:
            Mp, Mm = M.copy(), M.copy()
            Mp[i, j] += h
            Mm[i, j] -= h
            args_p = [A, B, C]
            args_m = [A, B, C]
            k = 0 if M is A else (1 if M is B else 2)
            args_p[k], args_m[k] = Mp, Mm
            fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
            assert abs(fd - g[i, j]) <= 1e-6 * max(1.0, abs(fd)), (k, i, j, fd, g[i, j])
        # outside the pattern the gradient is exactly zero
        assert np.all(g[~Pm] == 0.0)


@pytest.mark.parametrize("case", ["random", "solution", "growth"])
def test_device_residual_matches_oracle(T, case):
    rng = np.random.default_rng(3)
    m, n = 70, 45
    if case == "growth":
        A, B, C = W.growth_problem(2, 160, 150)
        Y, e, _ = oracle.drsylv(A, B, C, 32)
        assert e > 0
    else:
        A = W.quasi_triangular(rng, m, p2x2=0.3)
        B = W.quasi_triangular(rng, n, p2x2=0.3)
        C = rng.uniform(-1, 1, (m, n))
        if case == "random":
            Y, e = rng.standard_normal((m, n)), 3
        else:
            Y, e, _ = oracle.drsylv(A, B, C, 32)
    got = T.residual(A, B, Y, e, C)
    want = oracle.relres(A, B, Y, e, C)
    if case == "random":
        assert abs(got - want) <= 1e-12 * want
    else:
        assert got <= 1e-13 and want <= 1e-13
        assert 0.2 * want <= got <= 5.0 * want + 1e-18


def test_adjoint_batched_matches_single(T):
    """The batched adjoint: each problem bit-identical to trsyl_robust_adjoint with the same tiles;
    the transposed equation holds to eq. (9)'s bound."""
    import torch
    shapes = [(70, 90), (128, 64), (0, 4), (129, 33)]
    probs = []
    for i, (m, n) in enumerate(shapes):
        if m and n:
            A, B, _ = W.separated_problem(300 + i, m, n)
        else:
            A, B = np.eye(m), np.eye(n)
        Wm = np.random.default_rng(i).standard_normal((m, n))
        probs.append((A, B, Wm))
    tiles = [(32, 64), (64, 16), (16, 16), (64, 32)]
    out = T.adjoint_batched([p[0] for p in probs], [p[1] for p in probs], [p[2] for p in probs], tiles)
    for (A, B, Wm), (tm, tn), (G, e, info) in zip(probs, tiles, out):
        Gs, es, infos = T.adjoint(A, B, Wm, tile=tm, tile_n=tn)
        assert e == es and info == infos == 0
        assert torch.equal(G.cpu(), Gs.cpu())
        if A.size and B.size:
            Gn = G.cpu().numpy()
            R = A.T @ Gn + Gn @ B.T - np.ldexp(Wm, -e)
            q = np.linalg.norm(R) / ((np.linalg.norm(A) + np.linalg.norm(B)) * np.linalg.norm(Gn) + np.linalg.norm(Wm))
            assert q <= 1e-13, q
