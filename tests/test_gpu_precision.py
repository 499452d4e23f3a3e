"""GPU tests of the precision form (FP32-MFMA tile updates, FP64 tile solves / bounds / residual,
FP64 refinement sweeps): eq. (9) after the sweeps and agreement with the FP64 CPU oracle."""
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


@pytest.mark.parametrize("m,n,tile,sweeps", [(64, 64, 32, 2), (300, 257, 64, 2), (513, 260, 128, 3),
                                             (1000, 700, 128, 2)])
def test_fp32_refine_separated(T, m, n, tile, sweeps):
    A, B, C = W.separated_problem(m + n, m, n)
    Y, e, info = T.solve(A, B, C, tile=tile, precision="fp32_refine", max_sweeps=sweeps)
    assert info == 0 and e == 0
    res = T.residual(A, B, Y, e, C)
    assert res <= 1e-12, res
    Yo, eo, _ = oracle.drsylv(A, B, C, 64, threads=8)
    Y = Y.cpu().numpy()
    err = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    assert err <= 1e-10, err
    assert np.abs(Y - Yo).max() <= 1e-10 * np.abs(Yo).max()


def test_fp32_refine_growth(T):
    """Growth input: the FP32-update solves stay robust (alpha < 1, finite, bounded) and the
    refined pair satisfies eq. (9)."""
    A, B, C = W.growth_problem(1, 200, 180)
    Y, e, info = T.solve(A, B, C, tile=64, precision="fp32_refine", max_sweeps=3)
    assert e > 0 and info in (0, 1)
    Yn = Y.cpu().numpy()
    assert np.all(np.isfinite(Yn)) and np.abs(Yn).max() <= 2.0 ** 1022
    assert T.residual(A, B, Y, e, C) <= 1e-12


def test_fp32_refine_batched_matches_single(T):
    """The batched precision form: each problem's result is bit-identical to the single solve's
    with the same tiles and sweeps (same kernels in the same order per problem), and satisfies
    eq. (9) <= 1e-12; a growth problem in the batch stays robust; empty problems pass through."""
    shapes = [(130, 97), (64, 200), (0, 5), (257, 129), (90, 90)]
    probs = []
    for i, (m, n) in enumerate(shapes):
        if m == 0 or n == 0:
            probs.append((np.eye(m), np.eye(n), np.zeros((m, n))))
        elif i == 3:
            probs.append(W.growth_problem(7, m, n))
        else:
            probs.append(W.separated_problem(50 + i, m, n))
    tiles = [(64, 32), (32, 64), (16, 16), (64, 64), (48, 48)]
    out = T.solve_batched([p[0] for p in probs], [p[1] for p in probs], [p[2] for p in probs], tiles,
                          precision="fp32_refine", max_sweeps=2)
    for i, ((A, B, C), (tm, tn), (Y, e, info)) in enumerate(zip(probs, tiles, out)):
        m, n = C.shape
        print(f"  problem {i}: m={m} n={n} e={e} info={info}", flush=True)
        Ys, es, infos = T.solve(A, B, C, tile=tm, tile_n=tn, precision="fp32_refine", max_sweeps=2)
        assert e == es and info == infos
        assert torch.equal(Y.cpu(), Ys.cpu())
        if m and n:
            assert info == 0
            assert T.residual(A, B, Y, e, C) <= 1e-12
            if i == 3:
                assert e > 0


def test_refine_tol_stops_the_sweeps(T):
    """refine_tol: every sweep starts with an eq. (9) check of the current iterate on the device and
    the refinement stops once it is at most refine_tol.  A loose tolerance runs no sweep (the result
    is the FP32-update solve's), a vanishing one runs all of them, and the default stops after the
    sweeps it needs -- with exactly the result of running that many sweeps unconditionally."""
    A, B, C = W.separated_problem(21, 300, 257)
    kw = dict(tile=64, precision="fp32_refine", counters=True)
    Y0, e0, i0 = T.solve(A, B, C, max_sweeps=-1, **kw)[:3]
    Yl, el, il, cl = T.solve(A, B, C, max_sweeps=3, refine_tol=1.0, **kw)
    assert cl["refine_sweeps"] == 0 and torch.equal(Yl.cpu(), Y0.cpu())
    Ya, ea, ia, ca = T.solve(A, B, C, max_sweeps=3, refine_tol=1e-300, **kw)
    assert ca["refine_sweeps"] == 3
    Yd, ed, idd, cd = T.solve(A, B, C, max_sweeps=3, **kw)
    k = cd["refine_sweeps"]
    print(f"  default tolerance: {k} sweep(s)", flush=True)
    assert 1 <= k < 3 and idd == 0
    assert T.residual(A, B, Yd, ed, C) <= 1e-12
    Yk, ek, ik, ck = T.solve(A, B, C, max_sweeps=k, refine_tol=1e-300, **kw)
    assert ck["refine_sweeps"] == k and ek == ed and torch.equal(Yk.cpu(), Yd.cpu())
