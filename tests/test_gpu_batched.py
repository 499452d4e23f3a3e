"""GPU tests of the batched driver: many uneven problems in one persistent launch.

* Every problem's result is bit-identical to the single-problem solve with the same tiles (same
  task order per target, same kernels).
* Separated problems match the FP64 oracle to 1e-10 and satisfy eq. (9) <= 1e-13; growth problems
  return alpha < 1 with eq. (9) <= 1e-13.
* A malformed problem (two consecutive subdiagonals) reports status 2 without disturbing the
  others; empty problems return e = 0.
* The autotuner returns a tile from its candidate set for every bucket.
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


def _mixed(seed=0):
    rng = np.random.default_rng(seed)
    shapes = [(64, 64), (130, 37), (1, 200), (257, 129), (300, 300), (17, 5), (0, 12), (90, 260),
              (129, 129), (200, 150), (45, 45), (12, 0)]
    probs = []
    for i, (m, n) in enumerate(shapes):
        if i in (3, 9):                       # growth problems (rectangular pairing)
            A, B, C = W.growth_problem(100 + i, m, n)
        else:
            A, B, C = W.separated_problem(100 + i, m, n) if m and n else (np.eye(m), np.eye(n), np.zeros((m, n)))
        probs.append((A, B, C))
    tiles = [(int(rng.choice([16, 32, 64, 128])), int(rng.choice([16, 32, 64, 128]))) for _ in shapes]
    return probs, tiles


def test_batched_bit_identical_to_single(T):
    probs, tiles = _mixed()
    out = T.solve_batched([p[0] for p in probs], [p[1] for p in probs], [p[2] for p in probs], tiles)
    for (A, B, C), (tm, tn), (Y, e, info) in zip(probs, tiles, out):
        Ys, es, infos = T.solve(A, B, C, tile=tm, tile_n=tn)
        assert e == es and info == infos
        assert torch.equal(Y.cpu(), Ys.cpu())


@pytest.mark.parametrize("flags", [4, 8])
def test_batched_grouped_updates_bit_identical_to_single(T, flags):
    """The update-grouping options in the batched scheduler: each problem's result equals the single
    solve's with the same tiles and option bit for bit (same multi-term tasks, same order per
    target), and problems of both kinds keep eq. (9)."""
    probs, tiles = _mixed()
    out = T.solve_batched([p[0] for p in probs], [p[1] for p in probs], [p[2] for p in probs], tiles, flags=flags)
    for (A, B, C), (tm, tn), (Y, e, info) in zip(probs, tiles, out):
        Ys, es, infos = T.solve(A, B, C, tile=tm, tile_n=tn, flags=flags)
        assert e == es and info == infos
        assert torch.equal(Y.cpu(), Ys.cpu())
        if C.size:
            assert T.residual(A, B, Y, e, C) <= 1e-13


def test_batched_parity_and_residual(T):
    probs, tiles = _mixed()
    out = T.solve_batched([p[0] for p in probs], [p[1] for p in probs], [p[2] for p in probs], tiles)
    for i, ((A, B, C), (Y, e, info)) in enumerate(zip(probs, out)):
        m, n = C.shape
        if m == 0 or n == 0:
            assert e == 0 and info == 0
            continue
        assert info == 0
        assert T.residual(A, B, Y, e, C) <= 1e-13
        Yo, eo, _ = oracle.drsylv(A, B, C, 32)
        Yn = Y.cpu().numpy()
        if i in (3, 9):
            # growth members: both scale; backward error by the oracle in long double; normalised
            # solutions agree to within ten times the oracle's own spread between two tile sizes
            # (the forward solution of these inputs moves with the order of rounding)
            assert e > 0 and eo > 0
            assert oracle.relres(A, B, Yn, e, C) <= 1e-13
            Y2, e2, _ = oracle.drsylv(A, B, C, 24)
            so = int(np.frexp(np.abs(Yo).max())[1])
            norm_o = np.ldexp(Yo, -so)
            spread = np.linalg.norm(np.ldexp(Y2, (e2 - eo) - so) - norm_o) / np.linalg.norm(norm_o)
            sg = int(np.frexp(np.abs(Yn).max())[1])
            assert abs((sg + e) - (so + eo)) <= 1
            err = np.linalg.norm(np.ldexp(Yn, (e - eo) - so) - norm_o) / np.linalg.norm(norm_o)
            print(f"  growth member {i}: normalised difference {err:.2e}, oracle spread {spread:.2e}", flush=True)
            assert err <= max(1e-8, 10 * spread)
        else:
            assert e == 0 and eo == 0
            assert np.linalg.norm(Yn - Yo) <= 1e-10 * np.linalg.norm(Yo)
            assert np.abs(Yn - Yo).max() <= 1e-10 * np.abs(Yo).max()


def test_batched_isolates_bad_problem(T):
    rng = np.random.default_rng(4)
    A1, B1, C1 = W.separated_problem(1, 80, 70)
    A2, B2, C2 = W.separated_problem(2, 60, 50)
    A2 = A2.copy()
    A2[11, 10] = 0.5
    A2[12, 11] = 0.5                     # two consecutive nonzero subdiagonals
    A3, B3, C3 = W.separated_problem(3, 100, 40)
    out = T.solve_batched([A1, A2, A3], [B1, B2, B3], [C1, C2, C3], [(32, 32)] * 3)
    assert out[1][2] == 2
    for (A, B, C), (Y, e, info) in ((p, o) for i, (p, o) in enumerate(zip([(A1, B1, C1), (A2, B2, C2), (A3, B3, C3)], out)) if i != 1):
        assert info == 0 and e == 0
        assert T.residual(A, B, Y, e, C) <= 1e-13


def test_batched_isolates_tile_norm_violation(T):
    """A problem whose C has 32-wide tile rows summing past Omega (entries 2^1020, each at most
    Omega) fails Algorithm 4's data requirement: status 3 for it alone, as in the oracle."""
    A1, B1, C1 = W.separated_problem(1, 80, 70)
    A2, B2, C2 = W.separated_problem(2, 60, 50)
    C2 = np.full_like(C2, 2.0 ** 1020)
    A3, B3, C3 = W.separated_problem(3, 100, 40)
    assert oracle.drsylv(A2, B2, C2, 32)[2] == 3
    out = T.solve_batched([A1, A2, A3], [B1, B2, B3], [C1, C2, C3], [(32, 32)] * 3)
    assert out[1][2] == 3
    for (A, B, C), (Y, e, info) in (((A1, B1, C1), out[0]), ((A3, B3, C3), out[2])):
        assert info == 0 and e == 0
        assert T.residual(A, B, Y, e, C) <= 1e-13


def test_autotuner_table(T, tmp_path):
    """The tuner ranks the candidates by the median of its timed runs on a batch that mixes
    separated and growth problems, and writes the table (with the medians) as JSON."""
    import json
    path = str(tmp_path / "tiles.json")
    table = T.autotune_tiles(buckets=(64, 256), batch_flops=2e9, reps=3, path=path)
    assert set(table) >= {64, 256}
    for b, t in table.items():
        assert t in T.TILE_CANDIDATES
    rec = json.load(open(path))
    assert {int(k): v for k, v in rec["tiles"].items()} == table
    for b, med in rec["meta"]["median_ms"].items():
        assert min(med, key=med.get) == str(table[int(b)])
    probs, _ = _mixed(1)
    out = T.solve_batched([p[0] for p in probs], [p[1] for p in probs], [p[2] for p in probs], "auto")
    for (A, B, C), (Y, e, info) in zip(probs, out):
        if C.size:
            assert info == 0 and T.residual(A, B, Y, e, C) <= 1e-13
