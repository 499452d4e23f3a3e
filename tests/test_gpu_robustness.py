"""GPU tests of the robustness invariants of Alg. 4 (Sec. 2.2) on inputs built to hit them.

  * Every tile of the result satisfies ||Y_kl||_inf <= Omega (Alg. 4's postcondition, Alg. 3's
    precondition) even where Alg. 2 alone, which bounds only the 1x1 / 2x2 blocks, would leave a
    tile above it.
  * A tile emptied by a boundary that dodged a 2x2 block is a valid (empty) source: the target's
    norm after such an "update" is still its exact norm, so later scale decisions stay sound.
  * The two schedulers run the same arithmetic: results are bitwise equal.
  * The binding never writes the caller's C.
"""
import math

import numpy as np
import pytest

import trsyl_workloads as W

pytestmark = pytest.mark.gpu
OMEGA = 2.0 ** 1022


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_10574_amd as T
    T.lib()
    return T


def tile_norms(Y, ro, co):
    return np.array([[np.abs(Y[ro[k]:ro[k + 1], co[l]:co[l + 1]]).sum(axis=1).max(initial=0.0)
                      for l in range(len(co) - 1)] for k in range(len(ro) - 1)])


def normalised(Y):
    mx = np.abs(Y).max()
    if mx == 0:
        return Y.copy(), 0
    e = math.frexp(mx)[1]
    return np.ldexp(Y, -e), e


@pytest.mark.parametrize("sched", ["dag", "fronts"])
def test_tile_norms_bounded_by_omega(T, orc, sched):
    """Diagonal A, B with a + b = 2^-3 and C near Omega / 256: X = 8 C exactly, whose tiles have
    row sums of about 3.2 Omega.  The GPU must return 2^-e X exactly (every operation is a
    power-of-two scaling or an exact division) with every tile norm at most Omega; the oracle's
    minimal choice is e = 2, so e >= 2."""
    m = n = 256
    A = np.diag(np.full(m, 2.0 ** -4))
    B = np.diag(np.full(n, 2.0 ** -4))
    C = np.ldexp(np.random.default_rng(0).uniform(0.5, 1.0, (m, n)), 1022 - 8)
    print(f"  gpu solve tile-norm case m=n={m} tile 128 {sched}", flush=True)
    Y, e, info = T.solve(A, B, C, tile=128, scheduler=sched)
    Y = Y.cpu().numpy()
    assert info == 0 and e >= 2
    assert np.array_equal(Y, np.ldexp(8 * C, -e))
    ro, co = orc.tile_offsets(A, 128), orc.tile_offsets(B, 128)
    assert (tile_norms(Y, ro, co) <= OMEGA).all()


def test_empty_source_tile_keeps_target_norm(T, orc):
    """m = tile + 1 with a 2x2 block on rows tile-1, tile: the last row tile is empty, so every
    column update of the tiles above has an empty source.  The paper's test matrices with a small
    mu (scaling everywhere, Sec. 4) then need the targets' exact norms for the row updates that
    follow; the result must stay within Omega tile by tile and agree with the oracle after
    normalisation."""
    t = 64
    m, n = t + 1, 3 * t
    A, B, C = W.paper_problem(11, m, n, 1e-3, 1e-2, p2x2=0.0)
    A[t - 1, t] = 1e-3          # 2x2 block [[mu, mu], [-mu, mu]] on rows t-1, t
    A[t, t - 1] = -1e-3
    ro = orc.tile_offsets(A, t)
    assert ro == [0, m]         # the boundary moved to the end: the nominal last row tile is empty
    print(f"  gpu solve empty-source case m={m} n={n} tile {t}", flush=True)
    Y, e, info = T.solve(A, B, C, tile=t)
    Y = Y.cpu().numpy()
    assert info == 0 and e > 0 and np.isfinite(Y).all()
    assert (tile_norms(Y, ro, orc.tile_offsets(B, t)) <= OMEGA).all()
    assert orc.relres(A, B, Y, e, C) <= 1e-13
    Yo, eo, _ = orc.drsylv(A, B, C, t)
    ng, sg = normalised(Y)
    no, so = normalised(Yo)
    assert abs((sg + e) - (so + eo)) <= 1
    err = np.linalg.norm(np.ldexp(ng, (sg + e) - (so + eo)) - no) / np.linalg.norm(no)
    assert err <= 1e-8


@pytest.mark.parametrize("flags", [0, 4])
@pytest.mark.parametrize("m,n,tile", [(300, 257, 64), (513, 260, 128), (200, 170, 16)])
def test_schedulers_are_bitwise_equal(T, m, n, tile, flags):
    """Each target takes its updates in one fixed order and every reduction has a fixed order, so
    the persistent DAG and the per-front launches produce identical bits -- with one task per
    update and with same-front pairs as two-term updates (flag 4), which both schedulers form."""
    for seed, gen in ((1, lambda s: W.separated_problem(s, m, n, p2x2=0.25)),
                      (2, lambda s: W.growth_problem(s, m, n))):
        A, B, C = gen(seed)
        print(f"  gpu solve m={m} n={n} tile {tile} flags {flags} both schedulers seed {seed}", flush=True)
        Yd, ed, infod = T.solve(A, B, C, tile=tile, scheduler="dag", flags=flags)
        Yf, ef, infof = T.solve(A, B, C, tile=tile, scheduler="fronts", flags=flags)
        assert (ed, infod) == (ef, infof)
        assert np.array_equal(Yd.cpu().numpy(), Yf.cpu().numpy())


def test_column_major_c_is_not_overwritten(T):
    """A column-major float64 C on the device is passed without a copy elsewhere in the binding;
    the operand the library overwrites must still be a buffer of its own."""
    import torch
    A, B, C = W.separated_problem(3, 90, 70)
    dev = torch.device("cuda:0")
    Cd = torch.from_numpy(np.asfortranarray(C)).to(dev).t().contiguous().t()   # column-major
    keep = Cd.clone()
    print("  gpu solve with a column-major C", flush=True)
    Y, e, info = T.solve(A, B, Cd)
    assert info == 0 and torch.equal(Cd, keep)
    Ya, ea, infoa = T.adjoint(A, B, Cd)
    assert infoa == 0 and torch.equal(Cd, keep)
