"""trsyl_robust_noalloc (the entry point for callers that cannot allocate) against trsyl_robust on
the same inputs: two calls in a row, the second with a smaller problem, each bit-identical in Y,
e and the status to the workspace entry point with the same tiles (the two schedulers run the same
arithmetic).  The second call reuses the fixed array the first one left behind."""
import numpy as np
import pytest

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


def _both(T, A, B, C, tile):
    opts = T.make_opts(tile=tile)
    print(f"  noalloc vs workspace solve m={C.shape[0]} n={C.shape[1]} tile {tile}", flush=True)
    Yn, en, scn, infn = T.solve_noalloc_async(A, B, C, opts)
    torch.cuda.synchronize()
    Yr, er, scr, infr = T.solve_async(A, B, C, T.make_opts(tile=tile))
    torch.cuda.synchronize()
    return (Yn.cpu(), int(en.item()), float(scn.item()), int(infn.item())), \
           (Yr.cpu(), int(er.item()), float(scr.item()), int(infr.item()))


def test_noalloc_matches_workspace_entry_point_twice(T):
    cases = [(W.separated_problem(3, 700, 600, p2x2=0.25), 64),      # first call: larger
             (W.growth_problem(5, 130, 97), 32)]                       # second call: smaller, scales
    for (A, B, C), tile in cases:
        (Yn, en, scn, infn), (Yr, er, scr, infr) = _both(T, A, B, C, tile)
        assert infn == infr and en == er and scn == scr
        assert torch.equal(Yn, Yr)
        assert np.isfinite(Yn.numpy()).all()
    # the growth case really scaled
    assert en > 0
