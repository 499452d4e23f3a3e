"""Host-side checks of the persistent scheduler's static task order (no device call).

The order is the start order of a list-scheduling simulation; the kernel follows it blindly, so
it must be a topological order of the task graph of Algorithm 4: a tile update (Algorithm 3)
after the solve of its source tile and after the target's previous update in the target's fixed
order, a tile solve after every update of its tile.  The sources of target (i, l) are taken here
from their definition -- the solved tiles (k, l), k > i, and (i, j), j < l, ordered by their
anti-diagonal front (pt-1-k)+l, the column source first on a tie -- independently of the
library's closed-form index.  By default every update is its own task; multi-term tasks must
cover consecutive updates: the two updates whose sources share a front (paired grouping), or all
pending updates of a tile, at most 128 per task (deferred, left-looking grouping)."""
import pytest

import paper_1905_10574_amd as T


def sources(pt, qt, i, l):
    col = [((pt - 1 - k) + l, 0, k * qt + l) for k in range(i + 1, pt)]
    row = [((pt - 1 - i) + j, 1, i * qt + j) for j in range(l)]
    return sorted(col + row)


def decode(w):
    w = int(w)
    return w & 3, (w >> 2) & 63, (w >> 8) & 0xFFFFF, (w >> 28) & 0xFFFFF, (w >> 48) & 0xFFFF


def check_order(pt, qt, flags, slabs=1, workers=64):
    words = T.debug_task_order(pt, qt, 128, 128, slabs, workers, flags)
    srcs = {t: sources(pt, qt, t // qt, t % qt) for t in range(pt * qt)}
    solved = set()
    done = {t: 0 for t in range(pt * qt)}          # updates of t completed (in order)
    partial = {}                                   # (t, u) -> slabs seen
    groups = []
    for w in words:
        kind, slab, t, s, u = decode(w)
        U = len(srcs[t])
        if kind == 0:
            assert done[t] == U and t not in solved
            solved.add(t)
        elif kind == 3:
            g = s
            assert 2 <= g <= 128 and slab == 0 and slabs == 1
            assert done[t] == u and u + g <= U
            for j in range(g):
                assert srcs[t][u + j][2] in solved
            groups.append((t, u, g))
            done[t] = u + g
        else:
            assert 0 <= slab < slabs
            f, c, src = srcs[t][u]
            assert src == s and kind == (1 if c == 0 else 2)
            assert s in solved and done[t] == u
            partial[(t, u)] = partial.get((t, u), 0) + 1
            if partial[(t, u)] == slabs:
                done[t] = u + 1
    assert solved == set(range(pt * qt))
    assert all(done[t] == len(srcs[t]) for t in done)
    return words, groups, srcs


@pytest.mark.parametrize("pt,qt", [(1, 1), (1, 6), (6, 1), (3, 4), (7, 7), (12, 9)])
@pytest.mark.parametrize("workers", [4, 256])
def test_paired_groups_same_front_pairs(pt, qt, workers):
    words, groups, srcs = check_order(pt, qt, T.FLAG_PAIRED_UPDATES, workers=workers)
    for t, u, g in groups:
        assert g == 2 and srcs[t][u][0] == srcs[t][u + 1][0]
    # every pair of updates whose sources share a front is one task
    grouped = {(t, u) for t, u, g in groups}
    for t, ss in srcs.items():
        for u in range(len(ss) - 1):
            if ss[u][0] == ss[u + 1][0]:
                assert (t, u) in grouped
    assert len(words) == pt * qt + sum(len(s) for s in srcs.values()) - len(groups)


@pytest.mark.parametrize("pt,qt", [(3, 4), (7, 7)])
def test_single_updates_by_default_and_with_slabs(pt, qt):
    words, groups, _ = check_order(pt, qt, 0)
    assert not groups
    words, groups, _ = check_order(pt, qt, T.FLAG_PAIRED_UPDATES, slabs=2)
    assert not groups
    words, groups, _ = check_order(pt, qt, T.FLAG_DEFERRED_UPDATES, slabs=3)
    assert not groups


@pytest.mark.parametrize("pt,qt", [(2, 3), (9, 5), (66, 68)])
def test_deferred_takes_all_pending_updates(pt, qt):
    words, groups, srcs = check_order(pt, qt, T.FLAG_DEFERRED_UPDATES, workers=256)
    # one task per target (two when it has more than 128 updates), never a single update where a
    # group fits
    per = {}
    for t, u, g in groups:
        per.setdefault(t, []).append((u, g))
    for t, ss in srcs.items():
        U = len(ss)
        want = [(u, min(128, U - u)) for u in range(0, U, 128) if min(128, U - u) >= 2]
        assert per.get(t, []) == want
    assert max(len(s) for s in srcs.values()) > 128 or pt < 60


def test_task_order_argument_errors():
    lib = T.lib()
    assert lib.trsyl_debug_task_order(0, 3, 128, 128, 1, 4, 0, None, 0) == -1
    assert lib.trsyl_debug_task_order(3, 0, 128, 128, 1, 4, 0, None, 0) == -2
    assert lib.trsyl_debug_task_order(3, 3, 8, 128, 1, 4, 0, None, 0) == -3
    assert lib.trsyl_debug_task_order(3, 3, 128, 300, 1, 4, 0, None, 0) == -4
    assert lib.trsyl_debug_task_order(3, 3, 128, 128, 0, 4, 0, None, 0) == -5
    assert lib.trsyl_debug_task_order(3, 3, 128, 128, 1, 0, 0, None, 0) == -6
    assert lib.trsyl_debug_task_order(3, 3, 128, 128, 1, 4, 0, None, 5) == -9
    # 3 x 3 tiles: 9 solves and 18 updates, of which 5 same-front pairs run as one task each
    assert lib.trsyl_debug_task_order(3, 3, 128, 128, 1, 4, T.FLAG_PAIRED_UPDATES, None, 0) == 9 + 18 - 5
    assert lib.trsyl_debug_task_order(3, 3, 128, 128, 1, 4, 0, None, 0) == 9 + 18
