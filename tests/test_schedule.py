"""Host logic of the solver library (no GPU): the leaf partition and the
wave/update schedule.  Every coefficient entry must be applied exactly once
(the schedule's flop count equals the oracle's F_tri), and replaying the
schedule must find every dependency satisfied (Sec. 2.1: a block needs all
blocks after it along each mode; an update needs its sources solved and its
targets unsolved)."""
import ctypes

import numpy as np
import pytest

import oracle
import tt_inputs as ti

tt = pytest.importorskip("paper_1905_09539_amd")


def test_library_exports_every_declared_symbol():
    import os
    import re
    L = tt.lib()
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "tt.h")).read()
    declared = set(re.findall(r"^(?:int|double|const char\*|size_t)\s+(\w+)\(", hdr, re.M))
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(L, name), name
    assert declared <= set(tt.SYMBOLS)


@pytest.mark.parametrize("shape,bumps", [
    ((32, 32, 32), "every8"), ((512, 512, 512), "every8"), ((37, 20, 45), "random"),
    ((96, 96, 96, 96), "every8"), ((1024, 1024, 8, 8), "every8"), ((5, 7, 3), "none"),
    ((64,), "every8"), ((50, 70), "random"), ((200, 150, 180), "random"), ((33, 47, 190), "aligned"),
    ((1, 1, 1), "none"), ((768, 40, 3), "every8"), ((19, 23, 29, 17), "random"),
])
def test_schedule_complete_and_ordered(shape, bumps):
    p = ti.laplace_tri(shape, seed=3, bumps=bumps)
    info = tt.schedule_info(p["T"], shape)
    assert info["dependency_violation"] == 0
    assert info["flops"] == oracle.flops_tri(p["T"], shape)
    assert info["flops"] == info["flops_leaf"] + info["flops_update"]


@pytest.mark.parametrize("nmin", [2, 3, 5, 8, 12, 16])
def test_schedule_any_leaf_size(nmin):
    shape = (45, 38, 52)
    p = ti.laplace_tri(shape, seed=5, bumps="random")
    info = tt.schedule_info(p["T"], shape, nmin=nmin)
    assert info["dependency_violation"] == 0
    assert info["flops"] == oracle.flops_tri(p["T"], shape)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 8, 9, 10, 16, 17, 18, 33])
def test_schedule_block_counts_around_powers_of_two(m):
    """m = 2^L + 1 blocks per mode run the split tree over 2^L blocks with
    the last two merged; every block must still receive every later block of
    its fibres exactly once (index sums checked by the replay)."""
    shape = (4 * m, 4 * m, 12)
    p = ti.laplace_tri(shape, seed=7, bumps="none")
    info = tt.schedule_info(p["T"], shape, nmin=4)
    assert info["dependency_violation"] == 0
    assert info["flops"] == oracle.flops_tri(p["T"], shape)


def test_partition_never_cuts_a_bump():
    """Split points k always satisfy A(k+1, k) = 0 (Sec. 2.1, Algorithm 2)."""
    n = 512
    p = ti.laplace_tri((n, n, n), seed=1, bumps="every8")
    info = tt.schedule_info(p["T"], (n, n, n))
    # every 8th row starts a bump, so 32 blocks of 16 rows are impossible:
    # the planner takes 33 blocks of at most 16 rows (3 * 32 + 1 waves)
    assert info["bmax0"] == 16 and info["waves"] == 97
    assert info["dependency_violation"] == 0


def test_schedule_rejects_bad_structure():
    T = np.triu(np.ones((6, 6)))
    T[4, 2] = 1.0
    with pytest.raises(tt.TTError) as e:
        tt.schedule_info([T, np.eye(3), np.eye(2)], (6, 3, 2))
    assert e.value.code == tt.TT_EINVAL
    with pytest.raises(tt.TTError):
        tt.schedule_info([np.eye(4)] * 3, (4, 4, 4), nmin=64)


def test_plan_entry_points_reject_null_plan():
    """The plan entry points validate their arguments before any device
    call: a NULL plan is TT_EINVAL with a message (no GPU needed)."""
    L = tt.lib()
    null = ctypes.c_void_p(0)
    for fn in (L.tt_plan_solve, L.tt_plan_solve_graph):
        assert fn(null, null, null, null) == tt.TT_EINVAL
        assert b"NULL" in L.tt_last_error()


def _dense_bumps(n, g):
    """Upper quasi-triangular n x n with a 2x2 block at every even row: the
    most 2x2 blocks a real Schur form can hold."""
    T = np.triu(g.standard_normal((n, n)) / np.sqrt(n))
    for i in range(0, n - 1, 2):
        a, b = 1.0 + g.random(), 0.1 + 0.4 * g.random()
        T[i, i] = T[i + 1, i + 1] = a
        T[i, i + 1], T[i + 1, i] = b, -b
    if n % 2:
        T[n - 1, n - 1] = 1.0 + g.random()
    return T


@pytest.mark.parametrize("shape", [(32, 32, 32), (512, 512, 512), (37, 20, 45), (96, 96, 96, 96),
                                   (1024, 1024, 8, 8), (5, 7, 3), (64,), (50, 70), (200, 150, 180),
                                   (1, 1, 1), (768, 40, 3), (19, 23, 29, 17), (17, 16, 15)])
@pytest.mark.parametrize("bumps", ["every8", "aligned", "random", "none", "dense"])
def test_workspace_bound_covers_every_pattern(shape, bumps):
    """tt_workspace_bytes is a bound over every 2x2-block pattern: the plan's
    tables, coefficient copies and accumulators (exact, from the host
    schedule) plus the largest extra tensor of any call kind fit in it."""
    if bumps == "dense":
        g = np.random.default_rng(11)
        T = [_dense_bumps(n, g) for n in shape]
    else:
        T = ti.laplace_tri(shape, seed=3, bumps=bumps)["T"]
    info = tt.schedule_info(T, shape)
    N = int(np.prod(shape))
    for prec in (tt.TT_FP64, tt.TT_MP_FP32, tt.TT_MP_BF16):
        bound = tt.workspace_bytes(shape, prec)
        assert bound >= info["plan_bytes"] + 8 * N, (bound, info["plan_bytes"])
    assert tt.workspace_bytes(shape, tt.TT_MP_FP32) >= tt.workspace_bytes(shape, tt.TT_FP64)
    # the second class (same schedule at its default leaf edge 8 / 5): the
    # partial products W_1 .. W_{d-2} and one pipeline tensor besides
    if len(shape) >= 3:
        info2 = tt.schedule_info(T, shape, nmin=5 if len(shape) == 4 else 8)
        assert tt.workspace_bytes(shape) >= info2["plan_bytes"] + 8 * N * (len(shape) - 1)


def test_workspace_bytes_rejects_bad_shapes():
    assert tt.workspace_bytes((4, 4, 4, 4, 4)) == 0
    assert tt.workspace_bytes((4, -1, 4)) == 0
    assert tt.workspace_bytes((0, 5, 5)) > 0


@pytest.mark.parametrize("shape,nmin", [((192, 192, 192), 8), ((40, 36, 44, 30), 5), ((100, 90, 96), 6)])
def test_small_pencils_share_update_tiles(shape, nmin):
    """Second-class schedules: updates of at most 16 target rows whose
    pencils have at most 64 (128) columns share a 16 x 256 tile four (two)
    at a time, so there are far fewer tiles than tasks, and the replay
    (which checks that the tasks of a shared tile differ only in their
    pencil and that every task's tiles appear once) finds the schedule
    complete.  The Laplace-like schedule of the same shape shares no tile
    and covers the same tasks."""
    p = ti.laplace_tri(shape, seed=2, bumps="random")
    info = tt.schedule_info(p["T"], shape, nmin=nmin, cls=1)
    assert info["dependency_violation"] == 0
    assert info["flops"] == oracle.flops_tri(p["T"], shape)
    assert info["items"] < 0.6 * info["tasks"]
    lap = tt.schedule_info(p["T"], shape, nmin=nmin)
    assert lap["dependency_violation"] == 0
    assert lap["tasks"] == info["tasks"] and lap["items"] > info["items"]


def test_schedule_info_class_rejects_unknown_class():
    p = ti.laplace_tri((8, 8, 8), seed=1, bumps="none")
    with pytest.raises(tt.TTError):
        tt.schedule_info(p["T"], (8, 8, 8), cls=2)
