"""The batched ensemble, tile shapes, the autotuner and captured step graphs
(through the C ABI).

Every instance of an ensemble advances with its own grid, time and CFL step
inside the same launches, so each member must come out bitwise equal to a
run of that member alone; the tile shape, the autotuner's timing runs and
graph replay must not change any bit either.  One small ensemble is also
checked against the oracle member by member."""
import numpy as np
import pytest

import fvinputs as F
from oracle import Solver

pytestmark = pytest.mark.gpu


def _solver(cases, **kw):
    from paper_2210_04037_amd.solver import GpuSolver
    return GpuSolver(cases, **kw)


def _members(ms, n=None):
    return [F.make_case(4, member=m, n=n) for m in ms]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ensemble_members_equal_single_runs(precision):
    cases = _members(range(5))
    print("[ensemble]", precision, [c.n[0] for c in cases], flush=True)
    g = _solver(cases, precision=precision)
    g.step(25)
    t = g.time()
    ens = [g.state(i) for i in range(len(cases))]
    tot, out = g.totals()
    g.close()
    for i, c in enumerate(cases):
        s = _solver(c, precision=precision)
        s.step(25)
        assert s.time()[0] == t[i]
        assert np.array_equal(s.state(0), ens[i]), i
        t1, o1 = s.totals()
        assert np.array_equal(t1[0], tot[i]) and np.array_equal(o1[0], out[i])
        s.close()


def test_ensemble_members_match_oracle():
    """Ragged members (different edges and ring speeds) in one context
    against the oracle, 15 steps each."""
    cases = [F.make_case(4, member=m, n=n) for m, n in ((0, 40), (1, 56), (2, 33))]
    g = _solver(cases)
    g.step(15)
    for i, c in enumerate(cases):
        o = Solver(c)
        for _ in range(15):
            o.step()
        U = g.state(i)
        for f in range(U.shape[0]):
            sc = np.max(np.abs(o.U[f])) + 1e-300
            assert np.max(np.abs(U[f] - o.U[f])) <= 1e-9 * sc, (i, f)
        assert g.time()[i] == pytest.approx(o.t, rel=1e-12)
    g.close()


def test_ensemble_members_stop_at_their_end_time():
    cases = _members(range(3), n=48)
    g = _solver(cases)
    dt = g.cfl_dt()
    t_end = np.array([3.5 * dt[0], 1e-3, 7.25 * dt[2]])
    g.step(12, t_end=t_end)
    t = g.time()
    assert t[0] == pytest.approx(t_end[0], rel=1e-15)
    assert t[2] == pytest.approx(t_end[2], rel=1e-15)
    assert t[1] < t_end[1]
    g.step(3)                             # finished members stay put
    t2 = g.time()
    assert t2[0] == t[0] and t2[2] == t[2] and t2[1] > t[1]
    g.close()


def _tiles(case, precision):
    g = _solver(case, precision=precision)
    chosen, table = g.autotune(reps=3)
    g.close()
    return list(table)


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tile_shapes_give_identical_bits(precision, dim):
    # ragged against every tile shape, including those with spare threads
    case = F.make_case(2, n=200) if dim == 2 else F.make_case(1, n=1021)
    shapes = _tiles(case, precision)
    assert len(shapes) >= 3
    ref = None
    for tile in shapes:
        print("[tiles]", precision, tile, flush=True)
        g = _solver(case, precision=precision, tile=tile)
        g.step(20)
        U = g.state(0)
        g.close()
        if ref is None:
            ref = U
        else:
            assert np.array_equal(U, ref), tile


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_block_schedules_give_identical_bits(precision):
    """Every configuration the autotuner tries on a ragged ensemble (tile
    shape x block schedule) gives bitwise the same members."""
    cases = [F.make_case(4, member=m, n=n) for m, n in ((0, 70), (1, 45), (2, 96))]
    g = _solver(cases, precision=precision)
    _, table = g.autotune(reps=2)
    g.close()
    assert {k[2] for k in table} == {0, 1, 2}
    ref = None
    for cfg in table:
        g = _solver(cases, precision=precision, tile=cfg)
        g.step(12)
        U = [g.state(i) for i in range(len(cases))]
        g.close()
        if ref is None:
            ref = U
        else:
            for i in range(len(cases)):
                assert np.array_equal(U[i], ref[i]), (cfg, i)


def test_unknown_tile_is_rejected():
    from paper_2210_04037_amd import abi
    with pytest.raises(abi.FvError) as e:
        _solver(F.make_case(2, n=64), tile=(24, 24))
    assert e.value.code == abi.FV_EINVAL
    with pytest.raises(abi.FvError) as e:
        _solver(F.make_case(2, n=64), tile=(16, 15, 3))     # no such schedule
    assert e.value.code == abi.FV_EINVAL


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotune_leaves_the_run_unchanged(precision):
    case = F.make_case(2, n=160)
    a = _solver(case, precision=precision)
    b = _solver(case, precision=precision)
    a.step(10)
    b.step(10)
    chosen, table = b.autotune(reps=5)
    print("[autotune]", precision, chosen, table, flush=True)
    assert chosen in table and all(v > 0 for v in table.values())
    a.step(10)
    b.step(10)
    assert np.array_equal(a.state(0), b.state(0))
    assert a.time()[0] == b.time()[0]
    ta, oa = a.totals()
    tb, ob = b.totals()
    assert np.array_equal(ta, tb) and np.array_equal(oa, ob)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_match_eager(precision):
    """Replays of the captured step graph, with eager work of the program
    between them, against eager stepping: every replay bitwise."""
    cases = _members(range(3), n=96)
    e = _solver(cases, precision=precision)
    g = _solver(cases, precision=precision, use_graph=True)
    for rep, n in enumerate((4, 4, 4, 3, 3, 4)):   # odd counts flip parity
        e.step(n)
        g.step(n)
        # eager work between replays: reductions, host syncs, CFL
        te, _ = e.totals()
        tg, _ = g.totals()
        assert np.array_equal(te, tg), rep
        assert np.array_equal(e.cfl_dt(), g.cfl_dt()), rep
        for i in range(len(cases)):
            assert np.array_equal(e.state(i), g.state(i)), (rep, i)
        assert np.array_equal(e.time(), g.time())
    e.close()
    g.close()
