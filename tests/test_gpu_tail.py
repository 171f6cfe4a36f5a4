"""Loop schedules (DTSPH_OPT_TAIL_LOOP): 0 plain chunks; 1 the first chunk of a
batch's loop cut where, by the last loop's counts, few sims keep iterating, and
the rest of a small remainder run in one persistent cooperative launch with
per-sim barriers on the device; 2 the same cut with plain chunks over the
remaining sims' tiles. Every step must equal schedule 0 bit for bit (fields,
reports, status): batches whose sims stop at different iterations, with and
without walls, FP32 and FP64, 2D and 3D, at every lane count and workgroup size,
sims stopping at their iteration limit inside a tail launch, barriers over
several groups of workgroups, a single sim, and the fixed-iteration call; a
barrier wait that gives up (forced by a one-poll limit) is an error, not a hang."""
import numpy as np
import pytest

from paper_1904_00861_amd import dtsph as D
from paper_1904_00861_amd import inputs as I

from gpu_helpers import banner

pytestmark = pytest.mark.gpu


def _params(prob, **kw):
    prob.params = dict(prob.params, **kw)
    return prob


def _loose(prob):
    # stops after its first iteration: the rest of each loop is a small remainder
    return _params(prob, tol=1.0)


CASES = {
    "batch_mixed": lambda: [_loose(I.tgv2d(60, seed=1)), I.cavity(14, re=700.0), I.tgv2d(12, seed=3, re=300.0),
                            _loose(I.cavity(40)), I.tgv2d(10, seed=6)],
    "batch_tgv": lambda: [_loose(I.tgv2d(64, seed=4)), I.tgv2d(16, seed=5, re=800.0), I.tgv2d(10, seed=6)],
    "batch_3d": lambda: [_loose(I.tgv3d(16, seed=3)), I.tgv3d(8, seed=4, re=400.0)],
    # one sim stops at its iteration limit inside the tail launch
    "batch_maxiter": lambda: [_loose(I.tgv2d(60, seed=7)), _params(I.cavity(12, re=900.0), max_iter=9, tol=1e-12),
                              I.tgv2d(14, seed=8, re=600.0)],
    "single_cavity": lambda: I.cavity(24, re=400.0),
}
EXPECT_TAIL = {"batch_mixed", "batch_tgv", "batch_3d", "batch_maxiter"}


def _run(prob, prec, schedule, steps, lanes=None, block=None):
    sim = D.Sim(prob, precision=prec)
    sim.set_option(D.OPT_TAIL_LOOP, schedule)
    if lanes:
        sim.set_option(D.OPT_LANES, lanes)
    if block:
        sim.set_option(D.OPT_BLOCK, block)
    out = []
    for _ in range(steps):
        st, rep = sim.step(1)
        out.append((st, rep, sim.get_state()))
    n_tail = sim.timing()["tail_launches"]
    sim.close()
    return out, n_tail


def _same(ref, other, what):
    for k, ((st_a, rep_a, sa), (st_b, rep_b, sb)) in enumerate(zip(ref, other)):
        assert st_a == st_b, f"{what} step {k}: status"
        assert rep_a == rep_b, f"{what} step {k}: reports"
        for f in sa:
            assert np.array_equal(sa[f], sb[f]), f"{what} step {k}: field {f}"


@pytest.mark.parametrize("prec", [D.FP32, D.FP64])
@pytest.mark.parametrize("case", list(CASES))
def test_loop_schedules_match_plain_chunks(case, prec):
    banner(f"loop schedules {case} precision {prec}")
    plain, n0 = _run(CASES[case](), prec, 0, 6)
    tail, n1 = _run(CASES[case](), prec, 1, 6)
    cut, n2 = _run(CASES[case](), prec, 2, 6)
    assert n0 == 0 and n2 == 0
    assert (n1 > 0) == (case in EXPECT_TAIL), n1
    _same(plain, tail, f"{case} schedule 1")
    _same(plain, cut, f"{case} schedule 2")
    if case == "batch_maxiter":
        assert any(r["reason"] == 3 for _, rep, _ in tail for step in rep for r in step)


@pytest.mark.parametrize("lanes,block", [(1, 64), (2, 128), (4, 256), (8, 256), (8, 64)])
def test_tail_launches_every_lane_count(lanes, block):
    banner(f"tail launch lanes {lanes} block {block}")
    plain, _ = _run(CASES["batch_mixed"](), D.FP32, 0, 4, lanes, block)
    tail, n1 = _run(CASES["batch_mixed"](), D.FP32, 1, 4, lanes, block)
    assert n1 > 0
    _same(plain, tail, f"lanes {lanes} block {block}")


def test_tail_launch_multi_group_sims():
    # an 8100-particle vortex at 64-particle tiles: 127 tiles, so its barrier
    # spans 4 groups of workgroups, next to a cavity (the big vortex stops at
    # once: the two small sims are the remainder)
    banner("tail launch with multi-group sims")
    probs = lambda: [_loose(I.tgv2d(200, seed=11)), I.tgv2d(90, seed=9, re=500.0), I.cavity(30, re=800.0)]
    plain, _ = _run(probs(), D.FP32, 0, 5, 1, 64)
    tail, n1 = _run(probs(), D.FP32, 1, 5, 1, 64)
    assert n1 > 0
    _same(plain, tail, "multi-group")


def test_loop_schedules_in_fixed_iteration_call():
    banner("loop schedules in dtsph_pseudo_iterate with a fixed count")
    res = []
    for schedule in (0, 1, 2):
        sim = D.Sim(CASES["batch_mixed"](), precision=D.FP32)
        sim.set_option(D.OPT_TAIL_LOOP, schedule)
        sim.step(2)
        sim.predict()
        st, rep = sim.pseudo_iterate(17)
        sim.correct()
        res.append((st, rep, sim.get_state()))
        sim.close()
    st0, rep0, s0 = res[0]
    assert all(r["iters"] == 17 for r in rep0)
    for st, rep, s in res[1:]:
        assert st == st0 and rep == rep0
        for f in s0:
            assert np.array_equal(s0[f], s[f]), f


def test_loop_schedule_rejects_other_values():
    sim = D.Sim(CASES["batch_tgv"](), precision=D.FP32)
    for bad in (-1, 3):
        with pytest.raises(D.DtsphError):
            sim.set_option(D.OPT_TAIL_LOOP, bad)
    with pytest.raises(D.DtsphError):
        sim.set_option(D.OPT_TAIL_SPIN, -1)
    sim.close()


def test_tail_barrier_wait_that_gives_up_is_an_error():
    # Barrier waits limited to one poll: the first workgroup of a sim to arrive
    # leaves at once, the others give up at their next barrier, every kernel
    # ends, the sim publishes no report and the step returns an error. A fresh
    # context afterwards runs normally.
    banner("tail launch with barrier waits that give up")
    sim = D.Sim(CASES["batch_mixed"](), precision=D.FP32)
    sim.step(1)  # a first loop: the per-sim counts that cut the next ones
    sim.set_option(D.OPT_TAIL_SPIN, 1)
    with pytest.raises(D.DtsphError):
        for _ in range(6):
            sim.step(1)
    sim.close()
    plain, _ = _run(CASES["batch_tgv"](), D.FP32, 0, 3)
    tail, n1 = _run(CASES["batch_tgv"](), D.FP32, 1, 3)
    assert n1 > 0
    _same(plain, tail, "after an abandoned tail launch")
