"""Error handling of the C-ABI on the GPU: invalid descriptions, call order,
capacity overflow, non-finite state and the iteration cap. Every condition is
forced from the host; no kernel faults or hangs."""
import numpy as np
import pytest

from paper_1904_00861_amd import dtsph as D
from paper_1904_00861_amd import inputs as I

from gpu_helpers import banner

pytestmark = pytest.mark.gpu


def _create(prob, **over):
    prm = dict(prob.params, **over)
    return D.dtsph_create([prm], [prob.n_fluid], [prob.n_wall], D.FP32)


@pytest.mark.parametrize("over,msg", [
    (dict(h=0.2), "half the period"),       # kappa h = 0.6 >= L/2 on a periodic axis
    (dict(dim=1), "dim"),
    (dict(dt=0.0), "dt"),
    (dict(stall_window=9), "stall_window"),
    (dict(max_iter=0), "max_iter"),
    (dict(hi=(0.0, 1.0, 1.0)), "hi must exceed lo"),
])
def test_invalid_descriptions(over, msg):
    banner(f"invalid {over}")
    with pytest.raises(D.DtsphError) as e:
        _create(I.tgv2d(10), **over)
    assert e.value.status == D.EINVAL and msg in str(e.value)


def test_invalid_counts_and_precision():
    prob = I.tgv2d(10)
    with pytest.raises(D.DtsphError) as e:
        D.dtsph_create([prob.params], [0], [0], D.FP32)
    assert e.value.status == D.EINVAL
    with pytest.raises(D.DtsphError) as e:
        D.dtsph_create([prob.params], [prob.n], [0], 7)
    assert e.value.status == D.EINVAL
    with pytest.raises(D.DtsphError) as e:
        D.dtsph_create([prob.params, I.tgv3d(8).params], [prob.n, 512], [0, 0], D.FP32)
    assert e.value.status == D.EINVAL


def test_call_order():
    banner("call order")
    sim = D.Sim(I.tgv2d(12), precision=D.FP32)
    with pytest.raises(D.DtsphError) as e:
        sim.pseudo_iterate(1)
    assert e.value.status == D.EINVAL
    with pytest.raises(D.DtsphError):
        sim.correct()
    with pytest.raises(D.DtsphError):
        sim.get_state(loop=True)
    sim.predict()
    with pytest.raises(D.DtsphError):
        sim.predict()
    with pytest.raises(D.DtsphError):
        sim.step(1)
    sim.pseudo_iterate(2)
    sim.correct()
    st, reps = sim.step(1)
    assert st >= 0
    with pytest.raises(D.DtsphError):
        sim.set_option(D.OPT_BLOCK, 100)
    sim.close()


def test_neighbour_capacity_overflow():
    banner("capacity overflow")
    prob = I.tgv2d(16)
    prob.params["max_neighbors"] = 8
    sim = D.Sim(prob, precision=D.FP32)
    with pytest.raises(D.DtsphError) as e:
        sim.build_cells()
    assert e.value.status == D.EOVERFLOW and "needs" in str(e.value)
    sim.close()


def test_nonfinite_pressure():
    banner("non-finite")
    prob = I.tgv2d(16)
    prob.p[5] = np.nan
    sim = D.Sim(prob, precision=D.FP64)
    sim.predict()
    with pytest.raises(D.DtsphError) as e:
        sim.pseudo_iterate(0)
    assert e.value.status == D.ENONFINITE
    sim.close()


def test_iteration_cap():
    banner("max_iter")
    prob = I.tgv2d(16)
    prob.params.update(tol=0.0, stall_rel=0.0, max_iter=3)
    sim = D.Sim(prob, precision=D.FP32)
    st, reps = sim.step(2)
    sim.close()
    assert st == D.WARN_MAXITER
    assert all(r[0]["iters"] == 3 and D.REASONS[r[0]["reason"]] == "max_iter" for r in reps)


@pytest.mark.parametrize("block", [64, 128, 256])
def test_block_and_xcd_options_do_not_change_results(block):
    banner(f"block {block}")
    prob = I.tgv2d(30, seed=5)
    ref = D.Sim(prob, precision=D.FP32)
    ref.step(2)
    a = ref.get_state()
    ref.close()
    sim = D.Sim(prob, precision=D.FP32)
    sim.set_option(D.OPT_BLOCK, block)
    sim.set_option(D.OPT_XCD_REMAP, 0)
    sim.set_option(D.OPT_CHUNK, 1)
    sim.step(2)
    b = sim.get_state()
    sim.close()
    # fields do not depend on the launch shape (residual sums may differ in the last bit)
    for f in a:
        assert np.array_equal(a[f], b[f])


def test_autotune_keeps_state_and_results():
    banner("autotune")
    prob = I.tgv2d(40, seed=9)
    sim = D.Sim(prob, precision=D.FP32)
    before = sim.get_state()
    rep = sim.autotune(repeats=2)
    after = sim.get_state()
    for f in before:
        assert np.array_equal(before[f], after[f])
    assert rep["n_entries"] if "n_entries" in rep else len(rep["entries"]) == 12
    assert (rep["lanes"], rep["block"]) in [(e["lanes"], e["block"]) for e in rep["entries"]]
    assert sim.info["lanes"] == rep["lanes"] and sim.info["block"] == rep["block"]
    st, reps = sim.step(2)
    tuned = sim.get_state()
    sim.close()
    ref = D.Sim(prob, precision=D.FP32)
    ref.set_option(D.OPT_LANES, 1)
    ref.step(2)
    plain = ref.get_state()
    ref.close()
    nf = prob.n_fluid
    assert np.linalg.norm(tuned["v"][:nf] - plain["v"][:nf]) <= 1e-5 * np.linalg.norm(plain["v"][:nf])


def test_periodic_position_outside_box_is_rejected():
    banner("periodic position outside [lo, hi)")
    prob = I.tgv2d(16, seed=1)
    prob.x[3, 0] = prob.params["hi"][0]  # == hi lies outside [lo, hi)
    with pytest.raises(D.DtsphError) as e:
        D.Sim(prob, precision=D.FP32)
    assert e.value.status == D.EINVAL
    prob.x[3, 0] = prob.params["lo"][0]  # == lo is inside
    sim = D.Sim(prob, precision=D.FP32)
    st, _ = sim.step(1)
    sim.close()
    assert st >= 0


def test_first_pass_timing_mode():
    # timing mode -1 samples the first pair pass of every loop (the whole batch
    # takes part) and every full build; -2 is rejected
    probs = [I.tgv2d(24, seed=1), I.cavity(14)]
    banner("first-pass timing mode")
    sim = D.Sim(probs, precision=D.FP32)
    with pytest.raises(D.DtsphError):
        sim.set_option(D.OPT_TIMING, -2)
    sim.set_option(D.OPT_TIMING, -1)
    sim.set_option(D.OPT_RESET_TIMING, 0)
    st, reps = sim.step(4)
    tm = sim.timing()
    sim.close()
    assert tm["pass_launches"] == 4
    assert tm["pass_pairs"] == sum(sum(r["pairs"] for r in step) for step in reps)
    assert tm["pass_particles"] == 4 * sum(p.n_fluid for p in probs)
    assert tm["build_launches"] == tm["full_builds"] and tm["build_particles"] == tm["full_builds"] * sum(p.n for p in probs)
    assert tm["pass_ms"] > 0 and tm["build_ms"] > 0
