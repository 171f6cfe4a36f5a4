"""HIP-graph replay of the step segment (rate pass, build, first chunk of
pseudo-iterations): every replayed step must equal plain launches bit for bit,
with eager work and synchronisation between replays, across changes of the
launch configuration, workspace moves and sampled timing."""
import numpy as np
import pytest
import torch

from paper_1904_00861_amd import dtsph as D
from paper_1904_00861_amd import inputs as I

from gpu_helpers import banner

pytestmark = pytest.mark.gpu

CASES = {
    "tgv2d_30": lambda: I.tgv2d(30, seed=5),
    "cavity_18": lambda: I.cavity(18),
    "tgv3d_8": lambda: I.tgv3d(8, seed=3),
    "batch_4": lambda: [I.tgv2d(20, seed=1), I.cavity(14), I.tgv2d(26, seed=2), I.cavity(10)],
}


def _same(a, b, what):
    for f in a:
        assert np.array_equal(a[f], b[f]), f"{what}: field {f}"


def _pair(case, prec):
    prob = CASES[case]()
    eager = D.Sim(prob, precision=prec)
    eager.set_option(D.OPT_GRAPHS, 0)
    graph = D.Sim(prob, precision=prec)
    graph.set_option(D.OPT_GRAPHS, 1)
    return eager, graph


@pytest.mark.parametrize("prec", [D.FP32, D.FP64])
@pytest.mark.parametrize("case", list(CASES))
def test_graph_replays_match_plain_launches(case, prec):
    banner(f"graph replay {case} precision {prec}")
    eager, graph = _pair(case, prec)
    for step in range(6):  # first step records, later ones replay
        st_e, rep_e = eager.step(1)
        st_g, rep_g = graph.step(1)
        assert st_e == st_g
        assert rep_e == rep_g, f"step {step}"
        _same(eager.get_state(), graph.get_state(), f"step {step}")
        torch.cuda.synchronize()
    eager.close()
    graph.close()


def test_graph_with_sampled_timing_and_reconfiguration():
    banner("graph replay with timing, options and workspace moves")
    eager, graph = _pair("cavity_18", D.FP32)
    for s in (eager, graph):
        s.set_option(D.OPT_TIMING, 2)  # every other pair pass timed: mixes plain and replayed steps
    for step in range(4):
        eager.step(1)
        graph.step(1)
    _same(eager.get_state(), graph.get_state(), "timed")
    for s in (eager, graph):
        s.set_option(D.OPT_LANES, 4)
        s.set_option(D.OPT_BLOCK, 128)
    for step in range(3):
        eager.step(1)
        graph.step(1)
        _same(eager.get_state(), graph.get_state(), f"reconfigured step {step}")
    need = D.dtsph_workspace_bytes(graph.ctx)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    graph.use_workspace(ws)  # recorded graphs hold the old addresses
    for step in range(3):
        eager.step(1)
        graph.step(1)
        _same(eager.get_state(), graph.get_state(), f"moved step {step}")
    tg, te = graph.timing(), eager.timing()
    assert tg["pass_launches"] > 0 and te["pass_launches"] > 0
    eager.close()
    graph.close()


def test_graph_multi_step_call_matches():
    banner("graph replay inside one multi-step call")
    eager, graph = _pair("tgv2d_30", D.FP32)
    st_e, rep_e = eager.step(8)
    st_g, rep_g = graph.step(8)
    assert rep_e == rep_g
    _same(eager.get_state(), graph.get_state(), "8 steps")
    eager.close()
    graph.close()
