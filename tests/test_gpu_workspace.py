"""Caller-supplied workspace: moving a context's device arrays into a torch
tensor (and back) keeps every state field bit for bit, at any phase of the
step, and invalid workspaces are refused without touching the state."""
import numpy as np
import pytest
import torch

from paper_1904_00861_amd import dtsph as D
from paper_1904_00861_amd import inputs as I

from gpu_helpers import banner

pytestmark = pytest.mark.gpu


def _same(a, b):
    for f in a:
        assert np.array_equal(a[f], b[f]), f


@pytest.mark.parametrize("prec", [D.FP32, D.FP64])
def test_workspace_moves_state_bit_identical(prec):
    banner(f"workspace, precision {prec}")
    prob = I.cavity(20)  # walls and fluid: every array kind is in use
    ref = D.Sim(prob, precision=prec)
    sim = D.Sim(prob, precision=prec)
    need = D.dtsph_workspace_bytes(sim.ctx)
    assert need >= sim.info["device_bytes"]
    for s in (ref, sim):
        s.step(2)
    ws = torch.empty(need + 1024, dtype=torch.uint8, device="cuda")
    sim.use_workspace(ws)
    _same(ref.get_state(), sim.get_state())
    for s in (ref, sim):
        s.step(3)
    _same(ref.get_state(), sim.get_state())
    # move inside the pseudo-time loop, then continue the same step
    for s in (ref, sim):
        s.predict()
        s.pseudo_iterate(2)
    ws2 = torch.empty(need, dtype=torch.uint8, device="cuda")
    sim.use_workspace(ws2)
    del ws
    _same(ref.get_state(loop=True), sim.get_state(loop=True))
    for s in (ref, sim):
        s.pseudo_iterate(0)
        s.correct()
    _same(ref.get_state(), sim.get_state())
    sim.use_workspace(None)
    for s in (ref, sim):
        s.step(2)
    _same(ref.get_state(), sim.get_state())
    ref.close()
    sim.close()


def test_invalid_workspace_is_refused_and_state_kept():
    banner("invalid workspace")
    prob = I.tgv2d(24, seed=4)
    ref = D.Sim(prob, precision=D.FP32)
    sim = D.Sim(prob, precision=D.FP32)
    for s in (ref, sim):
        s.step(1)
    need = D.dtsph_workspace_bytes(sim.ctx)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(D.DtsphError) as e:
        D.dtsph_set_workspace(sim.ctx, small.data_ptr(), small.numel())
    assert e.value.status == D.ENOMEM
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(D.DtsphError) as e:
        D.dtsph_set_workspace(sim.ctx, big.data_ptr() + 4, need)
    assert e.value.status == D.EINVAL
    host = torch.empty(need, dtype=torch.uint8)
    with pytest.raises(D.DtsphError) as e:
        D.dtsph_set_workspace(sim.ctx, host.data_ptr(), need)
    assert e.value.status == D.EINVAL
    sim.use_workspace(big)
    with pytest.raises(D.DtsphError) as e:  # overlaps the current workspace
        D.dtsph_set_workspace(sim.ctx, big.data_ptr() + 256, need)
    assert e.value.status == D.EINVAL
    for s in (ref, sim):
        s.step(2)
    _same(ref.get_state(), sim.get_state())
    ref.close()
    sim.close()
