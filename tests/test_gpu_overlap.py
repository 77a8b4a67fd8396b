"""The overlapped fluid step against the serial one, through the C-ABI.

The overlapped step runs the coupling in the same launch as the node update of the tiles that
receive no spread force, and the body finishing (which marks the tiles under the next step's
bead stencils) with the node update of the marked tiles.  It must reproduce the serial step
bit for bit: populations and body records after graph replays and eager steps, on dense and
masked replicas, thermal and deterministic, with bodies that move across tiles, moving walls,
a batch of pores, a checkpoint reloaded, a policy switched mid-run and a body added mid-run.
Contexts it does not cover (mixed dense and masked replicas, MD sub-steps, excluded volume)
fall back to the serial step.
"""
import numpy as np
import pytest

from paper_1604_01829_amd import lbrb
from paper_1604_01829_amd import workloads as W
from tests.helpers import gpu_from_workload

pytestmark = pytest.mark.gpu


def _state(sim):
    return sim.save_state().cpu().numpy()


def _moving_sphere(precision):
    """A sphere crossing the 256-node tiles of a 24^3 box (about 5 lattice units in 60 steps)
    while it spins, thermal."""
    R = 3.0
    offs = W.sphere_beads(R, W.sphere_bead_count(R))
    m, I = W.solid_body_mass_inertia(1.0, R, R, R)
    body = W.body_record(offs, m, I, (5.3, 11.7, 19.2), quat=(0.9, 0.1, -0.3, 0.2),
                         vel=(0.08, -0.05, 0.03), omega=(0.01, -0.02, 0.015), gamma=W.GAMMA_FREE)
    return dict(name="moving sphere", precision=precision, steps=60,
                params=W.default_params(kT=4e-5),
                replicas=[dict(shape=(24, 24, 24), seed=77, mask=None, bodies=[body])])


def _case(name, precision):
    if name == "sphere":
        wl = W.workload(1)
        wl["params"]["kT"] = 4e-5
        return wl
    if name == "pore":
        return W.workload(2, scale=0.5)
    if name == "moving":
        return _moving_sphere(precision)
    if name == "walls":
        return W.stokes_flow_workload(L=16, radius=3.0)
    if name == "batch":
        return W.workload(4, scale=0.02)
    raise ValueError(name)


def _run(wl, precision, policy, steps, graph_steps):
    sim = gpu_from_workload(wl, precision=precision)
    sim.set_step_policy(policy)
    sim.set_graph_steps(graph_steps)
    sim.step(steps)
    return sim


@pytest.mark.parametrize("name", ["sphere", "pore", "moving", "walls", "batch"])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_overlapped_step_matches_serial_bitwise(name, precision):
    wl = _case(name, precision)
    a = _run(wl, precision, lbrb.LB_STEP_SERIAL, 0, 20)
    b = _run(wl, precision, lbrb.LB_STEP_OVERLAP, 0, 20)
    assert not a.step_overlapped() and b.step_overlapped()
    for n in (47, 13):            # graph replays of both buffer parities, then eager steps
        a.step(n)
        b.step(n)
        assert np.array_equal(_state(a), _state(b)), (name, precision, n)
    ta, ba, _, rc = a.observables(0)
    tb, bb, _, rc2 = b.observables(0)
    assert rc == 0 and rc2 == 0 and ta["step"] == tb["step"] == 60
    a.close()
    b.close()


def test_checkpoint_and_policy_switch():
    wl = W.workload(2, scale=0.5)
    ref = _run(wl, "f32", lbrb.LB_STEP_SERIAL, 30, 0)
    # overlapped 10, checkpoint, overlapped 20 more
    a = _run(wl, "f32", lbrb.LB_STEP_OVERLAP, 10, 0)
    ck = a.save_state()
    a.step(20)
    assert np.array_equal(_state(a), _state(ref))
    # resume the checkpoint in a fresh overlapped context
    b = gpu_from_workload(wl)
    b.set_step_policy(lbrb.LB_STEP_OVERLAP)
    b.load_state(ck)
    b.step(20)
    assert np.array_equal(_state(b), _state(ref))
    # serial 10, overlapped 10 (tile marks rebuilt), serial 10
    c = _run(wl, "f32", lbrb.LB_STEP_SERIAL, 10, 0)
    c.set_step_policy(lbrb.LB_STEP_OVERLAP)
    c.step(10)
    c.set_step_policy(lbrb.LB_STEP_SERIAL)
    c.step(10)
    assert np.array_equal(_state(c), _state(ref))
    for s in (ref, a, b, c):
        s.close()


def test_body_added_mid_run():
    wl = _moving_sphere("f32")
    R = 2.5
    offs = W.sphere_beads(R, W.sphere_bead_count(R))
    m, I = W.solid_body_mass_inertia(1.0, R, R, R)
    out = []
    for policy in (lbrb.LB_STEP_SERIAL, lbrb.LB_STEP_OVERLAP):
        sim = lbrb.simulation_from_workload(wl, max_extra_bodies=1,
                                            max_extra_beads=offs.shape[0])
        sim.set_step_policy(policy)
        sim.step(15)
        sim.add_body(0, offs, m, I, (17.0, 6.0, 9.5), (1.0, 0.0, 0.0, 0.0), (-0.04, 0.02, 0.0),
                     (0.0, 0.0, 0.0), W.GAMMA_FREE, False)
        sim.step(25)
        out.append(_state(sim))
        sim.close()
    assert np.array_equal(out[0], out[1])


def _overlap_requested(sim):
    sim.set_step_policy(lbrb.LB_STEP_OVERLAP)
    return sim.step_overlapped()


def test_uncovered_contexts_fall_back_to_the_serial_step():
    from tests.test_gpu_runtime import pore_batch
    plain = gpu_from_workload(W.workload(1))       # the default is the serial step
    assert not plain.step_overlapped() and _overlap_requested(plain)
    plain.close()
    mixed = gpu_from_workload(pore_batch())        # masked and dense replicas
    assert not _overlap_requested(mixed)
    mixed.close()
    wl = W.workload(1)
    wl["params"]["md_substeps"] = 2                # MD sub-steps
    md = gpu_from_workload(wl)
    assert not _overlap_requested(md)
    md.close()
    wl = W.workload(1)                             # excluded volume
    wl["params"]["wca_epsilon"] = 1e-4
    wl["replicas"][0]["bodies"][0]["ev"] = (W.inner_layer_sphere(3.0), 0.5)
    ev = gpu_from_workload(wl)
    assert not _overlap_requested(ev)
    ev.step(3)
    ev.close()
    empty = lbrb.simulation_from_workload(dict(name="empty", precision="f32", steps=0,
                                               params=W.default_params(),
                                               replicas=[dict(shape=(8, 8, 8), seed=1,
                                                              mask=None, bodies=[])]))
    assert not _overlap_requested(empty)           # no bodies: nothing to overlap
    with pytest.raises(lbrb.LBError):
        empty.set_step_policy(9)
    empty.close()
