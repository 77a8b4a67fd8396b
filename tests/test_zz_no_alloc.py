"""lb_rb_adjoint_noalloc (the reverse pass on the library's own scratch array, for callers that
cannot allocate device memory) against lb_rb_adjoint with a caller workspace, through the
C-ABI: two calls in a row on one GPU, the second with a smaller box and window, so the second
runs on whatever the first left in the scratch array; FP64 (gradients to 1e-12 relative: the
atomic accumulation of sampled-velocity adjoints is not order-deterministic) and FP32 (1e-6);
the contexts end in the same state bit for bit; the same with a free body and two MD steps
per fluid step (the body passes' tables and sums in the array); a window beyond the array is
refused before anything runs.
"""
import numpy as np
import pytest

from paper_1604_01829_amd import lbrb
from paper_1604_01829_amd import workloads as W
from tests.test_gpu_adjoint import TAUS, _case, _gpu, _weights

pytestmark = pytest.mark.gpu


def _small_case():
    rng = np.random.default_rng(21)
    shape = (8, 9, 7)
    bodies = [(W.sphere_beads(1.5, 12), np.array([3.7, 4.6, 3.2]), W.random_quaternion(rng),
               W.GAMMA_FIXED)]
    return shape, None, dict(u0=(0.006, -0.002, 0.001), g_ext=(1e-5, 0.0, 0.0), **TAUS), bodies


def _state(sim):
    return sim.save_state().cpu().numpy()


def _compare(with_ws, no_ws, tol):
    J0, g0, o0 = with_ws
    J1, g1, o1 = no_ws
    assert abs(J1 - J0) <= tol * abs(J0)
    assert np.abs(g1 - g0).max() <= tol * np.abs(g0).max()
    assert np.abs(o1 - o0).max() <= tol * np.abs(o0).max()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_reverse_pass_matches_the_workspace_one(precision):
    tol = 1e-12 if precision == "f64" else 1e-6
    for k, (case, T, K) in enumerate(((_case(False), 13, 5), (_case(True), 9, 4),
                                      (_small_case(), 6, 3))):
        shape, mask, pp, bodies = case
        a = _weights(T, len(bodies), seed=3 + k)
        ref = _gpu(shape, mask, pp, bodies, precision)
        sim = _gpu(shape, mask, pp, bodies, precision)
        ref.step(2)
        sim.step(2)
        need = lbrb.lb_adjoint_workspace_bytes(sim.ctx, T, K)
        assert 0 < need <= lbrb.LB_NOALLOC_SCRATCH_BYTES
        print(f"  call {k}: box {shape}, window {T}, checkpoints every {K}, {need} bytes",
              flush=True)
        want = ref.adjoint(T, a, checkpoint_every=K)
        got = sim.adjoint_noalloc(T, a, checkpoint_every=K)
        _compare(want, got, tol)
        assert np.array_equal(_state(ref), _state(sim))
        ref.close()
        sim.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_reverse_pass_with_free_bodies(precision):
    """The body passes (a free body beside a fixed one, two MD steps per fluid step, then one)
    on the scratch array: body tables, body adjoints and bead sums live there too."""
    from tests.test_gpu_adjoint import _free_case, _gpu_free
    tol = 1e-12 if precision == "f64" else 1e-6
    for k, (masked, md, T, K) in enumerate(((False, 2, 9, 4), (True, 1, 6, 3))):
        shape, mask, pp, bodies = _free_case(masked)
        a = _weights(T, len(bodies), seed=11 + k)
        ref = _gpu_free(shape, mask, pp, bodies, precision, md)
        sim = _gpu_free(shape, mask, pp, bodies, precision, md)
        need = lbrb.lb_adjoint_workspace_bytes(sim.ctx, T, K)
        assert 0 < need <= lbrb.LB_NOALLOC_SCRATCH_BYTES
        print(f"  call {k}: free body, {md} MD steps, window {T}, {need} bytes", flush=True)
        want = ref.adjoint(T, a, checkpoint_every=K)
        got = sim.adjoint_noalloc(T, a, checkpoint_every=K)
        _compare(want, got, tol)
        assert np.array_equal(_state(ref), _state(sim))
        ref.close()
        sim.close()


def test_noalloc_refuses_a_window_beyond_its_array():
    wl = W.workload(5)
    wl["params"]["kT"] = 0.0
    sim = lbrb.simulation_from_workload(wl, precision="f32")
    T, K = 40, 20
    assert lbrb.lb_adjoint_workspace_bytes(sim.ctx, T, K) > lbrb.LB_NOALLOC_SCRATCH_BYTES
    a = np.zeros((T, 1, 3))
    a[:, 0, 0] = 1.0 / T
    before = _state(sim)
    with pytest.raises(lbrb.LBError) as e:
        sim.adjoint_noalloc(T, a, checkpoint_every=K)
    assert e.value.code == lbrb.LB_ERR_ARG
    assert np.array_equal(before, _state(sim))
    sim.close()
