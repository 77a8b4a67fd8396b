"""The node-update launch settings (lb_autotune, lb_set_tuning) through the C-ABI: timing
them leaves the simulation state unchanged, and no setting changes a result -- every case
compares whole saved states (populations, bodies, step) bit for bit with the default settings.
"""
import numpy as np
import pytest

from paper_1604_01829_amd import lbrb
from paper_1604_01829_amd import workloads as W
from tests.helpers import gpu_from_workload
from tests.test_gpu_runtime import pore_batch

pytestmark = pytest.mark.gpu


def _state(sim):
    return sim.save_state().cpu().numpy()


def test_autotune_leaves_the_state_and_results_unchanged():
    wl = pore_batch()
    a = gpu_from_workload(wl)
    b = gpu_from_workload(wl)
    a.step(10)
    b.step(10)
    t = b.autotune(repeats=2)
    # small boxes: the populations fit in the Infinity Cache, so ordinary stores only
    assert t["tuned"] and t["candidates"] == 8 and not t["streaming_stores"]
    assert t["node_us_tuned"] <= t["node_us_default"]
    assert np.array_equal(_state(a), _state(b))     # timing the settings changed nothing
    a.step(30)
    b.step(30)
    assert np.array_equal(_state(a), _state(b))     # nor do the chosen settings
    # a second context of the same shape takes the kept result without timing
    c = gpu_from_workload(wl)
    assert c.autotune(repeats=0) == t
    for s in (a, b, c):
        s.close()


def test_autotune_times_both_store_kinds_beyond_the_cache():
    """A box whose two FP32 population buffers (2 x 0.8 GB) exceed the 256 MB Infinity Cache:
    ordinary and non-temporal stores are both timed; the state stays unchanged."""
    wl = dict(name="large", precision="f32", steps=4,
              params=W.default_params(kT=4e-5, g_ext=(1e-6, 0.0, 0.0)),
              replicas=[dict(shape=(256, 256, 80), seed=8, mask=None, bodies=[])])
    a = gpu_from_workload(wl)
    a.step(2)
    before = _state(a)
    t = a.autotune(repeats=1)
    assert t["tuned"] and t["candidates"] == 16
    assert np.array_equal(before, _state(a))
    a.close()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_every_launch_setting_gives_the_same_results(precision):
    wl = pore_batch()
    wl["precision"] = precision
    ref = gpu_from_workload(wl)
    ref.set_graph_steps(10)
    ref.step(23)
    want = _state(ref)
    ref.close()
    for per, cap, st in ((4, 0, False), (4, 5, True), (1, 4, False), (1, 6, True), (4, 1, False)):
        s = gpu_from_workload(wl)
        s.set_tuning(tiles_per_wg=per, wg_per_cu=cap, streaming=st)
        got = s.tuned_settings()
        assert got["tiles_per_wg"] == per and got["wg_per_cu"] == cap
        assert got["streaming_stores"] == st
        s.set_graph_steps(10)
        s.step(23)
        assert np.array_equal(want, _state(s)), (per, cap, st)
        s.close()


def test_tuning_arguments_are_checked():
    s = gpu_from_workload(W.workload(1))
    for bad in (dict(tiles_per_wg=0), dict(tiles_per_wg=2), dict(wg_per_cu=-1),
                dict(wg_per_cu=33)):
        with pytest.raises(lbrb.LBError) as e:
            s.set_tuning(**bad)
        assert e.value.code == lbrb.LB_ERR_ARG
    with pytest.raises(lbrb.LBError) as e:
        s.autotune(repeats=1001)
    assert e.value.code == lbrb.LB_ERR_ARG
    s.close()
