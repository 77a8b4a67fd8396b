"""General boundary masks (rows with several fluid runs) on the GPU against the oracle, through
the C-ABI.  Bounce-back boundary nodes (Sec. 1.1) may be arranged in any way: a fixed obstacle
inside a periodic box, two parallel pores in one box, a random porous medium, an obstacle of
moving-wall nodes.  The boundary nodes between the fluid runs of a row are stored as holes that
mirror their fluid neighbours' reflected populations; every case compares fields, all 19
populations, totals and bodies element by element with the oracle, whose mask is the plain
per-node rule, FP64 and FP32, thermal and deterministic, eager and in graph replays.
"""
import numpy as np
import pytest

from paper_1604_01829_amd import lbrb
from paper_1604_01829_amd import workloads as W
from tests.helpers import compare, gpu_from_workload, oracle_from_workload
from tests.test_gpu_parity import _assert_close, _print

pytestmark = pytest.mark.gpu


def _tol(precision):
    return (1e-11, 1e-13, 1e-12) if precision == "f64" else (1e-5, 1e-6, 1e-6)


def _sphere(c, R, rng, fixed=False):
    offs = W.sphere_beads(R, W.sphere_bead_count(R))
    m, I = W.solid_body_mass_inertia(1.0, R, R, R)
    return W.body_record(offs, m, I, c, quat=W.random_quaternion(rng),
                         vel=(0.0, 0.0, 0.0) if fixed else rng.normal(0, 1e-3, 3),
                         omega=(0.0, 0.0, 0.0) if fixed else rng.normal(0, 1e-3, 3),
                         gamma=W.GAMMA_FIXED if fixed else W.GAMMA_FREE, fixed=fixed)


def obstacle_mask():
    """20 x 18 x 22 periodic box with a solid block (wall 1) and a plate (wall 2) inside it:
    the rows through them hold two fluid runs."""
    m = np.zeros((22, 18, 20), dtype=np.uint8)
    m[8:14, 6:12, 7:12] = 1
    m[:, 0:9, 15] = 2
    return m


def two_pores_mask(nx=40, ny=20, nz=24, r=7.0):
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    fluid = np.zeros((ny, nx), dtype=bool)
    for cx in (nx / 4.0, 3 * nx / 4.0):
        fluid |= np.hypot(x[None, :] - cx, y[:, None] - ny / 2.0) <= r
    return np.ascontiguousarray(np.broadcast_to((~fluid).astype(np.uint8)[None], (nz, ny, nx)))


def obstacle_case(precision, kT, walls=None):
    rng = np.random.default_rng(5)
    return dict(name="obstacle", precision=precision, steps=30,
                params=W.default_params(kT=kT, g_ext=(2e-6, -1e-6, 3e-6), tau_shear=0.8,
                                        tau_bulk=1.1, tau_odd=0.9, tau_even=1.2),
                replicas=[dict(shape=(20, 18, 22), seed=2024, mask=obstacle_mask(),
                               walls=walls or {},
                               bodies=[_sphere(np.array([15.4, 14.1, 15.2]), 2.0, rng)])])


def two_pores_case(precision, kT):
    rng = np.random.default_rng(6)
    return dict(name="two pores", precision=precision, steps=30,
                params=W.default_params(kT=kT, g_ext=(0.0, 0.0, 2e-6), tau_shear=0.9),
                replicas=[dict(shape=(40, 20, 24), seed=77, mask=two_pores_mask(),
                               bodies=[_sphere(np.array([10.3, 9.8, 5.1]), 2.0, rng),
                                       _sphere(np.array([29.6, 10.4, 16.7]), 2.5, rng)])])


def porous_case(precision):
    rng = np.random.default_rng(7)
    m = (rng.random((16, 16, 16)) < 0.15).astype(np.uint8) * 3
    return dict(name="porous", precision=precision, steps=30,
                params=W.default_params(kT=0.0, g_ext=(1e-5, 2e-6, 0.0), tau_shear=0.7,
                                        tau_bulk=0.9, tau_odd=1.1, tau_even=1.3),
                replicas=[dict(shape=(16, 16, 16), seed=9, mask=m, bodies=[])])


def _run(wl, precision, steps=(1, 3, 30), graph=False, tag=""):
    gpu = gpu_from_workload(wl)
    gpu.set_graph_steps(10 if graph else 0)
    orc = oracle_from_workload(wl)
    done = 0
    for s in steps:
        gpu.step(s - done)
        orc.step(s - done)
        done = s
        e = compare(gpu, orc)
        _print(f"{tag} {precision} step {s}", e)
        _assert_close(e, *_tol(precision))
    return gpu, orc


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("kT", [0.0, 4e-5])
def test_obstacle_in_a_periodic_box(precision, kT):
    gpu, _ = _run(obstacle_case(precision, kT), precision, tag=f"obstacle kT={kT}")
    m = obstacle_mask()
    assert gpu.node_counts(0) == (m.size, int((m == 0).sum()))
    gpu.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_two_parallel_pores(precision):
    gpu, _ = _run(two_pores_case(precision, 4e-5), precision, tag="two pores")
    gpu.close()


def test_random_porous_medium_fp64():
    gpu, _ = _run(porous_case("f64"), "f64", steps=(1, 7, 30), tag="porous")
    gpu.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_moving_obstacle_walls(precision):
    """The plate's nodes (wall 2), holes of their rows, move; the block stays."""
    wl = obstacle_case(precision, 0.0, walls={2: (0.0, 0.0, 1e-3)})
    gpu, _ = _run(wl, precision, tag="moving plate")
    gpu.close()


def test_graph_replay_with_holes_matches_eager_bitwise():
    wl = two_pores_case("f32", 4e-5)
    a = gpu_from_workload(wl)
    b = gpu_from_workload(wl)
    a.set_graph_steps(0)
    b.set_graph_steps(10)
    a.step(23)
    b.step(23)
    assert np.array_equal(a.save_state().cpu().numpy(), b.save_state().cpu().numpy())
    a.close()
    b.close()
    _run(two_pores_case("f32", 4e-5), "f32", steps=(20, 40), graph=True, tag="two pores graph")


def test_batch_with_holed_and_plain_replicas():
    ob = obstacle_case("f32", 4e-5)["replicas"][0]
    tp = two_pores_case("f32", 4e-5)["replicas"][0]
    rng = np.random.default_rng(8)
    L = 24
    pore = dict(shape=(L, L, L), seed=5, mask=W.pore_mask(L, L, L, 9.0),
                bodies=[_sphere(np.array([12.4, 11.7, 6.0]), 2.0, rng)])
    dense = dict(shape=(12, 14, 10), seed=6, mask=None, bodies=[])
    wl = dict(name="mixed", precision="f32", steps=12,
              params=W.default_params(kT=4e-5, g_ext=(1e-6, 0.0, 2e-6)),
              replicas=[ob, pore, tp, dense])
    gpu = gpu_from_workload(wl)
    gpu.set_graph_steps(0)
    gpu.step(12)
    for r in range(4):
        orc = oracle_from_workload(wl, r)
        orc.step(12)
        e = compare(gpu, orc, r)
        _print(f"mixed batch replica {r}", e)
        _assert_close(e, *_tol("f32"))
    gpu.close()


def baffle_case(precision, kT, walls=None):
    """The 24 x 22 x 40 pore along z of the parity tests with a baffle (wall 2) across half of
    its cross-section at z = 20: the library stores this replica in rows along z (the pore
    axis), and the rows through the baffle hold two fluid runs (holes)."""
    from tests.test_gpu_parity import pore_case
    wl = pore_case(precision, kT)
    m = wl["replicas"][0]["mask"].copy()
    nz, ny, nx = m.shape
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    half = (yy < ny // 2) & (m[20] == 0)
    m[20][half] = 2
    wl["replicas"][0]["mask"] = m
    wl["replicas"][0]["walls"] = walls or {}
    # keep the bodies clear of the baffle
    wl["replicas"][0]["bodies"] = [b for b in wl["replicas"][0]["bodies"]
                                   if abs(b["pos"][2] - 20.5) > 5.0]
    return wl


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("moving", [False, True])
def test_pore_with_a_baffle_stored_along_the_pore(precision, moving):
    wl = baffle_case(precision, 0.0 if moving else 4e-5,
                     walls={2: (1e-3, 0.0, -5e-4)} if moving else None)
    gpu, _ = _run(wl, precision, tag=f"baffle moving={moving}")
    assert gpu.row_axis(0) == 2
    m = wl["replicas"][0]["mask"]
    assert gpu.node_counts(0) == (m.size, int((m == 0).sum()))
    gpu.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_reverse_pass_with_holes_matches_oracle(precision):
    """The reverse pass in the obstacle box (rows with two fluid runs, so the block and the
    plate are stored as holes): a free sphere in the flow and a fixed one whose stencils reach
    into the block, against the oracle's reverse pass (which reads the mask directly)."""
    from tests.helpers import oracle_from_workload
    rng = np.random.default_rng(3)
    free = _sphere(np.array([15.4, 14.1, 15.2]), 2.0, rng)
    fixed = _sphere(np.array([13.8, 9.0, 10.5]), 1.5, rng, fixed=True)
    wl = dict(name="obstacle", precision=precision, steps=11,
              params=W.default_params(kT=0.0, g_ext=(2e-6, -1e-6, 3e-6), tau_shear=0.8,
                                      tau_bulk=1.1, tau_odd=0.9, tau_even=1.2),
              replicas=[dict(shape=(20, 18, 22), seed=1, mask=obstacle_mask(),
                             bodies=[free, fixed])])
    # some bead of the fixed sphere samples a node of the block
    pos = fixed["pos"] + fixed["offsets"] @ _rotation(fixed["quat"]).T
    lo = np.floor(pos - 0.5).astype(int)
    m = obstacle_mask()
    assert any(m[(lo[k, 2] + dz) % 22, (lo[k, 1] + dy) % 18, (lo[k, 0] + dx) % 20] == 1
               for k in range(len(pos)) for dx in (0, 1) for dy in (0, 1) for dz in (0, 1))
    T, K = 11, 4
    a = np.zeros((T, 2, 3))
    a[:, 0, 0] = 1.0 / T
    a += 0.02 * rng.standard_normal(a.shape)
    print(f"reverse pass with holes: {precision}", flush=True)
    Jo, dgo, doo = oracle_from_workload(wl).adjoint(T, a)
    sim = gpu_from_workload(wl)
    Jg, dgg, dog = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    print(f"  J rel {abs(Jg - Jo) / abs(Jo):.2e}  dgamma rel "
          f"{np.abs(dgg - dgo).max() / np.abs(dgo).max():.2e}  doffsets rel "
          f"{np.abs(dog - doo).max() / np.abs(doo).max():.2e}", flush=True)
    tJ, tg = (1e-12, 1e-10) if precision == "f64" else (2e-6, 5e-6)
    assert abs(Jg - Jo) <= tJ * abs(Jo), (Jg, Jo)
    assert np.abs(dgg - dgo).max() <= tg * np.abs(dgo).max(), (dgg, dgo)
    assert np.abs(dog - doo).max() <= tg * np.abs(doo).max(), np.abs(dog - doo).max()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_reverse_pass_in_the_baffled_pore_stored_along_it(precision):
    """The reverse pass in the baffled pore, which the library stores in rows along z with
    holes in the rows through the baffle (axes exchanged: the transposed mirror and the
    transposed pull take c_i in storage coordinates), thermal, with the baffle moving, against
    the oracle's reverse pass."""
    from tests.helpers import oracle_from_workload
    wl = baffle_case(precision, 4e-5, walls={2: (1e-3, 0.0, -5e-4)})
    nb = len(wl["replicas"][0]["bodies"])
    assert nb >= 1
    T, K = 10, 4
    rng = np.random.default_rng(8)
    a = np.zeros((T, nb, 3))
    a[:, 0, 2] = 1.0 / T
    a += 0.02 * rng.standard_normal(a.shape)
    print(f"reverse pass, baffled pore stored along z: {precision}", flush=True)
    Jo, dgo, doo = oracle_from_workload(wl).adjoint(T, a)
    sim = gpu_from_workload(wl)
    assert sim.row_axis(0) == 2
    Jg, dgg, dog = sim.adjoint(T, a, checkpoint_every=K)
    sim.close()
    print(f"  J rel {abs(Jg - Jo) / abs(Jo):.2e}  dgamma rel "
          f"{np.abs(dgg - dgo).max() / np.abs(dgo).max():.2e}  doffsets rel "
          f"{np.abs(dog - doo).max() / np.abs(doo).max():.2e}", flush=True)
    tJ, tg = (1e-12, 1e-10) if precision == "f64" else (2e-6, 5e-6)
    assert abs(Jg - Jo) <= tJ * abs(Jo), (Jg, Jo)
    assert np.abs(dgg - dgo).max() <= tg * np.abs(dgo).max(), (dgg, dgo)
    assert np.abs(dog - doo).max() <= tg * np.abs(doo).max(), np.abs(dog - doo).max()


def _rotation(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
