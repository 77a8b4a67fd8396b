"""Python binding of the gfx950 raspberry / lattice-Boltzmann library (``liblbrb.so``).

The functions carry the C-ABI's names (``lb_init``, ``lb_set_boundary_mask``,
``rb_add_raspberry``, ``lb_rb_step``, ``lb_observables``, ...) and only marshal arguments:
every step of the method runs in the HIP kernels of the library.  ``Simulation`` wraps one
context and takes its device workspace and stream from PyTorch.

There is no CPU fallback: importing works anywhere, but loading the library raises if it
has not been built (``python -m paper_1604_01829_amd.build``) and creating a context raises if
no GPU is visible.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbrb.so")

LB_OK = 0
LB_ERR_ARG = -1
LB_ERR_STATE = -2
LB_ERR_HIP = -3
LB_ERR_UNSTABLE = -4
LB_ERR_CAPACITY = -5
LB_PRECISION_F64 = 0
LB_PRECISION_F32 = 1
LB_STORES_AUTO, LB_STORES_CACHED, LB_STORES_STREAMING = 0, 1, 2
LB_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

# every symbol declared in include/lbrb.h
EXPORTED = ["lb_workspace_bytes", "lb_init", "lb_set_boundary_mask", "lb_set_wall_velocity",
            "rb_add_raspberry", "rb_set_excluded_volume", "lb_add_wall_sites", "rb_record_poses",
            "lb_traj_lab_frame", "lb_traj_body_frame", "lb_traj_pore_frame", "lb_traj_msd",
            "lb_traj_rotation_msd", "lb_traj_binned_msd", "rb_relax_shells", "lb_rb_step",
            "lb_observables", "lb_body_count", "rb_bead_forces", "lb_export_populations",
            "lb_inject_nan", "lb_save_state", "lb_load_state", "lb_set_graph_steps",
            "lb_set_timing", "lb_kernel_times", "lb_set_store_policy", "lb_autotune",
            "lb_get_tuning", "lb_set_tuning", "lb_adjoint_workspace_bytes", "lb_rb_adjoint",
            "lb_rb_adjoint_noalloc", "lb_node_counts", "lb_row_axis", "lb_destroy",
            "lb_last_error"]


class lb_replica(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class lb_params(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rho0", ctypes.c_double),
                ("u0", ctypes.c_double * 3), ("tau_shear", ctypes.c_double),
                ("tau_bulk", ctypes.c_double), ("tau_odd", ctypes.c_double),
                ("tau_even", ctypes.c_double), ("kT", ctypes.c_double),
                ("g_ext", ctypes.c_double * 3), ("max_bodies", ctypes.c_int32),
                ("max_beads", ctypes.c_int32), ("max_wall_links", ctypes.c_int32),
                ("md_substeps", ctypes.c_int32), ("wca_epsilon", ctypes.c_double),
                ("max_ev_sites", ctypes.c_int32), ("max_wall_sites", ctypes.c_int32)]


class rb_relax_params(ctypes.Structure):
    _fields_ = [("k_surface", ctypes.c_double), ("sigma", ctypes.c_double),
                ("epsilon", ctypes.c_double), ("damping", ctypes.c_double),
                ("dt", ctypes.c_double), ("mass", ctypes.c_double)]


class lb_tuning(ctypes.Structure):
    _fields_ = [("tuned", ctypes.c_int32), ("tiles_per_wg", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("streaming", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("node_us_default", ctypes.c_double),
                ("node_us_tuned", ctypes.c_double)]


class lb_totals(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
                ("body_momentum", ctypes.c_double * 3), ("step", ctypes.c_int64),
                ("finite", ctypes.c_int32)]


class rb_state(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_double * 3), ("quat", ctypes.c_double * 4),
                ("vel", ctypes.c_double * 3), ("omega_body", ctypes.c_double * 3),
                ("force", ctypes.c_double * 3), ("torque", ctypes.c_double * 3)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p


def library():
    """Load liblbrb.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1604_01829_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.lb_workspace_bytes.restype = ctypes.c_size_t
    L.lb_workspace_bytes.argtypes = [ctypes.POINTER(lb_params), ctypes.POINTER(lb_replica),
                                     ctypes.c_int32]
    L.lb_init.restype = ctypes.c_int
    L.lb_init.argtypes = [ctypes.POINTER(lb_params), ctypes.POINTER(lb_replica), ctypes.c_int32,
                          _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]
    L.lb_set_boundary_mask.restype = ctypes.c_int
    L.lb_set_boundary_mask.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8)]
    L.lb_set_wall_velocity.restype = ctypes.c_int
    L.lb_set_wall_velocity.argtypes = [_VP, ctypes.c_int32, ctypes.c_int32, _D]
    L.rb_set_excluded_volume.restype = ctypes.c_int
    L.rb_set_excluded_volume.argtypes = [_VP, ctypes.c_int32, ctypes.c_int32, _D, ctypes.c_int32,
                                         ctypes.c_double]
    L.lb_add_wall_sites.restype = ctypes.c_int
    L.lb_add_wall_sites.argtypes = [_VP, ctypes.c_int32, _D, ctypes.c_int32, ctypes.c_double]
    L.rb_record_poses.restype = ctypes.c_int
    L.rb_record_poses.argtypes = [_VP, _VP]
    i32 = ctypes.c_int32
    for name in ("lb_traj_lab_frame", "lb_traj_body_frame"):
        getattr(L, name).restype = ctypes.c_int
        getattr(L, name).argtypes = [_VP, i32, i32, _VP, _VP]
    L.lb_traj_pore_frame.restype = ctypes.c_int
    L.lb_traj_pore_frame.argtypes = [_VP, i32, i32, ctypes.c_double, ctypes.c_double, _VP, _VP,
                                       _VP]
    L.lb_traj_msd.restype = ctypes.c_int
    L.lb_traj_msd.argtypes = [_VP, i32, i32, i32, i32, _VP, _VP]
    L.lb_traj_rotation_msd.restype = ctypes.c_int
    L.lb_traj_rotation_msd.argtypes = [_VP, i32, i32, _VP, i32, _VP, _VP]
    L.lb_traj_binned_msd.restype = ctypes.c_int
    L.lb_traj_binned_msd.argtypes = [_VP, _VP, i32, i32, i32, _VP, i32, i32, _VP, _VP, _VP]
    L.rb_relax_shells.restype = ctypes.c_int
    L.rb_relax_shells.argtypes = [ctypes.c_int32, _D, ctypes.POINTER(ctypes.c_int32), _VP, _VP,
                                  ctypes.POINTER(rb_relax_params), ctypes.c_int32, _VP]
    L.rb_add_raspberry.restype = ctypes.c_int
    L.rb_add_raspberry.argtypes = [_VP, ctypes.c_int32, _D, ctypes.c_int32, ctypes.c_double, _D,
                                   _D, _D, _D, _D, ctypes.c_double, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)]
    L.lb_rb_step.restype = ctypes.c_int
    L.lb_rb_step.argtypes = [_VP, ctypes.c_int32]
    L.lb_observables.restype = ctypes.c_int
    L.lb_observables.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(lb_totals),
                                 ctypes.POINTER(rb_state), _VP]
    L.lb_body_count.restype = ctypes.c_int
    L.lb_body_count.argtypes = [_VP, ctypes.c_int32]
    L.rb_bead_forces.restype = ctypes.c_int
    L.rb_bead_forces.argtypes = [_VP, ctypes.c_int32, ctypes.c_int32, _D, ctypes.c_int32]
    L.lb_export_populations.restype = ctypes.c_int
    L.lb_export_populations.argtypes = [_VP, ctypes.c_int32, _VP]
    L.lb_inject_nan.restype = ctypes.c_int
    L.lb_inject_nan.argtypes = [_VP] + [ctypes.c_int32] * 5
    L.lb_save_state.restype = ctypes.c_int
    L.lb_save_state.argtypes = [_VP, _VP, ctypes.POINTER(ctypes.c_size_t)]
    L.lb_load_state.restype = ctypes.c_int
    L.lb_load_state.argtypes = [_VP, _VP, ctypes.c_size_t]
    L.lb_set_graph_steps.restype = ctypes.c_int
    L.lb_set_graph_steps.argtypes = [_VP, ctypes.c_int32]
    L.lb_set_timing.restype = ctypes.c_int
    L.lb_set_timing.argtypes = [_VP, ctypes.c_int32]
    L.lb_set_store_policy.restype = ctypes.c_int
    L.lb_set_store_policy.argtypes = [_VP, ctypes.c_int32]
    L.lb_autotune.restype = ctypes.c_int
    L.lb_autotune.argtypes = [_VP, ctypes.c_int32]
    L.lb_get_tuning.restype = ctypes.c_int
    L.lb_get_tuning.argtypes = [_VP, ctypes.POINTER(lb_tuning)]
    L.lb_set_tuning.restype = ctypes.c_int
    L.lb_set_tuning.argtypes = [_VP, ctypes.POINTER(lb_tuning)]
    L.lb_kernel_times.restype = ctypes.c_int
    L.lb_kernel_times.argtypes = [_VP, _D, ctypes.POINTER(ctypes.c_int64), _D,
                                  ctypes.POINTER(ctypes.c_int64)]
    L.lb_adjoint_workspace_bytes.restype = ctypes.c_size_t
    L.lb_adjoint_workspace_bytes.argtypes = [_VP, ctypes.c_int32, ctypes.c_int32]
    L.lb_rb_adjoint.restype = ctypes.c_int
    L.lb_rb_adjoint.argtypes = [_VP, ctypes.c_int32, ctypes.c_int32, _VP, ctypes.c_size_t, _D, _D,
                                _D, _D]
    L.lb_rb_adjoint_noalloc.restype = ctypes.c_int
    L.lb_rb_adjoint_noalloc.argtypes = [_VP, ctypes.c_int32, ctypes.c_int32, _D, _D, _D, _D]
    L.lb_node_counts.restype = ctypes.c_int
    L.lb_node_counts.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64)]
    L.lb_row_axis.restype = ctypes.c_int
    L.lb_row_axis.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.lb_destroy.restype = None
    L.lb_destroy.argtypes = [_VP]
    L.lb_last_error.restype = ctypes.c_char_p
    L.lb_last_error.argtypes = [_VP]
    _lib = L
    return L


class LBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbrb error {code}: {msg}")
        self.code = code


def _arr(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))
    return a


def _dp(a):
    return a.ctypes.data_as(_D)


# ------------------------------------------------------------------ C-ABI names

def make_params(precision="f32", rho0=1.0, u0=(0.0, 0.0, 0.0), tau_shear=1.0, tau_bulk=None,
                tau_odd=1.0, tau_even=1.0, kT=0.0, g_ext=(0.0, 0.0, 0.0), max_bodies=0,
                max_beads=0, max_wall_links=0, md_substeps=0, wca_epsilon=0.0, max_ev_sites=0,
                max_wall_sites=0):
    p = lb_params()
    p.precision = LB_PRECISION_F32 if precision in ("f32", LB_PRECISION_F32) else LB_PRECISION_F64
    p.rho0 = rho0
    p.u0[:] = list(u0)
    p.tau_shear = tau_shear
    p.tau_bulk = tau_shear if tau_bulk is None else tau_bulk
    p.tau_odd = tau_odd
    p.tau_even = tau_even
    p.kT = kT
    p.g_ext[:] = list(g_ext)
    p.max_bodies = max_bodies
    p.max_beads = max_beads
    p.max_wall_links = max_wall_links
    p.md_substeps = md_substeps
    p.wca_epsilon = wca_epsilon
    p.max_ev_sites = max_ev_sites
    p.max_wall_sites = max_wall_sites
    return p


def make_replicas(shapes_seeds):
    arr = (lb_replica * len(shapes_seeds))()
    for k, (shape, seed) in enumerate(shapes_seeds):
        arr[k].nx, arr[k].ny, arr[k].nz = (int(v) for v in shape)
        arr[k].seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return arr


def lb_workspace_bytes(params, replicas):
    return library().lb_workspace_bytes(ctypes.byref(params), replicas, len(replicas))


def lb_init(params, replicas, dev_workspace, ws_bytes, hip_stream):
    h = _VP()
    rc = library().lb_init(ctypes.byref(params), replicas, len(replicas), _VP(dev_workspace),
                           ws_bytes, _VP(hip_stream), ctypes.byref(h))
    if rc != LB_OK:
        raise LBError(rc, "lb_init failed")
    return h


def _check(ctx, rc, what):
    if rc != LB_OK:
        raise LBError(rc, f"{what}: {library().lb_last_error(ctx).decode()}")


def lb_set_boundary_mask(ctx, replica, mask):
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(-1))
    _check(ctx, library().lb_set_boundary_mask(ctx, replica,
                                               m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
           "lb_set_boundary_mask")


def lb_set_wall_velocity(ctx, replica, wall, u):
    _check(ctx, library().lb_set_wall_velocity(ctx, int(replica), int(wall), _dp(_arr(u, 3))),
           "lb_set_wall_velocity")


def rb_set_excluded_volume(ctx, replica, body_id, offsets, radius):
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.float64).reshape(-1, 3))
    _check(ctx, library().rb_set_excluded_volume(ctx, int(replica), int(body_id), _dp(off),
                                                 off.shape[0], float(radius)),
           "rb_set_excluded_volume")


def lb_add_wall_sites(ctx, replica, positions, radius):
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 3))
    _check(ctx, library().lb_add_wall_sites(ctx, int(replica), _dp(pos), pos.shape[0],
                                            float(radius)), "lb_add_wall_sites")


def rb_add_raspberry(ctx, replica, offsets, mass, inertia, pos, quat=(1, 0, 0, 0),
                     vel=(0, 0, 0), omega=(0, 0, 0), gamma=0.0, fixed=False):
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.float64).reshape(-1, 3))
    bid = ctypes.c_int32(-1)
    rc = library().rb_add_raspberry(ctx, replica, _dp(off), off.shape[0], float(mass),
                                    _dp(_arr(inertia, 3)), _dp(_arr(pos, 3)), _dp(_arr(quat, 4)),
                                    _dp(_arr(vel, 3)), _dp(_arr(omega, 3)), float(gamma),
                                    1 if fixed else 0, ctypes.byref(bid))
    _check(ctx, rc, "rb_add_raspberry")
    return bid.value


def lb_rb_step(ctx, n_steps):
    _check(ctx, library().lb_rb_step(ctx, int(n_steps)), "lb_rb_step")


def lb_observables(ctx, replica, n_bodies, dev_rho_u=None, check=True):
    tot = lb_totals()
    bodies = (rb_state * max(1, n_bodies))()
    rc = library().lb_observables(ctx, replica, ctypes.byref(tot), bodies,
                                  _VP(dev_rho_u) if dev_rho_u else None)
    if check:
        _check(ctx, rc, "lb_observables")
    return rc, tot, list(bodies)[:n_bodies]


def lb_adjoint_workspace_bytes(ctx, n_steps, checkpoint_every):
    return library().lb_adjoint_workspace_bytes(ctx, int(n_steps), int(checkpoint_every))


def lb_rb_adjoint(ctx, n_steps, checkpoint_every, dev_ws, ws_bytes, dJ_dF, n_bodies, n_beads):
    """Returns (J, dJ/dgamma [n_bodies], dJ/doffsets [n_beads, 3]) in global body/bead order."""
    w = np.ascontiguousarray(np.asarray(dJ_dF, dtype=np.float64).reshape(-1))
    if w.size != 3 * n_bodies * int(n_steps):
        raise ValueError("dJ_dF must hold n_steps * n_bodies * 3 values")
    J = ctypes.c_double(0.0)
    dg = np.zeros(max(1, n_bodies))
    do = np.zeros((max(1, n_beads), 3))
    rc = library().lb_rb_adjoint(ctx, int(n_steps), int(checkpoint_every), _VP(dev_ws), ws_bytes,
                                 _dp(w), ctypes.byref(J), _dp(dg), _dp(do))
    _check(ctx, rc, "lb_rb_adjoint")
    return J.value, dg[:n_bodies], do[:n_beads]


def lb_rb_adjoint_noalloc(ctx, n_steps, checkpoint_every, dJ_dF, n_bodies, n_beads):
    """lb_rb_adjoint on the library's own scratch array (no workspace): same results."""
    w = np.ascontiguousarray(np.asarray(dJ_dF, dtype=np.float64).reshape(-1))
    if w.size != 3 * n_bodies * int(n_steps):
        raise ValueError("dJ_dF must hold n_steps * n_bodies * 3 values")
    J = ctypes.c_double(0.0)
    dg = np.zeros(max(1, n_bodies))
    do = np.zeros((max(1, n_beads), 3))
    rc = library().lb_rb_adjoint_noalloc(ctx, int(n_steps), int(checkpoint_every), _dp(w),
                                         ctypes.byref(J), _dp(dg), _dp(do))
    _check(ctx, rc, "lb_rb_adjoint_noalloc")
    return J.value, dg[:n_bodies], do[:n_beads]


def lb_destroy(ctx):
    library().lb_destroy(ctx)


# ------------------------------------------------------------------ convenience wrapper

class Simulation:
    """One context with its workspace held as a torch uint8 tensor on ``device``."""

    def __init__(self, params, replicas, device="cuda:0", stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lbrb library has no CPU path")
        self.torch = torch
        self.device = torch.device(device)
        self.params = params
        self.replicas = replicas
        self.shapes = [(r.nx, r.ny, r.nz) for r in replicas]
        self.f32 = params.precision == LB_PRECISION_F32
        self.dtype = torch.float32 if self.f32 else torch.float64
        nbytes = lb_workspace_bytes(params, replicas)
        if nbytes == 0:
            raise LBError(LB_ERR_ARG, "invalid parameters or boxes")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = lb_init(params, replicas, aligned, nbytes, self.stream.cuda_stream)
        self.n_bodies = [0] * len(replicas)
        self.n_beads = {}
        self.body_order = []    # (replica, body id) in the order the bodies were added

    def close(self):
        if getattr(self, "ctx", None):
            lb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mask(self, replica, mask):
        lb_set_boundary_mask(self.ctx, replica, mask)

    def set_wall_velocity(self, replica, wall, u):
        lb_set_wall_velocity(self.ctx, replica, wall, u)

    def set_excluded_volume(self, replica, body_id, offsets, radius):
        rb_set_excluded_volume(self.ctx, replica, body_id, offsets, radius)

    def add_wall_sites(self, replica, positions, radius):
        lb_add_wall_sites(self.ctx, replica, positions, radius)

    def add_body(self, replica, offsets, mass, inertia, pos, quat=(1, 0, 0, 0), vel=(0, 0, 0),
                 omega=(0, 0, 0), gamma=0.0, fixed=False):
        bid = rb_add_raspberry(self.ctx, replica, offsets, mass, inertia, pos, quat, vel, omega,
                               gamma, fixed)
        self.n_bodies[replica] += 1
        self.n_beads[(replica, bid)] = int(np.asarray(offsets).reshape(-1, 3).shape[0])
        self.body_order.append((replica, bid))
        return bid

    def adjoint(self, n_steps, dJ_dF, checkpoint_every=20):
        """Advance n_steps steps and return (J, dJ/dgamma, dJ/doffsets) of
        J = sum_n sum_b dJ_dF[n, b] . F_b(n) (global body order, body-frame offsets)."""
        torch = self.torch
        nbytes = lb_adjoint_workspace_bytes(self.ctx, n_steps, checkpoint_every)
        if nbytes == 0:
            raise LBError(LB_ERR_ARG, "invalid adjoint window")
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (ws.data_ptr() + 255) // 256 * 256
        n_beads = sum(self.n_beads[k] for k in self.body_order)
        out = lb_rb_adjoint(self.ctx, n_steps, checkpoint_every, aligned, nbytes, dJ_dF,
                            len(self.body_order), n_beads)
        del ws
        return out

    def adjoint_noalloc(self, n_steps, dJ_dF, checkpoint_every=20):
        """As adjoint(), on the library's scratch array instead of a torch workspace."""
        n_beads = sum(self.n_beads[k] for k in self.body_order)
        return lb_rb_adjoint_noalloc(self.ctx, n_steps, checkpoint_every, dJ_dF,
                                     len(self.body_order), n_beads)

    def step(self, n=1):
        lb_rb_step(self.ctx, n)

    def set_graph_steps(self, k):
        _check(self.ctx, library().lb_set_graph_steps(self.ctx, int(k)), "lb_set_graph_steps")

    def set_store_policy(self, policy):
        _check(self.ctx, library().lb_set_store_policy(self.ctx, int(policy)),
               "lb_set_store_policy")

    def autotune(self, repeats=0):
        """Time the node update's launch settings on this context and keep the fastest."""
        _check(self.ctx, library().lb_autotune(self.ctx, int(repeats)), "lb_autotune")
        return self.tuned_settings()

    def set_tuning(self, tiles_per_wg=1, wg_per_cu=0, streaming=False):
        t = lb_tuning(tuned=1, tiles_per_wg=tiles_per_wg, wg_per_cu=wg_per_cu,
                      streaming=1 if streaming else 0)
        _check(self.ctx, library().lb_set_tuning(self.ctx, ctypes.byref(t)), "lb_set_tuning")

    def tuned_settings(self):
        t = lb_tuning()
        _check(self.ctx, library().lb_get_tuning(self.ctx, ctypes.byref(t)), "lb_get_tuning")
        return {"tuned": bool(t.tuned), "tiles_per_wg": t.tiles_per_wg, "wg_per_cu": t.wg_per_cu,
                "streaming_stores": bool(t.streaming), "candidates": t.candidates,
                "node_us_default": round(t.node_us_default, 3),
                "node_us_tuned": round(t.node_us_tuned, 3)}

    def set_timing(self, on):
        _check(self.ctx, library().lb_set_timing(self.ctx, 1 if on else 0), "lb_set_timing")

    def kernel_times(self):
        tn, tc = ctypes.c_double(), ctypes.c_double()
        nn, nc = ctypes.c_int64(), ctypes.c_int64()
        _check(self.ctx, library().lb_kernel_times(self.ctx, ctypes.byref(tn), ctypes.byref(nn),
                                                   ctypes.byref(tc), ctypes.byref(nc)),
               "lb_kernel_times")
        return {"node_ms": tn.value, "node_launches": nn.value, "couple_ms": tc.value,
                "couple_launches": nc.value}

    def row_axis(self, replica=0):
        """0: the replica's fluid is stored in rows along x; 2: along z (a layout choice)."""
        a = ctypes.c_int32()
        _check(self.ctx, library().lb_row_axis(self.ctx, replica, ctypes.byref(a)), "lb_row_axis")
        return a.value

    def node_counts(self, replica=0):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(self.ctx, library().lb_node_counts(self.ctx, replica, ctypes.byref(a),
                                                  ctypes.byref(b)), "lb_node_counts")
        return a.value, b.value

    def observables(self, replica=0, fields=False, check=True):
        """(totals dict, [body dicts], fields (nz,ny,nx,4) numpy or None, return code)."""
        torch = self.torch
        nx, ny, nz = self.shapes[replica]
        buf = None
        if fields:
            buf = torch.empty(4 * nx * ny * nz, dtype=self.dtype, device=self.device)
        rc, tot, bodies = lb_observables(self.ctx, replica, self.n_bodies[replica],
                                         buf.data_ptr() if buf is not None else None, check)
        t = {"mass": tot.mass, "momentum": np.array(tot.momentum[:]),
             "body_momentum": np.array(tot.body_momentum[:]), "step": tot.step,
             "finite": bool(tot.finite)}
        bs = [{"pos": np.array(b.pos[:]), "quat": np.array(b.quat[:]), "vel": np.array(b.vel[:]),
               "omega": np.array(b.omega_body[:]), "force": np.array(b.force[:]),
               "torque": np.array(b.torque[:])} for b in bodies]
        f = None
        if buf is not None:
            f = buf.double().cpu().numpy().reshape(nz, ny, nx, 4)
        return t, bs, f, rc

    def fields(self, replica=0):
        return self.observables(replica, fields=True)[2]

    def populations(self, replica=0):
        torch = self.torch
        nx, ny, nz = self.shapes[replica]
        buf = torch.empty(19 * nx * ny * nz, dtype=torch.float64, device=self.device)
        _check(self.ctx, library().lb_export_populations(self.ctx, replica, _VP(buf.data_ptr())),
               "lb_export_populations")
        return buf.cpu().numpy().reshape(19, nz, ny, nx)

    def bead_forces(self, replica, body):
        n = self.n_beads[(replica, body)]
        out = np.zeros(3 * n)
        _check(self.ctx, library().rb_bead_forces(self.ctx, replica, body, _dp(out), n),
               "rb_bead_forces")
        return out.reshape(n, 3)

    def inject_nan(self, replica, x, y, z, i):
        """Fault injection for tests: population i of fluid node (x, y, z) becomes NaN."""
        _check(self.ctx, library().lb_inject_nan(self.ctx, int(replica), int(x), int(y), int(z),
                                                 int(i)), "lb_inject_nan")

    def save_state(self):
        torch = self.torch
        n = ctypes.c_size_t(0)
        _check(self.ctx, library().lb_save_state(self.ctx, None, ctypes.byref(n)), "lb_save_state")
        buf = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        _check(self.ctx, library().lb_save_state(self.ctx, _VP(buf.data_ptr()), ctypes.byref(n)),
               "lb_save_state")
        return buf

    def load_state(self, buf):
        _check(self.ctx, library().lb_load_state(self.ctx, _VP(buf.data_ptr()), buf.numel()),
               "lb_load_state")


def wall_link_bound(mask, walls):
    """Upper bound of the moving-wall links of one replica: 18 per boundary node of a wall
    given a velocity (a boundary node faces at most 18 fluid neighbours)."""
    if mask is None or not walls:
        return 0
    return 18 * int(np.isin(np.asarray(mask), [int(w) for w in walls]).sum())


def simulation_from_workload(wl, precision=None, device="cuda:0", replicas=None,
                             max_extra_bodies=0, max_extra_beads=0):
    """Build a Simulation from a record of ``paper_1604_01829_amd.workloads.workload``."""
    reps = wl["replicas"] if replicas is None else [wl["replicas"][r] for r in replicas]
    prec = precision or wl["precision"]
    n_bodies = sum(len(r["bodies"]) for r in reps) + max_extra_bodies
    n_beads = sum(b["offsets"].shape[0] for r in reps for b in r["bodies"]) + max_extra_beads
    pp = dict(wl["params"])
    n_ev = sum(np.asarray(b["ev"][0]).reshape(-1, 3).shape[0] for r in reps for b in r["bodies"]
               if b.get("ev") is not None)
    n_sites = sum(np.asarray(r["wall_sites"][0]).reshape(-1, 3).shape[0] for r in reps
                  if r.get("wall_sites") is not None)
    params = make_params(precision=prec, max_bodies=max(1, n_bodies), max_beads=max(1, n_beads),
                         max_wall_links=sum(wall_link_bound(r["mask"], r.get("walls"))
                                            for r in reps),
                         max_ev_sites=n_ev, max_wall_sites=n_sites, **pp)
    rr = make_replicas([(r["shape"], r["seed"]) for r in reps])
    sim = Simulation(params, rr, device=device)
    for k, r in enumerate(reps):
        if r["mask"] is not None:
            sim.set_mask(k, r["mask"])
        for wall, u in (r.get("walls") or {}).items():
            sim.set_wall_velocity(k, wall, u)
        for j, b in enumerate(r["bodies"]):
            sim.add_body(k, b["offsets"], b["mass"], b["inertia"], b["pos"], b["quat"], b["vel"],
                         b["omega"], b["gamma"], b["fixed"])
            if b.get("ev") is not None:
                sim.set_excluded_volume(k, j, *b["ev"])
        if r.get("wall_sites") is not None:
            sim.add_wall_sites(k, *r["wall_sites"])
    return sim


# ------------------------------------------------------------------ autograd

def _window_objective_class():
    import torch

    class WindowObjective(torch.autograd.Function):
        """J(gamma, offsets) = sum_n sum_b a(n,b) . F_b(n) over a window of steps of a fresh
        simulation made by ``builder(gamma, offsets)``; the backward pass returns the hand
        adjoint of the library (lb_rb_adjoint), computed together with J in the forward."""

        @staticmethod
        def forward(ctx, gamma, offsets, builder, n_steps, weights, checkpoint_every):
            sim = builder(gamma.detach().cpu().numpy().astype(np.float64),
                          offsets.detach().cpu().numpy().astype(np.float64))
            try:
                J, dg, do = sim.adjoint(n_steps, weights, checkpoint_every)
            finally:
                sim.close()
            ctx.save_for_backward(torch.as_tensor(dg, dtype=gamma.dtype),
                                  torch.as_tensor(do, dtype=offsets.dtype))
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, grad):
            dg, do = ctx.saved_tensors
            return grad * dg, grad * do, None, None, None, None

    return WindowObjective


_WO = None


def window_objective(gamma, offsets, builder, n_steps, weights, checkpoint_every=20):
    """Differentiable window objective: gamma [n_bodies] and offsets [n_beads, 3] are torch
    tensors (CPU, float64); builder(gamma_np, offsets_np) returns a Simulation whose bodies
    use them.  Gradients flow through the library's reverse pass."""
    global _WO
    if _WO is None:
        _WO = _window_objective_class()
    return _WO.apply(gamma, offsets, builder, n_steps, weights, checkpoint_every)


def calibrate_gamma(builder, n_steps, weights, target, gamma0, checkpoint_every=20, tol=1e-10,
                    max_iter=20):
    """Newton iteration for the bead friction gamma (one value for every body of the
    simulation) such that the window objective J(gamma) = sum_n sum_b weights[n, b] . F_b(n)
    equals `target`; dJ/dgamma comes from the reverse pass.  builder(gamma) returns a fresh
    Simulation whose bodies use that friction.  Returns (gamma, J, iterations)."""
    g = float(gamma0)
    for it in range(1, max_iter + 1):
        sim = builder(g)
        try:
            J, dg, _ = sim.adjoint(n_steps, weights, checkpoint_every)
        finally:
            sim.close()
        slope = float(np.sum(dg))
        if not np.isfinite(J) or slope == 0.0:
            raise LBError(LB_ERR_UNSTABLE, "calibration: non-finite objective or zero slope")
        if abs(J - target) <= tol * max(1.0, abs(target)):
            return g, J, it
        g_new = g - (J - target) / slope
        # stay positive: halve towards zero instead of stepping through it
        g = g_new if g_new > 0 else 0.5 * g
    raise LBError(LB_ERR_UNSTABLE, "calibration did not converge")


def calibrate_gamma_to_radius(builder, box, target_radius, u0, rho0, eta, window, gamma0,
                              axis=0, checkpoint_every=40, tol=1e-10, max_iter=20):
    """Bead friction gamma of a fixed raspberry (every body of the builder's simulation) whose
    Hasimoto-corrected hydrodynamic radius is `target_radius`: the simulation is a periodic
    cubic box of side `box` whose fluid starts at the uniform velocity u0 along `axis` and is
    not driven; the friction over `window` (steps, 1-based, inclusive) is measured as in
    analysis.decay_friction and must equal Hasimoto's friction at the target radius.  That
    condition is linear in the per-step drags, so calibrate_gamma (Newton with the reverse
    pass's exact slope) solves it.  Returns (gamma, iterations, friction)."""
    from . import analysis as AN
    n_nodes = box ** 3
    xi = AN.hasimoto_friction(target_radius, box, eta)
    c, target = AN.decay_friction_weights(xi, u0, rho0, n_nodes, window, window[1])
    weights = np.zeros((window[1], 1, 3))
    weights[:, 0, axis] = c
    g, _, it = calibrate_gamma(builder, window[1], weights, target, gamma0,
                               checkpoint_every=checkpoint_every, tol=tol, max_iter=max_iter)
    return g, it, xi


# ------------------------------------------------------------------ Stokes-flow resistance

def stokes_flow_resistance(sim, replica, body, u_wall, n_develop, n_samples=100, every=10):
    """Colloid resistance from Stokes flow past a fixed raspberry (Sec. 2.3, eq.
    (stokesflow)): run n_develop steps for the flow to develop, then take n_samples
    measurements, `every` steps apart, of the summed bead force on the body; their mean F
    balances the resistance times the imposed boundary velocity, so
    xi_col = (F . u) / |u|^2 (the force on a fixed colloid points along the flow).
    Returns (mean force (3,), xi_col)."""
    u = np.asarray(u_wall, dtype=np.float64)
    if not float(u @ u) > 0.0:
        raise ValueError("the imposed velocity must be nonzero")
    sim.step(n_develop)
    acc = np.zeros(3)
    for _ in range(n_samples):
        sim.step(every)
        _, bodies, _, _ = sim.observables(replica)
        acc += bodies[body]["force"]
    F = acc / n_samples
    return F, float(F @ u / (u @ u))
