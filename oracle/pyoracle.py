"""ctypes wrapper of the FP64 CPU oracle (``oracle/liborc.so``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg of
the benchmark.  Argument marshalling only; all arithmetic is in the C sources of ``oracle/``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("rho0", ctypes.c_double),
        ("u0", ctypes.c_double * 3),
        ("tau_shear", ctypes.c_double),
        ("tau_bulk", ctypes.c_double),
        ("tau_odd", ctypes.c_double),
        ("tau_even", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("g_ext", ctypes.c_double * 3),
        ("seed", ctypes.c_uint64),
        ("md_substeps", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("wca_epsilon", ctypes.c_double),
    ]


class RelaxParams(ctypes.Structure):
    _fields_ = [("k_surface", ctypes.c_double), ("sigma", ctypes.c_double),
                ("epsilon", ctypes.c_double), ("damping", ctypes.c_double),
                ("dt", ctypes.c_double), ("mass", ctypes.c_double)]


def relax_params(k_surface=10.0, sigma=1.4, epsilon=0.1, damping=1000.0, dt=0.001, mass=1.0):
    return RelaxParams(k_surface, sigma, epsilon, damping, dt, mass)


def closest_point(axes, x):
    """(rs, t): closest point on the ellipsoid with semi-axes `axes` to the point x."""
    rs = np.zeros(3)
    t = lib().orc_closest_point(_dp(_vec(axes, 3)), _dp(_vec(x, 3)), _dp(rs))
    return rs, t


def relax_shell(axes, pos, vel, params, n_steps):
    """Advance a bead shell n_steps (copies in, returns (pos, vel))."""
    p = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3)).copy()
    v = np.ascontiguousarray(np.asarray(vel, dtype=np.float64).reshape(-1, 3)).copy()
    if lib().orc_relax_shell(_dp(_vec(axes, 3)), p.shape[0], _dp(p), _dp(v),
                             ctypes.byref(params), int(n_steps)) != 0:
        raise RuntimeError("orc_relax_shell failed")
    return p, v


def shell_energy(axes, pos, params):
    p = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
    return lib().orc_shell_energy(_dp(_vec(axes, 3)), p.shape[0], _dp(p), ctypes.byref(params))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build
            build.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_velocity.restype = ctypes.c_int
        L.orc_velocity.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_weight.restype = ctypes.c_double
        L.orc_weight.argtypes = [ctypes.c_int]
        L.orc_opposite.restype = ctypes.c_int
        L.orc_opposite.argtypes = [ctypes.c_int]
        L.orc_basis.restype = ctypes.c_double
        L.orc_basis.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_basis_norm.restype = ctypes.c_double
        L.orc_basis_norm.argtypes = [ctypes.c_int]
        L.orc_philox4x32_10.restype = None
        L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.orc_uniform16.restype = ctypes.c_double
        L.orc_uniform16.argtypes = [ctypes.c_uint32]
        L.orc_collide_node.restype = None
        L.orc_collide_node.argtypes = [ctypes.POINTER(OrcParams), _D, _D, _D, _D]
        L.orc_equilibrium.restype = None
        L.orc_equilibrium.argtypes = [ctypes.c_double, _D, _D]
        L.orc_trilinear.restype = None
        L.orc_trilinear.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D,
                                    ctypes.POINTER(ctypes.c_int64), _D]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(OrcParams)]
        L.orc_destroy.restype = None
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_set_mask.restype = ctypes.c_int
        L.orc_set_mask.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8)]
        L.orc_set_wall_velocity.restype = ctypes.c_int
        L.orc_set_wall_velocity.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.orc_add_body.restype = ctypes.c_int
        L.orc_add_body.argtypes = [ctypes.c_void_p, _D, ctypes.c_int, ctypes.c_double, _D, _D,
                                   _D, _D, _D, ctypes.c_double, ctypes.c_int]
        L.orc_set_excluded_volume.restype = ctypes.c_int
        L.orc_set_excluded_volume.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, ctypes.c_int,
                                              ctypes.c_double]
        L.orc_add_wall_sites.restype = ctypes.c_int
        L.orc_add_wall_sites.argtypes = [ctypes.c_void_p, _D, ctypes.c_int, ctypes.c_double]
        L.orc_wca_forces.restype = ctypes.c_int
        L.orc_wca_forces.argtypes = [ctypes.c_void_p, _D]
        L.orc_wca_energy.restype = ctypes.c_double
        L.orc_wca_energy.argtypes = [ctypes.c_void_p]
        L.orc_step.restype = ctypes.c_int
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_step_count.restype = ctypes.c_int64
        L.orc_step_count.argtypes = [ctypes.c_void_p]
        L.orc_fields.restype = None
        L.orc_fields.argtypes = [ctypes.c_void_p, _D]
        L.orc_populations.restype = None
        L.orc_populations.argtypes = [ctypes.c_void_p, _D]
        L.orc_set_populations.restype = None
        L.orc_set_populations.argtypes = [ctypes.c_void_p, _D]
        L.orc_totals.restype = None
        L.orc_totals.argtypes = [ctypes.c_void_p, _D]
        L.orc_body_state.restype = ctypes.c_int
        L.orc_body_state.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.orc_bead_forces.restype = ctypes.c_int
        L.orc_bead_forces.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_closest_point.restype = ctypes.c_double
        L.orc_closest_point.argtypes = [_D, _D, _D]
        L.orc_relax_shell.restype = ctypes.c_int
        L.orc_relax_shell.argtypes = [_D, ctypes.c_int, _D, _D, ctypes.POINTER(RelaxParams),
                                      ctypes.c_int]
        L.orc_shell_energy.restype = ctypes.c_double
        L.orc_shell_energy.argtypes = [_D, ctypes.c_int, _D, ctypes.POINTER(RelaxParams)]
        L.orc_collide_vjp.restype = None
        L.orc_collide_vjp.argtypes = [ctypes.POINTER(OrcParams), _D, _D, _D, _D, _D]
        L.orc_adjoint.restype = ctypes.c_int
        L.orc_adjoint.argtypes = [ctypes.c_void_p, ctypes.POINTER(OrcParams), ctypes.c_int,
                                  ctypes.c_int, _D, _D, _D, _D]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _vec(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))
    return a


def make_params(rho0=1.0, u0=(0.0, 0.0, 0.0), tau_shear=1.0, tau_bulk=None, tau_odd=1.0,
                tau_even=1.0, kT=0.0, g_ext=(0.0, 0.0, 0.0), seed=0, md_substeps=0,
                wca_epsilon=0.0):
    p = OrcParams()
    p.rho0 = rho0
    p.u0[:] = list(u0)
    p.tau_shear = tau_shear
    p.tau_bulk = tau_shear if tau_bulk is None else tau_bulk
    p.tau_odd = tau_odd
    p.tau_even = tau_even
    p.kT = kT
    p.g_ext[:] = list(g_ext)
    p.seed = seed
    p.md_substeps = md_substeps
    p.wca_epsilon = wca_epsilon
    return p


# ---------------------------------------------------------------- tables and pure functions

def velocities():
    L = lib()
    return np.array([[L.orc_velocity(i, a) for a in range(3)] for i in range(19)], dtype=np.int64)


def weights():
    L = lib()
    return np.array([L.orc_weight(i) for i in range(19)])


def opposite():
    L = lib()
    return np.array([L.orc_opposite(i) for i in range(19)], dtype=np.int64)


def basis():
    L = lib()
    return np.array([[L.orc_basis(k, i) for i in range(19)] for k in range(19)])


def basis_norms():
    L = lib()
    return np.array([L.orc_basis_norm(k) for k in range(19)])


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform16(h):
    return lib().orc_uniform16(int(h))


def equilibrium(rho, u):
    out = np.zeros(19)
    lib().orc_equilibrium(float(rho), _dp(_vec(u, 3)), _dp(out))
    return out


def collide_node(params, f_in, F, unoise=None):
    out = np.zeros(19)
    fin = _vec(f_in, 19)
    Fv = _vec(F, 3)
    un = None if unoise is None else _vec(unoise, 19)
    lib().orc_collide_node(ctypes.byref(params), _dp(fin), _dp(Fv),
                           None if un is None else _dp(un), _dp(out))
    return out


def collide_vjp(params, f_in, F, lam_out):
    lam_in = np.zeros(19)
    lam_F = np.zeros(3)
    lib().orc_collide_vjp(ctypes.byref(params), _dp(_vec(f_in, 19)), _dp(_vec(F, 3)),
                          _dp(_vec(lam_out, 19)), _dp(lam_in), _dp(lam_F))
    return lam_in, lam_F


def trilinear(shape, r):
    idx = np.zeros(8, dtype=np.int64)
    w = np.zeros(8)
    nx, ny, nz = shape
    lib().orc_trilinear(nx, ny, nz, _dp(_vec(r, 3)), idx.ctypes.data_as(
        ctypes.POINTER(ctypes.c_int64)), _dp(w))
    return idx, w


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------- a box

class OracleSim:
    """One box of the oracle: same call sequence as the GPU library's C-ABI."""

    def __init__(self, shape, params):
        self.shape = tuple(int(v) for v in shape)
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        self.params = params
        self._h = lib().orc_create(self.shape[0], self.shape[1], self.shape[2],
                                   ctypes.byref(params))
        if not self._h:
            raise RuntimeError("orc_create failed")
        self.n_bodies = 0
        self.beads_per_body = []

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def set_mask(self, mask):
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(-1))
        assert m.size == self.n
        rc = lib().orc_set_mask(self._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        if rc != 0:
            raise RuntimeError("orc_set_mask failed")

    def set_wall_velocity(self, wall, u):
        rc = lib().orc_set_wall_velocity(self._h, int(wall), _dp(_vec(u, 3)))
        if rc != 0:
            raise RuntimeError("orc_set_wall_velocity failed")

    def add_body(self, offsets, mass, inertia, pos, quat=(1, 0, 0, 0), vel=(0, 0, 0),
                 omega=(0, 0, 0), gamma=0.0, fixed=False):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.float64).reshape(-1, 3))
        bid = lib().orc_add_body(self._h, _dp(off), off.shape[0], float(mass),
                                 _dp(_vec(inertia, 3)), _dp(_vec(pos, 3)), _dp(_vec(quat, 4)),
                                 _dp(_vec(vel, 3)), _dp(_vec(omega, 3)), float(gamma),
                                 1 if fixed else 0)
        if bid < 0:
            raise RuntimeError("orc_add_body failed")
        self.n_bodies += 1
        self.beads_per_body.append(off.shape[0])
        return bid

    def set_excluded_volume(self, body, offsets, radius):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.float64).reshape(-1, 3))
        if lib().orc_set_excluded_volume(self._h, int(body), _dp(off), off.shape[0],
                                         float(radius)) != 0:
            raise RuntimeError("orc_set_excluded_volume failed")

    def add_wall_sites(self, positions, radius):
        pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 3))
        if lib().orc_add_wall_sites(self._h, _dp(pos), pos.shape[0], float(radius)) != 0:
            raise RuntimeError("orc_add_wall_sites failed")

    def wca_forces(self):
        """(n_bodies, 6): WCA force and torque (lab, about the centre) at the current poses."""
        out = np.zeros(6 * max(self.n_bodies, 1))
        lib().orc_wca_forces(self._h, _dp(out))
        return out[:6 * self.n_bodies].reshape(-1, 6)

    def wca_energy(self):
        return lib().orc_wca_energy(self._h)

    def step(self, n=1):
        if lib().orc_step(self._h, int(n)) != 0:
            raise RuntimeError("orc_step failed")

    @property
    def step_count(self):
        return lib().orc_step_count(self._h)

    def fields(self):
        """(nz, ny, nx, 4) array of rho, ux, uy, uz; zeros on boundary nodes."""
        out = np.zeros(self.n * 4)
        lib().orc_fields(self._h, _dp(out))
        return out.reshape(self.shape[2], self.shape[1], self.shape[0], 4)

    def populations(self):
        """(19, nz, ny, nx) pre-collision populations."""
        out = np.zeros(19 * self.n)
        lib().orc_populations(self._h, _dp(out))
        return out.reshape(19, self.shape[2], self.shape[1], self.shape[0])

    def set_populations(self, f):
        a = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
        assert a.size == 19 * self.n
        lib().orc_set_populations(self._h, _dp(a))

    def totals(self):
        out = np.zeros(8)
        lib().orc_totals(self._h, _dp(out))
        return {"mass": out[0], "momentum": out[1:4].copy(), "body_momentum": out[4:7].copy(),
                "finite": bool(out[7])}

    def body_state(self, b):
        out = np.zeros(19)
        if lib().orc_body_state(self._h, int(b), _dp(out)) != 0:
            raise IndexError(b)
        return {"pos": out[0:3].copy(), "quat": out[3:7].copy(), "vel": out[7:10].copy(),
                "omega": out[10:13].copy(), "force": out[13:16].copy(),
                "torque": out[16:19].copy()}

    def adjoint(self, n_steps, dJ_dF):
        """Advance n_steps and return (J, dJ/dgamma per body, dJ/doffsets per bead (n, 3))."""
        a = np.ascontiguousarray(np.asarray(dJ_dF, dtype=np.float64).reshape(-1))
        assert a.size == n_steps * self.n_bodies * 3
        J = np.zeros(1)
        dg = np.zeros(self.n_bodies)
        do = np.zeros(3 * sum(self.beads_per_body))
        rc = lib().orc_adjoint(self._h, ctypes.byref(self.params), int(n_steps), self.n_bodies,
                               _dp(a), _dp(J), _dp(dg), _dp(do))
        if rc != 0:
            raise RuntimeError("orc_adjoint failed")
        return float(J[0]), dg, do.reshape(-1, 3)

    def bead_forces(self, b):
        out = np.zeros(self.beads_per_body[b] * 3)
        if lib().orc_bead_forces(self._h, int(b), _dp(out)) != 0:
            raise IndexError(b)
        return out.reshape(-1, 3)
