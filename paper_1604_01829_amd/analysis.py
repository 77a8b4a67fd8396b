"""Trajectory analysis of raspberry colloids on the GPU (Sec. 2.4-2.8 of arXiv:1604.01829).

Recording: ``record(sim, n_frames, every)`` steps a Simulation and stores every body's pose
after each `every` steps into a device tensor traj[frame, body, 7] (centre, quaternion w,x,y,z)
through ``rb_record_poses``.  Analysis: thin wrappers over the library's ``lb_traj_*``
kernels (argument marshalling only) that return device tensors:

  lab_frame(traj)        -> [body, frame, 3]   centre minus its first position
  body_frame(traj)       -> [body, frame, 6]   body-frame displacement and rotation angles
  pore_frame(traj, c)    -> ([body, frame, 3], radial [body, frame])
  msd(series, n_lags)    -> [body, lag, k]     mean over origins, lags 1..n_lags
  rotation_msd(traj, ref, n_lags) -> [body, lag]   reference-vector angle MSD
  binned_msd(series, radial, edges, n_lags) -> (sums [bin, lag, k], counts [bin, lag])

and the paper's formulas on the resulting curves (host, a handful of numbers):
``diffusivity`` (slope of the MSD over the chosen lags divided by 6 for eqs. (dt_lab),
(dr_lab), 2 for (dt_body) and per pore-frame axis, 3 = (3/2) 2 for (dr_body)),
``hasimoto_intercept`` (D0 from D(L) = D0 - c / L, eq. (hasimoto)) and ``einstein`` (xi = kT/D0,
eq. (einstein_trans)).
"""
import numpy as np

from . import lbrb


def _stream(t):
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


def _chk(rc, what):
    if rc != lbrb.LB_OK:
        raise lbrb.LBError(rc, what)


def record(sim, n_frames, every, traj=None):
    """Record n_frames poses of every body, `every` steps apart (the first after `every`
    steps), into a device tensor [n_frames, n_bodies, 7] (float64)."""
    torch = sim.torch
    nb = len(sim.body_order)
    if traj is None:
        traj = torch.empty((n_frames, nb, 7), dtype=torch.float64, device=sim.device)
    L = lbrb.library()
    for f in range(n_frames):
        sim.step(every)
        _chk(L.rb_record_poses(sim.ctx, lbrb._VP(traj[f].data_ptr())), "rb_record_poses")
    return traj


def _shape(traj):
    assert traj.dtype.itemsize == 8 and traj.is_contiguous() and traj.shape[-1] == 7
    return int(traj.shape[0]), int(traj.shape[1])


def lab_frame(traj):
    import torch
    F, B = _shape(traj)
    out = torch.empty((B, F, 3), dtype=torch.float64, device=traj.device)
    _chk(lbrb.library().lb_traj_lab_frame(traj.data_ptr(), F, B, out.data_ptr(),
                                          _stream(traj)), "lb_traj_lab_frame")
    return out


def body_frame(traj):
    import torch
    F, B = _shape(traj)
    out = torch.empty((B, F, 6), dtype=torch.float64, device=traj.device)
    _chk(lbrb.library().lb_traj_body_frame(traj.data_ptr(), F, B, out.data_ptr(),
                                           _stream(traj)), "lb_traj_body_frame")
    return out


def pore_frame(traj, centre):
    import torch
    F, B = _shape(traj)
    out = torch.empty((B, F, 3), dtype=torch.float64, device=traj.device)
    rad = torch.empty((B, F), dtype=torch.float64, device=traj.device)
    _chk(lbrb.library().lb_traj_pore_frame(traj.data_ptr(), F, B, float(centre[0]),
                                           float(centre[1]), out.data_ptr(), rad.data_ptr(),
                                           _stream(traj)), "lb_traj_pore_frame")
    return out, rad


def msd(series, n_lags):
    import torch
    B, F, k = (int(v) for v in series.shape)
    assert series.is_contiguous() and series.dtype == torch.float64
    out = torch.empty((B, n_lags, k), dtype=torch.float64, device=series.device)
    _chk(lbrb.library().lb_traj_msd(series.data_ptr(), F, B, k, int(n_lags), out.data_ptr(),
                                    _stream(series)), "lb_traj_msd")
    return out


def rotation_msd(traj, ref_body, n_lags):
    import torch
    F, B = _shape(traj)
    ref = torch.as_tensor(np.asarray(ref_body, dtype=np.float64).reshape(B, 3), device=traj.device)
    out = torch.empty((B, n_lags), dtype=torch.float64, device=traj.device)
    _chk(lbrb.library().lb_traj_rotation_msd(traj.data_ptr(), F, B, ref.data_ptr(), int(n_lags),
                                             out.data_ptr(), _stream(traj)),
         "lb_traj_rotation_msd")
    return out


def binned_msd(series, radial, edges, n_lags):
    import torch
    B, F, k = (int(v) for v in series.shape)
    e = torch.as_tensor(np.asarray(edges, dtype=np.float64), device=series.device)
    nb = int(e.numel()) - 1
    sums = torch.empty((nb, n_lags, k), dtype=torch.float64, device=series.device)
    counts = torch.empty((nb, n_lags), dtype=torch.float64, device=series.device)
    _chk(lbrb.library().lb_traj_binned_msd(series.data_ptr(), radial.data_ptr(), F, B, k,
                                           e.data_ptr(), nb, int(n_lags), sums.data_ptr(),
                                           counts.data_ptr(), _stream(series)),
         "lb_traj_binned_msd")
    return sums, counts


# ------------------------------------------------------------------ fits (host)

def diffusivity(lag_times, msd_curve, denominator):
    """Least-squares slope (line with intercept) of the MSD over the given lag times, divided
    by the formula's denominator."""
    t = np.asarray(lag_times, dtype=np.float64)
    m = np.asarray(msd_curve, dtype=np.float64)
    tc, mc = t - t.mean(), m - m.mean()
    return float((tc * mc).sum() / (tc * tc).sum()) / denominator


def hasimoto_intercept(box_lengths, diffusivities):
    """(D0, c) of the straight line D = D0 - c x through (x = 1/L, D)."""
    x = 1.0 / np.asarray(box_lengths, dtype=np.float64)
    d = np.asarray(diffusivities, dtype=np.float64)
    xc, dc = x - x.mean(), d - d.mean()
    slope = float((xc * dc).sum() / (xc * xc).sum())
    return float(d.mean() - slope * x.mean()), -slope


def hasimoto_radius(xi, L, eta):
    """Hydrodynamic radius of a sphere whose friction in a periodic cubic box of side L is xi
    (Hasimoto's series for a periodic array, eq. (hasimoto), in its resistance form:
    6 pi eta R / xi = 1 - 2.837 x + 4.19 x^3 - 27.4 x^6, x = R / L), by bisection."""
    lo, hi = 1e-6, L / 3.0
    for _ in range(200):
        R = 0.5 * (lo + hi)
        x = R / L
        if 6 * np.pi * eta * R / xi > 1 - 2.837 * x + 4.19 * x ** 3 - 27.4 * x ** 6:
            hi = R
        else:
            lo = R
    return 0.5 * (lo + hi)


def hasimoto_friction(R, L, eta):
    """The friction in a periodic box of side L of a sphere of hydrodynamic radius R."""
    x = R / L
    return 6 * np.pi * eta * R / (1 - 2.837 * x + 4.19 * x ** 3 - 27.4 * x ** 6)


def decay_friction(drag, u0, rho0, n_nodes, window):
    """Friction of a fixed body in a periodic box whose fluid started at the uniform velocity
    u0 (along the drag axis) and is not driven: the fluid loses the body's drag F(m) every step,
    so its mean velocity after step n is U(n) = u0 - sum_{m<=n} F(m) / (rho0 n_nodes), and over a
    window of steps (1-based, inclusive) the friction is sum F / sum U.  drag[m-1] = F(m)."""
    F = np.asarray(drag, dtype=np.float64)
    U = u0 - np.cumsum(F) / (rho0 * n_nodes)
    a, b = window
    return float(F[a - 1:b].sum() / U[a - 1:b].sum())


def decay_friction_weights(xi, u0, rho0, n_nodes, window, n_steps):
    """Weights c[m-1] and target t of the linear condition sum_m c_m F(m) = t that holds when
    decay_friction(...) equals xi: sum_W F - xi sum_W U = 0 with U as in decay_friction."""
    a, b = window
    c = np.zeros(n_steps)
    c[a - 1:b] = 1.0
    for m in range(1, b + 1):
        c[m - 1] += xi / (rho0 * n_nodes) * (b - max(a, m) + 1)
    return c, xi * (b - a + 1) * u0


def einstein(kT, d0):
    return kT / d0
