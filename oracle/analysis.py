"""Trajectory analysis of raspberry colloids, plain numpy, FP64.

TEST INFRASTRUCTURE ONLY: the reference the GPU analysis kernels are checked against.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may import it.  It shares
no code with the GPU library.

What it computes (Ustach & Faller, arXiv:1604.01829), from a trajectory of recorded poses
traj[frame, body] = (centre x, y, z, quaternion w, x, y, z):
  - lab-frame translational MSD (Sec. 2.4, eq. (dt_lab)) and diffusivity MSD / (6 tau);
  - lab-frame rotational MSD of the reference vector p = R(q) b_ref (Sec. 2.5, eqs. (dr_lab),
    (delta_theta)): Delta Theta = arccos(p^(t) . p^(t+tau)), diffusivity MSD / (6 tau);
  - body-frame displacements (Sec. 2.6, eqs. (labdisp)-(bodyframetrajectory); SI "Body-frame
    translational displacement"): the lab displacement over each recording interval turned into
    the body frame with the inverse rotation, then summed; diffusivity MSD / (2 tau) per axis;
  - body-frame rotations by projection (Sec. 2.7; SI "Body-frame angular displacement"): the
    body axes at t projected onto the planes normal to the axes at t - 1, angles by arctan,
    summed; diffusivity MSD / ((3/2) 2 tau) (eq. (dr_body));
  - pore-frame displacements (Sec. 2.8; SI "Pore-frame coordinate determination"): centre
    relative to the pore axis, displacement rotated by -theta, summed; MSD of the
    subtrajectories starting at the frames of each radial bin (Sec. 2.8);
  - slope fits, the Hasimoto extrapolation D(L) = D0 - c / L (eq. (hasimoto), intercept of D
    against 1/L) and the Einstein relation xi = kT / D0 (eq. (einstein_trans)).
Readings where the paper is ambiguous or misprinted (each pinned in tests/test_oracle_analysis.py):
  - the printed quaternion matrix has the sign of its (1,3) entry wrong; the matrix used is the
    rotation R(q) of the body frame into the lab frame, and lab vectors go into the body frame
    with R(q)^T;
  - the orientation that turns the displacement over (t_{n-1}, t_n] is the one at t_{n-1}, the
    start of the interval (the same for the pore angle theta);
  - the printed pore matrix multiplies by undefined x1, y1; it is read as the rotation by -theta
    with theta = atan2(y_c, x_c);
  - "MSD^2" in eq. (dr_body) and "X^p(t_n)(t)" in eq. (poreframetrajectory) are typos for MSD
    and X^p(t).
"""
import numpy as np


def quat_matrix(q):
    """Rotation matrices R(q) (body frame -> lab frame) of unit quaternions (..., 4) = (w,x,y,z)."""
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - z * w)
    R[..., 0, 2] = 2 * (x * z + y * w)
    R[..., 1, 0] = 2 * (x * y + z * w)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - x * w)
    R[..., 2, 0] = 2 * (x * z - y * w)
    R[..., 2, 1] = 2 * (y * z + x * w)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _cumulate(delta):
    """Sum of the per-interval displacements (frames-1, ...) into a trajectory starting at 0."""
    out = np.zeros((delta.shape[0] + 1,) + delta.shape[1:])
    for n in range(delta.shape[0]):
        out[n + 1] = out[n] + delta[n]
    return out


def lab_frame(traj):
    """Lab-frame centre trajectory relative to the first frame: (frames, bodies, 3)."""
    pos = np.asarray(traj, dtype=np.float64)[..., :3]
    return pos - pos[0:1]


def body_frame_translation(traj):
    """X^b(t_n) = sum_k R(q(t_{k-1}))^T (X(t_k) - X(t_{k-1})): (frames, bodies, 3)."""
    traj = np.asarray(traj, dtype=np.float64)
    pos, R = traj[..., :3], quat_matrix(traj[..., 3:7])
    d = pos[1:] - pos[:-1]
    db = np.einsum("fbji,fbj->fbi", R[:-1], d)       # R^T d
    return _cumulate(db)


def body_frame_rotation(traj):
    """Theta_{x^b}, Theta_{y^b}, Theta_{z^b} summed over the intervals: (frames, bodies, 3).

    Over (t-1, t], with body axes i, j, k (columns of R) at t-1 and i', j', k' at t: k' is
    projected onto the plane normal to i (k'_P = k' - i (k' . i)) and expressed in the frame
    of the axes at t-1 (A k'_P, rows of A = i, j, k); dTheta_x = arctan(component 2 /
    component 3); likewise dTheta_y from i'_P (components 3 / 1, plane normal to j) and
    dTheta_z from j'_P (components 1 / 2, plane normal to k)."""
    traj = np.asarray(traj, dtype=np.float64)
    R = quat_matrix(traj[..., 3:7])
    F, B = R.shape[0], R.shape[1]
    out = np.zeros((F - 1, B, 3))
    for n in range(1, F):
        for b in range(B):
            A = R[n - 1, b].T                  # rows: body axes at t-1 in lab coordinates
            ax_prev = [A[0], A[1], A[2]]
            ax_now = [R[n, b][:, 0], R[n, b][:, 1], R[n, b][:, 2]]
            kP = ax_now[2] - ax_prev[0] * np.dot(ax_now[2], ax_prev[0])
            iP = ax_now[0] - ax_prev[1] * np.dot(ax_now[0], ax_prev[1])
            jP = ax_now[1] - ax_prev[2] * np.dot(ax_now[1], ax_prev[2])
            k2, i2, j2 = A @ kP, A @ iP, A @ jP
            out[n - 1, b, 0] = np.arctan(k2[1] / k2[2])
            out[n - 1, b, 1] = np.arctan(i2[2] / i2[0])
            out[n - 1, b, 2] = np.arctan(j2[0] / j2[1])
    return _cumulate(out)


def pore_frame(traj, centre):
    """Pore-frame trajectory (frames, bodies, 3) and the radial coordinate (frames, bodies):
    x^c = x - centre_x, y^c = y - centre_y, theta = atan2(y^c, x^c) at the start of each
    interval; the interval's displacement rotated by -theta (x^p radial, y^p tangential,
    z^p axial), then summed."""
    traj = np.asarray(traj, dtype=np.float64)
    xc = traj[..., 0] - centre[0]
    yc = traj[..., 1] - centre[1]
    th = np.arctan2(yc, xc)
    d = traj[1:, :, :3] - traj[:-1, :, :3]
    c, s = np.cos(th[:-1]), np.sin(th[:-1])
    dp = np.stack([c * d[..., 0] + s * d[..., 1], -s * d[..., 0] + c * d[..., 1], d[..., 2]],
                  axis=-1)
    return _cumulate(dp), np.hypot(xc, yc)


def msd(series, n_lags):
    """Mean over time origins of the squared displacement, per lag 1..n_lags and component:
    series (frames, bodies, comps) -> (bodies, n_lags, comps)."""
    s = np.asarray(series, dtype=np.float64)
    F, B, C = s.shape
    out = np.zeros((B, n_lags, C))
    for tau in range(1, n_lags + 1):
        d = s[tau:] - s[:F - tau]
        out[:, tau - 1, :] = (d * d).sum(axis=0) / (F - tau)
    return out


def rotation_msd(traj, ref, n_lags):
    """Mean over time origins of Delta Theta^2, Delta Theta = arccos(p^(t) . p^(t+tau)) with
    p = R(q) ref_b: (bodies, n_lags).  ref: (bodies, 3) body-frame reference vectors."""
    traj = np.asarray(traj, dtype=np.float64)
    R = quat_matrix(traj[..., 3:7])
    p = np.einsum("fbij,bj->fbi", R, np.asarray(ref, dtype=np.float64))
    p /= np.linalg.norm(p, axis=-1, keepdims=True)
    F, B = p.shape[:2]
    out = np.zeros((B, n_lags))
    for tau in range(1, n_lags + 1):
        c = np.clip((p[tau:] * p[:F - tau]).sum(axis=-1), -1.0, 1.0)
        out[:, tau - 1] = (np.arccos(c) ** 2).sum(axis=0) / (F - tau)
    return out


def binned_msd(series, radial, edges, n_lags):
    """Subtrajectory MSDs per radial bin (Sec. 2.8): every origin frame t of every body falls in
    bin k when edges[k] <= r(t) < edges[k+1]; for each bin and lag the sums of the squared
    displacements from those origins and their count.  Returns (sums (bins, lags, comps),
    counts (bins, lags))."""
    s = np.asarray(series, dtype=np.float64)
    r = np.asarray(radial, dtype=np.float64)
    F, B, C = s.shape
    nb = len(edges) - 1
    sums = np.zeros((nb, n_lags, C))
    counts = np.zeros((nb, n_lags))
    for tau in range(1, n_lags + 1):
        d2 = (s[tau:] - s[:F - tau]) ** 2
        r0 = r[:F - tau]
        for k in range(nb):
            m = (r0 >= edges[k]) & (r0 < edges[k + 1])
            sums[k, tau - 1] = d2[m].sum(axis=0)
            counts[k, tau - 1] = m.sum()
    return sums, counts


def slope(lag_times, values):
    """Least-squares slope of values against lag time (a line with intercept)."""
    t = np.asarray(lag_times, dtype=np.float64)
    v = np.asarray(values, dtype=np.float64)
    A = np.stack([t, np.ones_like(t)], axis=1)
    return np.linalg.lstsq(A, v, rcond=None)[0][0]


def diffusivity(lag_times, msd_values, denominator):
    """Slope of the MSD divided by the formula's denominator factor: 6 for eqs. (dt_lab) and
    (dr_lab), 2 for eq. (dt_body), 3 = (3/2) 2 for eq. (dr_body), 2 per pore-frame axis."""
    return slope(lag_times, msd_values) / denominator


def hasimoto_d0(box_lengths, diffusivities):
    """Intercept of D against 1/L (eq. (hasimoto)): (D0, c) with D(L) = D0 - c / L."""
    x = 1.0 / np.asarray(box_lengths, dtype=np.float64)
    A = np.stack([np.ones_like(x), -x], axis=1)
    d0, c = np.linalg.lstsq(A, np.asarray(diffusivities, dtype=np.float64), rcond=None)[0]
    return d0, c


def einstein_resistance(kT, d0):
    """xi = kT / D0 (eq. (einstein_trans))."""
    return kT / d0
