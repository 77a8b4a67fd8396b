// lbrb_adjoint_device.h -- the bead pass of the reverse step as a device function, shared by
// its own kernel and by the launch that also runs the next reverse step's coupling.
#pragma once

#include "lbrb_device.h"

namespace lbrb {

// Lanes per workgroup of the bead pass: one wave, so that its atomics issue from every XCD.
constexpr int kAdjBeadBlock = 64;

// The adjoint of an MD step's body force F and lab torque T (6 values) from the adjoint ab of
// the body's state after the step (19 words: position, quaternion, velocity, body-frame
// angular velocity, force, body-frame torque) and the objective's weight a: the second half
// kick V += dt F/2M, w += dt (tau - w x I w)/2I with tau = Q^T T (rot: Q of the step's pose,
// row-major); a fixed body takes the weight alone.
__device__ __forceinline__ void force_torque_adjoint(const Body& B, const double* rot,
                                                     const double* ab, const double* a,
                                                     double out[6])
{
    if (B.fixed) {
        for (int k = 0; k < 3; ++k) { out[k] = a[k]; out[3 + k] = 0.0; }
        return;
    }
    const double hh = 0.5 * B.dt;
    double tb[3];
    for (int k = 0; k < 3; ++k) {
        out[k] = ab[13 + k] + a[k] + hh * ab[7 + k] / B.mass;
        tb[k] = ab[16 + k] + hh * ab[10 + k] / B.inertia[k];
    }
    for (int r = 0; r < 3; ++r)
        out[3 + r] = rot[3 * r] * tb[0] + rot[3 * r + 1] * tb[1] + rot[3 * r + 2] * tb[2];
}

// Bead pass for lane `tid` (8 lanes per bead, one per stencil corner): the transpose of
// spreading, friction and interpolation, and of the velocity sampling; with FREE also of the
// torque sum and of the bead kinematics (the adjoint of the body force and torque comes from
// the body's state adjoint A.body_adj).  Lanes past the last bead return at once (the 8 lanes of a bead leave
// together).
template <typename Real, bool FREE = false>
__device__ __forceinline__ void adj_bead_lanes(const AdjArgs<Real>& A, int tid)
{
    const StepArgs<Real>& a = A.a;
    const int bead = tid >> 3, corner = tid & 7;
    if (bead >= A.n_beads) return;   // the 8 lanes of a bead leave together
    // the bead record: friction and replica geometry, and for fixed bodies also the lab
    // position (the only pose); with FREE the position, arm and velocity come from the step's
    // stored pose, as the body finishing wrote them into the records of the step (the records
    // may already hold the previous step's, for a coupling recompute sharing this launch)
    const BeadRec X = load_record(A.recs + bead);
    const int32_t body = A.beads[bead].body;
    double r[3], arm[3], vel[3];
    if constexpr (FREE) {
        const Body& Bd = A.snap[body];
        const Pose& P = Bd.pose[A.pose_par];
        const double* off = A.beads[bead].off;
        for (int ax = 0; ax < 3; ++ax) {
            arm[ax] = P.rot[3 * ax] * off[0] + P.rot[3 * ax + 1] * off[1] + P.rot[3 * ax + 2] * off[2];
            r[ax] = P.pos[ax] + arm[ax];
        }
        if (Bd.fixed) {
            vel[0] = vel[1] = vel[2] = 0.0;
        } else {
            const double* wl = P.omega_lab;
            vel[0] = P.vel[0] + (wl[1] * arm[2] - wl[2] * arm[1]);
            vel[1] = P.vel[1] + (wl[2] * arm[0] - wl[0] * arm[2]);
            vel[2] = P.vel[2] + (wl[0] * arm[1] - wl[1] * arm[0]);
        }
    } else {
        for (int ax = 0; ax < 3; ++ax) { r[ax] = X.r[ax]; arm[ax] = X.dv[ax]; vel[ax] = X.v[ax]; }
    }
    double fr[3];
    int i0[3];
    i0[0] = wrap_floor(r[0] - 0.5, X.nx, fr[0]);
    i0[1] = wrap_floor(r[1] - 0.5, X.ny, fr[1]);
    i0[2] = wrap_floor(r[2] - 0.5, X.nz, fr[2]);
    const int o[3] = {corner & 1, (corner >> 1) & 1, corner >> 2};
    const int px = i0[0] + o[0] == X.nx ? 0 : i0[0] + o[0];
    const int py = i0[1] + o[1] == X.ny ? 0 : i0[1] + o[1];
    const int pz = i0[2] + o[2] == X.nz ? 0 : i0[2] + o[2];
    double t[3];
    for (int ax = 0; ax < 3; ++ax) t[ax] = o[ax] ? fr[ax] : 1.0 - fr[ax];
    const double w = t[0] * t[1] * t[2];
    double gw[3];   // gradient of the weight with respect to the bead position
    gw[0] = (o[0] ? 1.0 : -1.0) * t[1] * t[2];
    gw[1] = (o[1] ? 1.0 : -1.0) * t[0] * t[2];
    gw[2] = (o[2] ? 1.0 : -1.0) * t[0] * t[1];

    // the record holds the box's sides; a swapped replica is stored with axes x and z
    // exchanged (bit 8 of masked), so its node and sides in storage coordinates are these
    const int masked = X.masked & 0xFF;
    const bool swap = (X.masked >> 8) != 0;
    const int sx = swap ? pz : px, sz = swap ? px : pz;
    ReplicaDesc R{};
    R.nx = swap ? X.nz : X.nx; R.ny = X.ny; R.nz = swap ? X.nx : X.nz; R.masked = masked;
    R.base = X.base; R.row_base = X.row_base; R.swap = swap ? 1 : 0;
    int64_t local;
    Real d[Q];
    if (masked) {
        const RowDesc self = a.rowinfo[X.row_base + py + X.ny * sz];
        const int off = sx - self.xlo;
        local = (unsigned)off < (unsigned)self.len ? self.start + off : -1;
        // a hole is a boundary node: no velocity sampled, no force spread
        if (masked == 2 && local >= 0 && a.hole[X.base + local] != 0) local = -1;
        if (local >= 0) pull<Real, true, 1>(a.src, a.N, R, a.rowinfo, sx, py, sz, local, self, d);
    } else {
        local = px + (int64_t)X.nx * (py + (int64_t)X.ny * pz);
        const RowDesc self{0, 0, X.nx, 0};
        pull<Real, false, 1>(a.src, a.N, R, a.rowinfo, px, py, pz, local, self, d);
    }
    const int64_t g = X.base + local;
    double uc[3] = {0.0, 0.0, 0.0}, lFc[3] = {0.0, 0.0, 0.0}, ir = 0.0;
    if (local >= 0) {
        Real drho, j[3];
        density_momentum<Real>(d, drho, j);
        ir = 1.0 / ((double)a.cp.rho0 + (double)drho);
        for (int ax = 0; ax < 3; ++ax) {
            uc[ax] = ((double)j[ax] + 0.5 * (double)a.gext[ax]) * ir;
            lFc[ax] = (double)A.lamF[(int64_t)ax * a.N + g];
        }
    }
    // uk = sum_c w u(x_c), sF = sum_c w lamF(x_c) over the 8 corner lanes
    double s6[6] = {w * uc[0], w * uc[1], w * uc[2], w * lFc[0], w * lFc[1], w * lFc[2]};
#pragma unroll
    for (int m = 1; m < 8; m <<= 1)
        for (int k = 0; k < 6; ++k) s6[k] += __shfl_xor(s6[k], m, 8);
    const double* Fk = A.bead_force + 3 * (int64_t)bead;
    const double* an = A.weights + 3 * (int64_t)body;
    double lFk[3], luk[3], bj[6];
    if constexpr (FREE) {
        // the body force F = sum F_k and the lab torque T = sum d_k x F_k
        const Body& Bd = A.snap[body];
        force_torque_adjoint(Bd, Bd.pose[A.pose_par].rot, A.body_adj + kBodyAdjWords * (int64_t)body,
                             an, bj);
        const double* dv = arm;
        const double h = A.spread_h;
        lFk[0] = bj[0] + (bj[4] * dv[2] - bj[5] * dv[1]) - h * s6[3];
        lFk[1] = bj[1] + (bj[5] * dv[0] - bj[3] * dv[2]) - h * s6[4];
        lFk[2] = bj[2] + (bj[3] * dv[1] - bj[4] * dv[0]) - h * s6[5];
    } else {
        for (int ax = 0; ax < 3; ++ax) lFk[ax] = an[ax] - s6[3 + ax];
    }
    for (int ax = 0; ax < 3; ++ax) luk[ax] = X.gamma * lFk[ax];
    // position derivative through the interpolation and the spreading weights of this corner
    double dr[3] = {0.0, 0.0, 0.0};
    if (local >= 0) {
        double su = 0.0, sF = 0.0;
        for (int ax = 0; ax < 3; ++ax) { su += uc[ax] * luk[ax]; sF += Fk[ax] * lFc[ax]; }
        if constexpr (FREE) sF *= A.spread_h;
        for (int ax = 0; ax < 3; ++ax) dr[ax] = gw[ax] * (su - sF);
        // this corner's share of the sampled velocity's adjoint, through u to the populations
        const double l0 = w * luk[0] * ir, l1 = w * luk[1] * ir, l2 = w * luk[2] * ir;
        const double cu = uc[0] * l0 + uc[1] * l1 + uc[2] * l2;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            atomicAdd(A.lam_cur + pop_at(i, g),
                      (Real)(cx_of(i) * l0 + cy_of(i) * l1 + cz_of(i) * l2 - cu));
    }
#pragma unroll
    for (int m = 1; m < 8; m <<= 1)
        for (int ax = 0; ax < 3; ++ax) dr[ax] += __shfl_xor(dr[ax], m, 8);
    if (corner != 0) return;
    double jp = 0.0, dg = 0.0;
    if constexpr (FREE) {
        // F_k = -gamma (v_k - u_k); the arm d = Q b enters the torque, d and v = V + w x d the
        // kinematics; dr is kept in the body frame of the step's pose
        const Pose& P = A.snap[body].pose[A.pose_par];
        const double* w = P.omega_lab;
        const double* d = arm;
        // (the objective is taken from the body forces by the body pass)
        double lv[3], db[3], y[3];
        // thermal: F_k also holds sqrt(2 kT gamma / h) xi_k = F_k + gamma (v_k - u_k), whose
        // derivative in gamma is itself over 2 gamma (the noise draws are the forward run's)
        const bool noise = a.thermal && X.gamma > 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            dg += lFk[ax] * (s6[ax] - vel[ax]);
            if (noise) dg += lFk[ax] * (Fk[ax] + X.gamma * (vel[ax] - s6[ax])) / (2.0 * X.gamma);
            lv[ax] = -X.gamma * lFk[ax];
        }
        db[0] = dr[0] + (Fk[1] * bj[5] - Fk[2] * bj[4]);
        db[1] = dr[1] + (Fk[2] * bj[3] - Fk[0] * bj[5]);
        db[2] = dr[2] + (Fk[0] * bj[4] - Fk[1] * bj[3]);
        y[0] = db[0] + (lv[1] * w[2] - lv[2] * w[1]);
        y[1] = db[1] + (lv[2] * w[0] - lv[0] * w[2]);
        y[2] = db[2] + (lv[0] * w[1] - lv[1] * w[0]);
        for (int ax = 0; ax < 3; ++ax)
            A.dr[3 * (int64_t)bead + ax] += P.rot[ax] * y[0] + P.rot[3 + ax] * y[1] + P.rot[6 + ax] * y[2];
        const double wd[3] = {w[1] * d[2] - w[2] * d[1], w[2] * d[0] - w[0] * d[2],
                              w[0] * d[1] - w[1] * d[0]};
        double* o = A.bead_sums + kBeadSumWords * (int64_t)bead;
        for (int ax = 0; ax < 3; ++ax) {
            o[ax] = dr[ax];
            o[3 + ax] = lv[ax];
        }
        o[6] = (d[1] * db[2] - d[2] * db[1]) + (wd[1] * lv[2] - wd[2] * lv[1]);
        o[7] = (d[2] * db[0] - d[0] * db[2]) + (wd[2] * lv[0] - wd[0] * lv[2]);
        o[8] = (d[0] * db[1] - d[1] * db[0]) + (wd[0] * lv[1] - wd[1] * lv[0]);
        o[9] = d[1] * lv[2] - d[2] * lv[1];
        o[10] = d[2] * lv[0] - d[0] * lv[2];
        o[11] = d[0] * lv[1] - d[1] * lv[0];
    } else {
        const bool noise = a.thermal && X.gamma > 0.0;   // as above, with v_k = 0
        for (int ax = 0; ax < 3; ++ax) {
            jp += an[ax] * Fk[ax];
            dg += lFk[ax] * s6[ax];
            if (noise) dg += lFk[ax] * (Fk[ax] - X.gamma * s6[ax]) / (2.0 * X.gamma);
            A.dr[3 * (int64_t)bead + ax] += dr[ax];
        }
    }
    A.Jpart[bead] += jp;
    A.dgam[bead] += dg;
}

}  // namespace lbrb
