// lbrb_adjoint.hip -- gfx950 kernels of the reverse pass (hand adjoint of the step).
//
// Objective over a window of steps: J = sum_n sum_b a(n,b) . F_b(n), F_b the summed bead force
// of body b.  For a deterministic fluid, one reverse step n takes the adjoint lambda of the
// pre-collision populations of step n+1 to that of step n, and accumulates the derivatives
// with respect to each bead's position (turned into body-frame offsets) and each body's
// friction gamma:
//   adj_node : per fluid node, the transpose of streaming (gather along +c_i, transposed
//              bounce-back) then the vector-Jacobian product of the collision at (f^n, F^n);
//              writes lambda^n (collision part) and the adjoint of the node's force density.
//   adj_bead : per bead corner (8 lanes per bead, as the forward coupling), the transpose of
//              spreading, friction and interpolation: adjoint of the bead force, d/dgamma,
//              d/dposition through the trilinear weights, and the adjoint of the sampled node
//              velocity.  That velocity u = (j + g_ext/2)/rho depends on the node's
//              populations, so lambda^n_i(x_c) += (c_i - u) . (w_c lambda_uk) / rho; the term is
//              linear in each bead's lambda_uk, so every corner adds its own share straight
//              into lambda^n (atomic adds where beads share a node) and no pass over the
//              sampled nodes follows.
// The forward state f^n is re-pulled from the stored post-collision populations of step n-1.
// With free bodies the bead pass forms each body's force and torque adjoint from the adjoint
// of its state after the step (the second half kick) and the weights, and one small launch
// follows it (the rigid-body integrator of Sec. 2.3 and the virtual-site kinematics of
// Sec. 1.2, transposed):
//   adj_body_post: per body, the bead pass's sums (fixed order), then the second half kick,
//                  the torque's body-frame rotation, the bead kinematics, the rotation of the
//                  quaternion, the drift and the first half kick, transposed: the adjoint of
//                  the state before the step.  The rotation's adjoint is gathered as a
//                  lab-frame angle vector theta (the first-order change of J under a small lab
//                  rotation of the pose) and enters the quaternion as (0, 2 theta) (x) q.
#include <hip/hip_runtime.h>

#include "lbrb_adjoint_device.h"

namespace lbrb {

template <typename Real, bool MASKED>
__global__ __launch_bounds__(kNodeBlock) void adj_node_kernel(const AdjArgs<Real> A)
{
    const StepArgs<Real>& a = A.a;
    const NodeTile t = a.tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const ReplicaDesc R = a.reps[t.replica];
    const int64_t local = t.begin + threadIdx.x;
    int x, y, z;
    RowDesc self;
    locate<MASKED>(R, a.rows, t.row_lo, t.row_hi, local, x, y, z, self);
    if (MASKED && R.masked == 2 && a.hole[R.base + local] != 0) {
        // a hole is a boundary node: no adjoint of its own (the transposed mirror later fills
        // the slots its fluid neighbours read)
        const int64_t g = R.base + local;
#pragma unroll
        for (int i = 0; i < Q; ++i) A.lam_cur[pop_at(i, g)] = (Real)0;
        for (int ax = 0; ax < 3; ++ax) A.lamF[(int64_t)ax * a.N + g] = (Real)0;
        if (a.flags[g]) a.flags[g] = 0;
        return;
    }
    Real d[Q], lam[Q];
    pull<Real, MASKED, 1>(a.src, a.N, R, a.rowinfo, x, y, z, local, self, d);
    pull<Real, MASKED, -1>(A.lam_next, a.N, R, a.rowinfo, x, y, z, local, self, lam);
    const int64_t g = R.base + local;
    Real F[3] = {a.gext[0], a.gext[1], a.gext[2]};
    if (a.flags[g]) {
        take_spread_force<Real>(a.gforce, g, F);
        a.flags[g] = 0;
    }
    Real lF[3];
    collide_vjp<Real>(a.cp, d, F, lam, lF);
#pragma unroll
    for (int i = 0; i < Q; ++i) A.lam_cur[pop_at(i, g)] = lam[i];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) A.lamF[(int64_t)ax * a.N + g] = lF[ax];
}

template <typename Real, bool FREE>
__global__ __launch_bounds__(kAdjBeadBlock) void adj_bead_kernel(const AdjArgs<Real> A)
{
    adj_bead_lanes<Real, FREE>(A, blockIdx.x * kAdjBeadBlock + threadIdx.x);
}

template <typename Real>
void launch_adjoint_step(const AdjArgs<Real>& A, bool masked, hipStream_t s)
{
    const dim3 block(kNodeBlock);
    if (A.a.n_tiles > 0) {
        if (masked) hipLaunchKernelGGL((adj_node_kernel<Real, true>), dim3(A.a.n_tiles), block, 0, s, A);
        else hipLaunchKernelGGL((adj_node_kernel<Real, false>), dim3(A.a.n_tiles), block, 0, s, A);
    }
}

template <typename Real>
void launch_adjoint_beads(const AdjArgs<Real>& A, hipStream_t s)
{
    if (A.n_beads <= 0) return;
    const int threads = A.n_beads * kBeadLanes;
    const dim3 grid((threads + kAdjBeadBlock - 1) / kAdjBeadBlock);
    if (A.body_adj)
        hipLaunchKernelGGL((adj_bead_kernel<Real, true>), grid, dim3(kAdjBeadBlock), 0, s, A);
    else
        hipLaunchKernelGGL((adj_bead_kernel<Real, false>), grid, dim3(kAdjBeadBlock), 0, s, A);
}

// ------------------------------------------------------------------ free bodies

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// transpose of the derivative of w x (I w) with respect to w, applied to m:
// (I w) x m + I (m x w)
__device__ __forceinline__ void euler_transpose(const double w[3], const double I[3],
                                                const double m[3], double o[3])
{
    const double Iw[3] = {I[0] * w[0], I[1] * w[1], I[2] * w[2]};
    double a[3], b[3];
    cross3(Iw, m, a);
    cross3(m, w, b);
    for (int k = 0; k < 3; ++k) o[k] = a[k] + I[k] * b[k];
}

// quaternion product a (x) b, components (w, x, y, z)
__device__ __forceinline__ void qmul(const double a[4], const double b[4], double o[4])
{
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

__global__ __launch_bounds__(256) void adj_body_post_kernel(const Body* in, const Body* out, int par,
                                                            const double* weights,
                                                            const double* bead_sums, double* adj,
                                                            double* wadj, double* J)
{
    const Body& B = in[blockIdx.x];
    if (threadIdx.x == 0) {   // the objective: the weight on the force after the MD step
        const double* a = weights + 3 * (int64_t)blockIdx.x;
        const double* Fo = out[blockIdx.x].force;
        J[blockIdx.x] += a[0] * Fo[0] + a[1] * Fo[1] + a[2] * Fo[2];
    }
    if (B.fixed) return;   // uniform over the workgroup
    const int first = B.first_bead, nb = B.n_beads, tid = threadIdx.x;
    double acc[kBeadSumWords];
    for (int j = 0; j < kBeadSumWords; ++j) acc[j] = 0.0;
    for (int k = tid; k < nb; k += 256)
        for (int j = 0; j < kBeadSumWords; ++j) acc[j] += bead_sums[kBeadSumWords * (int64_t)(first + k) + j];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        for (int j = 0; j < kBeadSumWords; ++j) acc[j] += __shfl_down(acc[j], m, 64);
    __shared__ double part[4][kBeadSumWords];
    if ((tid & 63) == 0)
        for (int j = 0; j < kBeadSumWords; ++j) part[tid >> 6][j] = acc[j];
    __syncthreads();
    if (tid != 0) return;
    double S[kBeadSumWords];
    for (int j = 0; j < kBeadSumWords; ++j) S[j] = (part[0][j] + part[1][j]) + (part[2][j] + part[3][j]);
    double* ab = adj + kBodyAdjWords * (int64_t)blockIdx.x;
    double A[kBodyAdjWords];
    for (int j = 0; j < kBodyAdjWords; ++j) A[j] = ab[j];
    const Pose& P = B.pose[par];
    const double* rot = P.rot;
    const double hh = 0.5 * B.dt, dt = B.dt;
    // second half kick
    double mu[3], em[3], wm[3], Vm[3], tau[3], Tb[3], T[3], th[3], Rc[3];
    for (int k = 0; k < 3; ++k) mu[k] = hh * A[10 + k] / B.inertia[k];
    euler_transpose(P.omega, B.inertia, mu, em);
    for (int k = 0; k < 3; ++k) {
        wm[k] = A[10 + k] - em[k] + (rot[k] * S[9] + rot[3 + k] * S[10] + rot[6 + k] * S[11]);
        Vm[k] = A[7 + k] + S[3 + k];
        tau[k] = A[16 + k] + mu[k];
        Rc[k] = A[k] + S[k];
    }
    // tau = Q^T T: its rotation part, with the beads' arms and velocities
    const double* tq = out[blockIdx.x].torque;
    for (int r = 0; r < 3; ++r) {
        Tb[r] = rot[3 * r] * tau[0] + rot[3 * r + 1] * tau[1] + rot[3 * r + 2] * tau[2];
        T[r] = rot[3 * r] * tq[0] + rot[3 * r + 1] * tq[1] + rot[3 * r + 2] * tq[2];
    }
    cross3(Tb, T, th);
    double* wa = wadj + 6 * (int64_t)blockIdx.x;   // the excluded-volume pass's share
    for (int k = 0; k < 3; ++k) {
        th[k] += S[6 + k] + wa[3 + k];
        Rc[k] += wa[k];
    }
    for (int k = 0; k < 6; ++k) wa[k] = 0.0;
    // the pose's quaternion: its own adjoint plus the rotation's
    const double* qc = P.quat;
    const double t2[4] = {0.0, 2.0 * th[0], 2.0 * th[1], 2.0 * th[2]};
    double qt[4], qcb[4], qib[4];
    qmul(t2, qc, qt);
    for (int k = 0; k < 4; ++k) qcb[k] = A[3 + k] + qt[k];
    // q_c = p/|p|, p = q_in (x) (cos(dt|w|/2), sin(dt|w|/2) w/|w|); q_c = q_in when w = 0
    const double* qi = B.quat;
    const double wn = sqrt(P.omega[0] * P.omega[0] + P.omega[1] * P.omega[1] + P.omega[2] * P.omega[2]);
    if (wn > 0.0) {
        const double ang = hh * wn, sn = sin(ang) / wn, cs = cos(ang);
        const double dq[4] = {cs, sn * P.omega[0], sn * P.omega[1], sn * P.omega[2]};
        double p[4];
        qmul(qi, dq, p);
        const double np = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
        const double qq = qc[0] * qcb[0] + qc[1] * qcb[1] + qc[2] * qcb[2] + qc[3] * qcb[3];
        double pb[4], dqb[4];
        for (int k = 0; k < 4; ++k) pb[k] = (qcb[k] - qc[k] * qq) / np;
        const double dqc[4] = {dq[0], -dq[1], -dq[2], -dq[3]};
        const double qic[4] = {qi[0], -qi[1], -qi[2], -qi[3]};
        qmul(pb, dqc, qib);
        qmul(qic, pb, dqb);
        const double dsn = (hh * cs - sn) / wn;
        const double wdq = P.omega[0] * dqb[1] + P.omega[1] * dqb[2] + P.omega[2] * dqb[3];
        for (int k = 0; k < 3; ++k) {
            const double u = P.omega[k] / wn;
            wm[k] += -sin(ang) * hh * u * dqb[0] + sn * dqb[1 + k] + dsn * u * wdq;
        }
    } else {
        for (int k = 0; k < 4; ++k) qib[k] = qcb[k];
    }
    // drift R_c = R_in + dt V_m, first half kick from the previous force and torque
    double mu2[3], em2[3];
    for (int k = 0; k < 3; ++k) {
        Vm[k] += dt * Rc[k];
        mu2[k] = hh * wm[k] / B.inertia[k];
    }
    euler_transpose(B.omega, B.inertia, mu2, em2);
    for (int k = 0; k < 3; ++k) {
        ab[k] = Rc[k];
        ab[7 + k] = Vm[k];
        ab[10 + k] = wm[k] - em2[k];
        ab[13 + k] = hh * Vm[k] / B.mass;
        ab[16 + k] = mu2[k];
    }
    for (int k = 0; k < 4; ++k) ab[3 + k] = qib[k];
}

void launch_adjoint_body_post(const Body* in, const Body* out, int par, const double* weights,
                              const double* bead_sums, double* adj, double* wadj, double* J,
                              int n_bodies, hipStream_t s)
{
    if (n_bodies <= 0) return;
    hipLaunchKernelGGL(adj_body_post_kernel, dim3(n_bodies), dim3(256), 0, s, in, out, par,
                       weights, bead_sums, adj, wadj, J);
}

// ------------------------------------------------------------------ excluded volume

__device__ __forceinline__ void min_image3(const double a[3], const double b[3], const double L[3],
                                           double d[3])
{
    for (int k = 0; k < 3; ++k) {
        d[k] = a[k] - b[k];
        d[k] -= L[k] * round(d[k] / L[k]);
    }
}

// WCA pair at separation d: the force on the first site is c d; returns false beyond the
// cutoff, else c and its derivative c' with respect to |d|^2
__device__ __forceinline__ bool wca_pair_c(double eps, double sigma, const double d[3], double& c,
                                           double& cp)
{
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(r2 < 1.2599210498948732 * sigma * sigma)) return false;   // 2^(1/3) sigma^2
    const double s2 = sigma * sigma / r2, s6 = s2 * s2 * s2, s12 = s6 * s6;
    c = 24.0 * eps * (2.0 * s12 - s6) / r2;
    cp = 24.0 * eps * (4.0 * s6 - 14.0 * s12) / (r2 * r2);
    return true;
}

__device__ __forceinline__ int coarse_cell(double x, double L, double w, int n)
{
    const double xw = x - L * floor(x / L);
    const int c = (int)(xw / w);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// Workgroups of kWcaAdjBlock lanes along blockIdx.y over one body's sites (blockIdx.x),
// eight lanes per site: lane `sub` of a site takes the entries sub, sub + 8, ... of the site's
// coarse-cell neighbourhood list (skipped when the site's fine cell is flagged clear of every
// static site) and of each other body's sites in reach.  Each pair's share for the partner goes
// out by atomic adds; the site's own shares are summed over the workgroup (shuffles, LDS, fixed
// order) and added once.
constexpr int kWcaAdjBlock = 256;
constexpr int kWcaAdjLanes = 8;

__global__ __launch_bounds__(kWcaAdjBlock) void adj_wca_kernel(const BodyArgs ba, int par,
                                                               const double* weights,
                                                               const double* adj, double* wadj)
{
    const int b = blockIdx.x;
    const Body& B = ba.bodies[b];
    const int per_wg = kWcaAdjBlock / kWcaAdjLanes;
    if (B.n_ev == 0 || (int)blockIdx.y * per_wg >= B.n_ev) return;   // uniform over the workgroup
    const Pose& P = B.pose[par];
    const WcaRep W = ba.wrep[B.replica];
    const double L[3] = {(double)B.box.nx, (double)B.box.ny, (double)B.box.nz};
    const double eps = ba.wca_eps;
    double bj[6];   // Fbar_b, Tbar_b (lab)
    force_torque_adjoint(B, P.rot, adj + kBodyAdjWords * (int64_t)b, weights + 3 * (int64_t)b, bj);
    const bool free_b = B.fixed == 0;
    const int k = blockIdx.y * per_wg + (int)threadIdx.x / kWcaAdjLanes;
    const int sub = (int)threadIdx.x % kWcaAdjLanes;
    double acc[6] = {0, 0, 0, 0, 0, 0};             // this body's centre and angle adjoints
    if (k < B.n_ev) {
        const double* off = ba.ev[B.first_ev + k].off;
        double d[3], x[3], g[3];
        for (int ax = 0; ax < 3; ++ax) {
            d[ax] = P.rot[3 * ax] * off[0] + P.rot[3 * ax + 1] * off[1] + P.rot[3 * ax + 2] * off[2];
            x[ax] = P.pos[ax] + d[ax];
        }
        g[0] = bj[0] + (bj[4] * d[2] - bj[5] * d[1]);
        g[1] = bj[1] + (bj[5] * d[0] - bj[3] * d[2]);
        g[2] = bj[2] + (bj[3] * d[1] - bj[4] * d[0]);
        // one pair at separation dd: the adjoint of the separation (df/dd g) and the force
        auto pair = [&](const double dd[3], double sigma, double db[3], double f[3]) {
            double c, cp;
            if (!wca_pair_c(eps, sigma, dd, c, cp)) return false;
            const double dg = dd[0] * g[0] + dd[1] * g[1] + dd[2] * g[2];
            for (int ax = 0; ax < 3; ++ax) {
                db[ax] = c * g[ax] + 2.0 * cp * dg * dd[ax];
                f[ax] = c * dd[ax];
            }
            return true;
        };
        // the site's own share: x = R + d; d also the torque's arm
        auto own = [&](const double db[3], const double f[3]) {
            if (!free_b) return;
            const double a0 = db[0] + (f[1] * bj[5] - f[2] * bj[4]);
            const double a1 = db[1] + (f[2] * bj[3] - f[0] * bj[5]);
            const double a2 = db[2] + (f[0] * bj[4] - f[1] * bj[3]);
            acc[0] += db[0]; acc[1] += db[1]; acc[2] += db[2];
            acc[3] += d[1] * a2 - d[2] * a1;
            acc[4] += d[2] * a0 - d[0] * a2;
            acc[5] += d[0] * a1 - d[1] * a0;
        };
        // static sites: the coarse cell's neighbourhood holds every one in range; the fine flag
        // tells whether any can be
        if (W.cx > 0 &&
            ba.near[W.fine0 + coarse_cell(x[0], L[0], W.fw[0], W.gx) +
                    W.gx * (coarse_cell(x[1], L[1], W.fw[1], W.gy) +
                            W.gy * coarse_cell(x[2], L[2], W.fw[2], W.gz))] != 0) {
            const int cell = W.cell0 + coarse_cell(x[0], L[0], W.cw[0], W.cx) +
                             W.cx * (coarse_cell(x[1], L[1], W.cw[1], W.cy) +
                                     W.cy * coarse_cell(x[2], L[2], W.cw[2], W.cz));
            for (int i = ba.nb_start[cell] + sub; i < ba.nb_start[cell + 1]; i += kWcaAdjLanes) {
                const WallSite ws = ba.nb_sites[i];
                double dd[3], db[3], f[3];
                min_image3(x, ws.p, L, dd);
                if (pair(dd, B.ev_radius + ws.radius, db, f)) own(db, f);
            }
        }
        for (int j = 0; j < W.n_bodies; ++j) {   // the other bodies' sites
            const int o = ba.rep_bodies[W.first_body + j];
            if (o == b) continue;
            const Body& O = ba.bodies[o];
            if (O.n_ev == 0) continue;
            const Pose& Q = O.pose[par];
            double dc[3];
            min_image3(P.pos, Q.pos, L, dc);
            const double reach = B.ev_reach + O.ev_reach + 1.1224620483093730 * (B.ev_radius + O.ev_radius);
            if (!(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2] < reach * reach)) continue;
            const bool free_o = O.fixed == 0;
            for (int m = sub; m < O.n_ev; m += kWcaAdjLanes) {
                const double* oo = ba.ev[O.first_ev + m].off;
                double dq[3], y[3], dd[3], db[3], f[3];
                for (int ax = 0; ax < 3; ++ax) {
                    dq[ax] = Q.rot[3 * ax] * oo[0] + Q.rot[3 * ax + 1] * oo[1] + Q.rot[3 * ax + 2] * oo[2];
                    y[ax] = Q.pos[ax] + dq[ax];
                }
                min_image3(x, y, L, dd);
                if (!pair(dd, B.ev_radius + O.ev_radius, db, f)) continue;
                own(db, f);
                if (free_o) {   // y = R_o + d_o enters the separation with the opposite sign
                    double* wo = wadj + 6 * (int64_t)o;
                    atomicAdd(wo + 0, -db[0]);
                    atomicAdd(wo + 1, -db[1]);
                    atomicAdd(wo + 2, -db[2]);
                    atomicAdd(wo + 3, -(dq[1] * db[2] - dq[2] * db[1]));
                    atomicAdd(wo + 4, -(dq[2] * db[0] - dq[0] * db[2]));
                    atomicAdd(wo + 5, -(dq[0] * db[1] - dq[1] * db[0]));
                }
            }
        }
    }
    if (!free_b) return;   // uniform
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        for (int q = 0; q < 6; ++q) acc[q] += __shfl_down(acc[q], m, 64);
    __shared__ double part[kWcaAdjBlock / 64][6];
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 6; ++q) part[threadIdx.x >> 6][q] = acc[q];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; ++q)
            atomicAdd(wadj + 6 * (int64_t)b + q, (part[0][q] + part[1][q]) + (part[2][q] + part[3][q]));
}

void launch_adjoint_wca(const BodyArgs& ba, int par, const double* weights, const double* adj,
                        double* wadj, int max_ev, hipStream_t s)
{
    if (ba.n_bodies <= 0 || !ba.wca_ft || max_ev <= 0) return;
    const int per_wg = kWcaAdjBlock / kWcaAdjLanes;
    hipLaunchKernelGGL(adj_wca_kernel, dim3(ba.n_bodies, (max_ev + per_wg - 1) / per_wg),
                       dim3(kWcaAdjBlock), 0, s, ba, par, weights, adj, wadj);
}

template void launch_adjoint_step<float>(const AdjArgs<float>&, bool, hipStream_t);
template void launch_adjoint_step<double>(const AdjArgs<double>&, bool, hipStream_t);
template void launch_adjoint_beads<float>(const AdjArgs<float>&, hipStream_t);
template void launch_adjoint_beads<double>(const AdjArgs<double>&, hipStream_t);

}  // namespace lbrb
