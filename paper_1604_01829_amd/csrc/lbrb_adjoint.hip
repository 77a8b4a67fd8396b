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
// With free bodies two small launches frame the bead pass (the rigid-body integrator of
// Sec. 2.3 and the virtual-site kinematics of Sec. 1.2, transposed):
//   adj_body_pre : per body, the adjoint of the step's force and lab torque from the adjoint
//                  of the state after the step (the second half kick) and the weights;
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

__global__ __launch_bounds__(64) void adj_body_pre_kernel(const Body* in, int par,
                                                          const double* weights, const double* adj,
                                                          double* body_adj, int n)
{
    const int b = blockIdx.x * 64 + threadIdx.x;
    if (b >= n) return;
    const Body& B = in[b];
    const double* a = weights + 3 * (int64_t)b;
    double* o = body_adj + 6 * (int64_t)b;
    if (B.fixed) {
        for (int k = 0; k < 3; ++k) { o[k] = a[k]; o[3 + k] = 0.0; }
        return;
    }
    // V_out = V_m + dt F/2M and w_out = w_m + dt (tau - w_m x I w_m)/2I, tau = Q^T T
    const double* ab = adj + kBodyAdjWords * (int64_t)b;
    const double* rot = B.pose[par].rot;
    const double hh = 0.5 * B.dt;
    double tb[3];
    for (int k = 0; k < 3; ++k) {
        o[k] = ab[13 + k] + a[k] + hh * ab[7 + k] / B.mass;
        tb[k] = ab[16 + k] + hh * ab[10 + k] / B.inertia[k];
    }
    for (int r = 0; r < 3; ++r) o[3 + r] = rot[3 * r] * tb[0] + rot[3 * r + 1] * tb[1] + rot[3 * r + 2] * tb[2];
}

__global__ __launch_bounds__(256) void adj_body_post_kernel(const Body* in, const Body* out, int par,
                                                            const double* bead_sums, double* adj)
{
    const Body& B = in[blockIdx.x];
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
    for (int k = 0; k < 3; ++k) th[k] += S[6 + k];
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

void launch_adjoint_body_pre(const Body* in, int par, const double* weights, const double* adj,
                             double* body_adj, int n_bodies, hipStream_t s)
{
    if (n_bodies <= 0) return;
    hipLaunchKernelGGL(adj_body_pre_kernel, dim3((n_bodies + 63) / 64), dim3(64), 0, s, in, par,
                       weights, adj, body_adj, n_bodies);
}

void launch_adjoint_body_post(const Body* in, const Body* out, int par, const double* bead_sums,
                              double* adj, int n_bodies, hipStream_t s)
{
    if (n_bodies <= 0) return;
    hipLaunchKernelGGL(adj_body_post_kernel, dim3(n_bodies), dim3(256), 0, s, in, out, par,
                       bead_sums, adj);
}

template void launch_adjoint_step<float>(const AdjArgs<float>&, bool, hipStream_t);
template void launch_adjoint_step<double>(const AdjArgs<double>&, bool, hipStream_t);
template void launch_adjoint_beads<float>(const AdjArgs<float>&, hipStream_t);
template void launch_adjoint_beads<double>(const AdjArgs<double>&, hipStream_t);

}  // namespace lbrb
