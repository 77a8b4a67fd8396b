// lbrb_adjoint.hip -- gfx950 kernels of the reverse pass (hand adjoint of the step).
//
// Objective over a window of steps: J = sum_n sum_b a(n,b) . F_b(n), F_b the summed bead force
// of body b.  For fixed bodies and a deterministic fluid, one reverse step n takes the adjoint
// lambda of the pre-collision populations of step n+1 to that of step n, and accumulates the
// derivatives with respect to each bead's position (later turned into body-frame offsets)
// and each body's friction gamma:
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

template <typename Real>
__global__ __launch_bounds__(kAdjBeadBlock) void adj_bead_kernel(const AdjArgs<Real> A)
{
    adj_bead_lanes<Real>(A, blockIdx.x * kAdjBeadBlock + threadIdx.x);
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
    hipLaunchKernelGGL((adj_bead_kernel<Real>), dim3((threads + kAdjBeadBlock - 1) / kAdjBeadBlock),
                       dim3(kAdjBeadBlock), 0, s, A);
}

template void launch_adjoint_step<float>(const AdjArgs<float>&, bool, hipStream_t);
template void launch_adjoint_step<double>(const AdjArgs<double>&, bool, hipStream_t);
template void launch_adjoint_beads<float>(const AdjArgs<float>&, hipStream_t);
template void launch_adjoint_beads<double>(const AdjArgs<double>&, hipStream_t);

}  // namespace lbrb
