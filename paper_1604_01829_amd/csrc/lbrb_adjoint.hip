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

#include "lbrb_device.h"

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
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) F[ax] += take_spread_force<Real>(a.gforce, a.N, ax, g);
        a.flags[g] = 0;
    }
    Real lF[3];
    collide_vjp<Real>(a.cp, d, F, lam, lF);
#pragma unroll
    for (int i = 0; i < Q; ++i) A.lam_cur[pop_at(i, g)] = lam[i];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) A.lamF[(int64_t)ax * a.N + g] = lF[ax];
}

// one wave per workgroup: the atomics of a bead pass this short spread over every XCD
constexpr int kAdjBeadBlock = 64;

template <typename Real>
__global__ __launch_bounds__(kAdjBeadBlock) void adj_bead_kernel(const AdjArgs<Real> A)
{
    const StepArgs<Real>& a = A.a;
    const int tid = blockIdx.x * kAdjBeadBlock + threadIdx.x;
    const int bead = tid >> 3, corner = tid & 7;
    if (bead >= A.n_beads) return;   // the 8 lanes of a bead leave together
    // the bead record the forward coupling read: lab position, friction, replica geometry
    // (the bodies are fixed, so one record serves every step of the window)
    const BeadRec& X = A.recs[bead];
    const int32_t body = A.beads[bead].body;
    const double r[3] = {X.r[0], X.r[1], X.r[2]};
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

    ReplicaDesc R{};
    R.nx = X.nx; R.ny = X.ny; R.nz = X.nz; R.masked = X.masked;
    R.base = X.base; R.row_base = X.row_base;
    int64_t local;
    Real d[Q];
    if (X.masked) {
        const RowDesc self = a.rowinfo[X.row_base + py + X.ny * pz];
        const int off = px - self.xlo;
        local = (unsigned)off < (unsigned)self.len ? self.start + off : -1;
        if (local >= 0) pull<Real, true, 1>(a.src, a.N, R, a.rowinfo, px, py, pz, local, self, d);
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
    double lFk[3], luk[3];
    for (int ax = 0; ax < 3; ++ax) {
        lFk[ax] = an[ax] - s6[3 + ax];
        luk[ax] = X.gamma * lFk[ax];
    }
    // position derivative through the interpolation and the spreading weights of this corner
    double dr[3] = {0.0, 0.0, 0.0};
    if (local >= 0) {
        double su = 0.0, sF = 0.0;
        for (int ax = 0; ax < 3; ++ax) { su += uc[ax] * luk[ax]; sF += Fk[ax] * lFc[ax]; }
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
    if (corner == 0) {
        double jp = 0.0, dg = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            jp += an[ax] * Fk[ax];
            dg += lFk[ax] * s6[ax];
            A.dr[3 * (int64_t)bead + ax] += dr[ax];
        }
        A.Jpart[bead] += jp;
        A.dgam[bead] += dg;
    }
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
