// lbrb_kernels.hip -- gfx950 kernels of the raspberry / lattice-Boltzmann step.
//
// A step is two launches on one stream:
//   couple     : the bead coupling of eq. (latticeboltzmannfriction) of the paper: 8 threads
//                per bead, one per corner of the trilinear stencil; bead position and velocity
//                from the bead's record of the step, fluid velocity from the corner node's
//                pulled populations, lane-butterfly sum, friction + noise, spreading of the
//                opposite force with 64-bit fixed-point atomics (order-independent, hence
//                deterministic), per-bead force and torque.
//   node_step  : the fused lattice-Boltzmann update of every fluid node (Sec. 1.1) -- pull of
//                the 19 populations along the links with halfway bounce-back at boundary
//                nodes, moments, multiple-relaxation-time collision with the external and
//                spread force and thermal noise, back-transform, store; one thread per node,
//                256 nodes per workgroup (one population block), loads/stores coalesced
//                along x.  Its leading workgroups finish the raspberries: per-body
//                force/torque sums (shuffle + LDS tree, fixed order), torque into the body
//                frame, second half kick (Sec. 2.3), pose and bead records of the next step.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

#include "lbrb_adjoint_device.h"
#include "lbrb_device.h"

namespace lbrb {

// launch, timed by events of the dispatch itself when ev.start is set
template <typename K, typename... Args>
void launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t s, const LaunchEvents& ev,
                  Args... args)
{
    if (ev.start)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev.start, ev.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// ------------------------------------------------------------------ node update

// One fluid node: pull, add the force density (external, plus the spread force when the
// node's flag is set and FORCES), collide with the node's noise, store (non-temporal stores
// with NT: they bypass the caches, which pays once the population buffers are far larger than
// the Infinity Cache and costs when they fit in it).
template <typename Real, bool MASKED, bool THERMAL, bool FORCES, bool NARROW, bool NT>
__device__ __forceinline__ void update_node(const StepArgs<Real>& a, const ReplicaDesc& R,
                                            int64_t local, int x, int y, int z,
                                            const RowDesc& self, int64_t step)
{
    // the force flag is loaded before the populations: loads complete in order, so a flag
    // loaded after them would make its branch wait for all of them, and the noise rounds
    // (which need no loaded value) could not run while they are in flight
    const int64_t g = R.base + local;
    uint8_t flag = 0;
    if constexpr (FORCES) flag = a.flags[g];
    Real d[Q];
    pull<Real, MASKED, 1, NARROW>(a.src, a.N, R, a.rowinfo, x, y, z, local, self, d);

    uint32_t w[8];
    if constexpr (THERMAL) {
        // the noise stream of the node in the box's own coordinates
        const uint32_t dense = (uint32_t)box_index(R, x, y, z);
        const U4 b0 = noise_block((uint64_t)step, dense, 0u, 0u, R.key0, R.key1);
        const U4 b1 = noise_block((uint64_t)step, dense, 0u, 1u, R.key0, R.key1);
        w[0] = b0.x; w[1] = b0.y; w[2] = b0.z; w[3] = b0.w;
        w[4] = b1.x; w[5] = b1.y; w[6] = b1.z; w[7] = b1.w;
    }

    Real F[3] = {a.gext[0], a.gext[1], a.gext[2]};
    if constexpr (FORCES) {
        if (flag) {
            take_spread_force<Real>(a.gforce, g, F);
            a.flags[g] = 0;
        }
    }

    if constexpr (THERMAL) {
        Real U[15];
#pragma unroll
        for (int h = 0; h < 15; ++h) U[h] = uniform16<Real>((h & 1) ? (w[h >> 1] >> 16) : w[h >> 1]);
        collide<Real>(a.cp, d, F, U);
    } else {
        collide<Real>(a.cp, d, F, nullptr);
    }

    if constexpr (NARROW) {
        char* __restrict__ rb = (char*)(a.dst + (int64_t)Q * R.base);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            Real* p = (Real*)(rb + pop_byte32<Real>((uint32_t)i, (uint32_t)local));
            if constexpr (NT) __builtin_nontemporal_store(d[i], p);
            else *p = d[i];
        }
    } else {
        Real* __restrict__ dst = a.dst;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if constexpr (NT) __builtin_nontemporal_store(d[i], &dst[pop_at(i, g)]);
            else dst[pop_at(i, g)] = d[i];
        }
    }
}

// What a bead record takes from its body besides the pose (uniform over the workgroup, read
// once into registers).
struct RecConst {
    double gamma, noise_amp;
    int32_t first_in_replica, fixed;
    BodyBox box;
};

__device__ __forceinline__ RecConst rec_const(const Body& B)
{
    return RecConst{B.gamma, B.noise_amp, B.first_bead_in_replica, B.fixed, B.box};
}

// the pose terms a bead record takes, held in scalar registers
struct RecPose {
    double rot[9], pos[3], vel[3], omega_lab[3];
};

__device__ __forceinline__ double uniform_value(double x)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ int32_t uniform_int(int32_t x)
{
    return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
}

__device__ __forceinline__ RecPose uniform_rec_pose(const Pose& P)
{
    RecPose r;
    for (int k = 0; k < 9; ++k) r.rot[k] = uniform_value(P.rot[k]);
    for (int k = 0; k < 3; ++k) {
        r.pos[k] = uniform_value(P.pos[k]);
        r.vel[k] = uniform_value(P.vel[k]);
        r.omega_lab[k] = uniform_value(P.omega_lab[k]);
    }
    return r;
}

// The part of a bead record that follows its body's pose: position, arm r - R and velocity
// (72 bytes, written as four 16-byte stores and one 8-byte store).  r receives the position.
template <typename PoseT>
__device__ __forceinline__ void write_bead_pose(const PoseT& P, bool fixed, const double off[3],
                                                BeadRec& o, double r[3])
{
    static_assert(offsetof(BeadRec, r) == 0 && offsetof(BeadRec, dv) == 24 &&
                  offsetof(BeadRec, v) == 48, "position, arm and velocity lead the record");
    double dv[3], v[3];
    for (int ax = 0; ax < 3; ++ax) {
        dv[ax] = P.rot[3 * ax] * off[0] + P.rot[3 * ax + 1] * off[1] + P.rot[3 * ax + 2] * off[2];
        r[ax] = P.pos[ax] + dv[ax];
    }
    if (fixed) {
        v[0] = v[1] = v[2] = 0.0;
    } else {
        const double* w = P.omega_lab;
        v[0] = P.vel[0] + (w[1] * dv[2] - w[2] * dv[1]);
        v[1] = P.vel[1] + (w[2] * dv[0] - w[0] * dv[2]);
        v[2] = P.vel[2] + (w[0] * dv[1] - w[1] * dv[0]);
    }
    double2* q = reinterpret_cast<double2*>(&o);   // records are 128-byte aligned
    q[0] = make_double2(r[0], r[1]);
    q[1] = make_double2(r[2], dv[0]);
    q[2] = make_double2(dv[1], dv[2]);
    q[3] = make_double2(v[0], v[1]);
    o.v[2] = v[2];
}

// The part of a bead record that stays fixed for the body's lifetime: friction, noise
// amplitude and stream, replica geometry (written when the pose is predicted from the body
// state: after the body was added, a mask was set or a state loaded).
__device__ __forceinline__ void write_bead_const(const RecConst& C, int32_t user, BeadRec& o)
{
    const BodyBox& X = C.box;
    o.gamma = C.gamma;
    o.noise_amp = C.noise_amp;
    o.noise_idx = C.first_in_replica + user;   // noise follows the caller's order
    o.row_base = X.row_base;
    // the box's sides; bit 8 of masked: the replica is stored with axes x and z exchanged
    o.nx = X.nx; o.ny = X.ny; o.nz = X.nz;
    o.masked = X.masked | (X.swap << 8);
    o.base = X.base;
    o.key0 = X.key0; o.key1 = X.key1;
}

// ------------------------------------------------------------------ excluded volume (WCA)

// separation a - b with each component taken to its nearest periodic image
__device__ __forceinline__ void min_image(const double a[3], const double b[3],
                                          const double L[3], double d[3])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d[k] = a[k] - b[k];
        d[k] -= L[k] * round(d[k] / L[k]);
    }
}

// WCA pair at separation d (first site minus second), sigma = r_a + r_b: adds the force on
// the first site to F; nothing at or beyond 2^(1/6) sigma
__device__ __forceinline__ void wca_add(double eps, double sigma, const double d[3], double F[3])
{
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(r2 < 1.2599210498948732 * sigma * sigma)) return;   // 2^(1/3) sigma^2
    const double s2 = sigma * sigma / r2, s6 = s2 * s2 * s2, s12 = s6 * s6;
    const double coef = 24.0 * eps * (2.0 * s12 - s6) / r2;
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] += coef * d[k];
}

__device__ __forceinline__ int cell_of(double x, double L, double w, int n)
{
    const double xw = x - L * floor(x / L);
    int c = (int)(xw / w);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// per-body sums of a workgroup's acc[6] (shuffle + LDS tree, fixed order), valid in thread 0
__device__ __forceinline__ void block_sum6(double acc[6], double (*part)[6], double out[6])
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        for (int k = 0; k < 6; ++k) acc[k] += __shfl_down(acc[k], m, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 6; ++k) part[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) out[k] = (part[0][k] + part[1][k]) + (part[2][k] + part[3][k]);
}

// LDS of one excluded-volume workgroup: the other bodies in range, 64 at a time; the sites
// near static sites of one pass of 256, compacted in site order
struct WcaLds {
    double pose[64][13];         // centre, rotation matrix, site radius
    int32_t site0[64], nsite[64];
    int32_t n;
    double part[4][6];
    double flagged[256][6];      // lab position and arm of each flagged site
    int32_t wave_count[4];
};

// lab position of a body-frame offset at a pose given as centre + row-major rotation
__device__ __forceinline__ void site_at(const double* pos, const double* rot, const double off[3],
                                        double d[3], double x[3])
{
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        d[ax] = rot[3 * ax] * off[0] + rot[3 * ax + 1] * off[1] + rot[3 * ax + 2] * off[2];
        x[ax] = pos[ax] + d[ax];
    }
}

// One workgroup: the WCA force and torque (lab, about the centre) on the excluded-volume
// sites of body b at its pose of MD step S (parity = S & 1), from the static sites of its
// replica (through the cell grid) and from the sites of the replica's other bodies at their
// poses of the same MD step; 6 doubles into ba.wca_ft.  The other bodies are screened 64 at
// a time by their centre distance; the ones in range are compacted in body order (ballot),
// so the sums do not depend on timing.
__device__ __forceinline__ void wca_block(const BodyArgs& ba, int b, int parity, WcaLds& S)
{
    const Body& B = ba.bodies[b];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (B.n_ev > 0) {
        const Pose& P = B.pose[parity];
        const WcaRep W = ba.wrep[B.replica];
        const double L[3] = {(double)B.box.nx, (double)B.box.ny, (double)B.box.nz};
        const double eps = ba.wca_eps;
        // static sites, 256 per pass: the fine flag of each; the flagged ones are compacted
        // in site order (wave ballots, then the waves' offsets) and each is walked by eight
        // lanes over the coarse cell's neighbourhood list (entries l, l + 8, ...; the eight
        // partial forces combined in a fixed butterfly), the group's first lane adding the
        // site's force and torque
        if (W.cx > 0) {
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            const int grp = threadIdx.x >> 3, sub = threadIdx.x & 7;
            for (int k0 = 0; k0 < B.n_ev; k0 += blockDim.x) {
                const int k = k0 + threadIdx.x;
                double d[3] = {0.0, 0.0, 0.0}, x[3] = {0.0, 0.0, 0.0};
                bool flag = false;
                if (k < B.n_ev) {
                    site_at(P.pos, P.rot, ba.ev[B.first_ev + k].off, d, x);
                    const int g0 = cell_of(x[0], L[0], W.fw[0], W.gx);
                    const int g1 = cell_of(x[1], L[1], W.fw[1], W.gy);
                    const int g2 = cell_of(x[2], L[2], W.fw[2], W.gz);
                    flag = ba.near[W.fine0 + g0 + W.gx * (g1 + W.gy * g2)] != 0;
                }
                const unsigned long long mask = __ballot(flag);
                if (lane == 0) S.wave_count[wave] = __popcll(mask);
                __syncthreads();
                int pos = __popcll(mask & ((1ull << lane) - 1ull)), nflag = 0;
                for (int w = 0; w < 4; ++w) {
                    if (w < wave) pos += S.wave_count[w];
                    nflag += S.wave_count[w];
                }
                if (flag)
                    for (int t = 0; t < 3; ++t) {
                        S.flagged[pos][t] = x[t];
                        S.flagged[pos][3 + t] = d[t];
                    }
                __syncthreads();
                for (int c0 = 0; c0 < nflag; c0 += 32) {
                    const int f = c0 + grp;
                    double F[3] = {0.0, 0.0, 0.0};
                    double xs[3] = {0.0, 0.0, 0.0};
                    if (f < nflag) {
                        for (int t = 0; t < 3; ++t) xs[t] = S.flagged[f][t];
                        const int c0c = cell_of(xs[0], L[0], W.cw[0], W.cx);
                        const int c1c = cell_of(xs[1], L[1], W.cw[1], W.cy);
                        const int c2c = cell_of(xs[2], L[2], W.cw[2], W.cz);
                        const int cell = W.cell0 + c0c + W.cx * (c1c + W.cy * c2c);
                        const int i1 = ba.nb_start[cell + 1];
                        for (int i = ba.nb_start[cell] + sub; i < i1; i += 8) {
                            const WallSite ws = ba.nb_sites[i];
                            double dd[3];
                            min_image(xs, ws.p, L, dd);
                            wca_add(eps, B.ev_radius + ws.radius, dd, F);
                        }
                    }
#pragma unroll
                    for (int m = 1; m < 8; m <<= 1)
                        for (int t = 0; t < 3; ++t) F[t] += __shfl_xor(F[t], m, 8);
                    if (f < nflag && sub == 0) {
                        const double* ds = &S.flagged[f][3];
                        acc[0] += F[0]; acc[1] += F[1]; acc[2] += F[2];
                        acc[3] += ds[1] * F[2] - ds[2] * F[1];
                        acc[4] += ds[2] * F[0] - ds[0] * F[2];
                        acc[5] += ds[0] * F[1] - ds[1] * F[0];
                    }
                }
                __syncthreads();
            }
        }
        // other bodies, 64 candidates at a time
        for (int j0 = 0; j0 < W.n_bodies; j0 += 64) {
            if (threadIdx.x < 64) {
                const int lane = threadIdx.x, j = j0 + lane;
                bool close = false;
                int o = -1;
                if (j < W.n_bodies) {
                    o = ba.rep_bodies[W.first_body + j];
                    if (o != b && ba.bodies[o].n_ev > 0) {
                        const Body& O = ba.bodies[o];
                        double dc[3];
                        min_image(P.pos, O.pose[parity].pos, L, dc);
                        const double reach = B.ev_reach + O.ev_reach +
                                             1.1224620483093730 * (B.ev_radius + O.ev_radius);
                        close = dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2] < reach * reach;
                    }
                }
                const unsigned long long mask = __ballot(close);
                if (close) {
                    const int q = __popcll(mask & ((1ull << lane) - 1ull));
                    const Body& O = ba.bodies[o];
                    const Pose& Q = O.pose[parity];
                    for (int t = 0; t < 3; ++t) S.pose[q][t] = Q.pos[t];
                    for (int t = 0; t < 9; ++t) S.pose[q][3 + t] = Q.rot[t];
                    S.pose[q][12] = O.ev_radius;
                    S.site0[q] = O.first_ev;
                    S.nsite[q] = O.n_ev;
                }
                if (lane == 0) S.n = __popcll(mask);
            }
            __syncthreads();
            const int nc = S.n;
            for (int k = threadIdx.x; k < B.n_ev && nc > 0; k += blockDim.x) {
                double d[3], x[3], F[3] = {0.0, 0.0, 0.0};
                site_at(P.pos, P.rot, ba.ev[B.first_ev + k].off, d, x);
                for (int q = 0; q < nc; ++q) {
                    const double sigma = B.ev_radius + S.pose[q][12];
                    for (int m = 0; m < S.nsite[q]; ++m) {
                        double dq[3], xo[3], dd[3];
                        site_at(&S.pose[q][0], &S.pose[q][3], ba.ev[S.site0[q] + m].off, dq, xo);
                        min_image(x, xo, L, dd);
                        wca_add(eps, sigma, dd, F);
                    }
                }
                acc[0] += F[0]; acc[1] += F[1]; acc[2] += F[2];
                acc[3] += d[1] * F[2] - d[2] * F[1];
                acc[4] += d[2] * F[0] - d[0] * F[2];
                acc[5] += d[0] * F[1] - d[1] * F[0];
            }
            __syncthreads();
        }
    }
    double out[6];
    block_sum6(acc, S.part, out);
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; ++q) ba.wca_ft[6 * b + q] = out[q];
}

// one workgroup per body: sum the bead forces and torques (shuffle + LDS tree, fixed order),
// add the excluded-volume force and torque of the MD step, turn the torque into the body
// frame, second half kick, pose of the next MD step and the pose part of its bead records
// (write_bead_pose).  parity: of the MD step being finished.  Two dependent rounds of loads:
// the body's bead range, then together the bead forces, each thread's first two bead
// offsets (parked in LDS), and the step's pose, mass, inertia, dt and excluded-volume sums
// (one word per lane into LDS).  The next pose is built in LDS, stored by 25 lanes, and read
// back into scalar registers for the records, so that this code needs fewer registers than
// the node update it shares a kernel with.
__device__ __forceinline__ void body_finish(const BodyArgs& ba, int b, int parity)
{
    constexpr int kPre = 2;                       // bead offsets fetched with the forces
    constexpr int kPoseWords = sizeof(Pose) / sizeof(double);
    static_assert(sizeof(Pose) == 25 * sizeof(double), "a pose is 25 doubles");
    static_assert(offsetof(Body, dt) == offsetof(Body, mass) + 6 * sizeof(double),
                  "mass, inertia, gamma, noise_amp, dt are consecutive");
    __shared__ double part[4][6];
    __shared__ Pose cur, next;
    __shared__ double st[12];                     // vel, omega, force, body torque after the step
    __shared__ double cst[13];                    // mass, inertia[3], gamma, noise, dt, wca F, T
    const Body& B = ba.bodies[b];
    const int first = B.first_bead, n = B.n_beads;
    const int tid = threadIdx.x;
    const int fixed = B.fixed;
    const bool has_wca = ba.wca_ft != nullptr;
    if (tid < kPoseWords) {
        reinterpret_cast<double*>(&cur)[tid] = reinterpret_cast<const double*>(&B.pose[parity])[tid];
    } else if (tid < kPoseWords + 7) {
        cst[tid - kPoseWords] = reinterpret_cast<const double*>(&B.mass)[tid - kPoseWords];
    } else if (tid < kPoseWords + 13) {
        cst[tid - kPoseWords] = has_wca ? ba.wca_ft[6 * b + tid - kPoseWords - 7] : 0.0;
    }
    __shared__ double pre_off[kPre][3][256];     // body-frame offsets of each thread's first beads
    const double* __restrict__ bf = ba.bead_force;
    const double* __restrict__ bt = ba.bead_torque;
    double acc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
        const int k = tid + q * 256;
        if (k < n) {
            const int64_t e = 3 * (int64_t)(first + k);
            const Bead& bd = ba.beads[first + k];
            const double o0 = bd.off[0], o1 = bd.off[1], o2 = bd.off[2];
            const double f0 = bf[e], f1 = bf[e + 1], f2 = bf[e + 2];
            const double t0 = bt[e], t1 = bt[e + 1], t2 = bt[e + 2];
            acc[0] += f0; acc[1] += f1; acc[2] += f2;
            acc[3] += t0; acc[4] += t1; acc[5] += t2;
            pre_off[q][0][tid] = o0; pre_off[q][1][tid] = o1; pre_off[q][2][tid] = o2;
        }
    }
    for (int k = tid + kPre * 256; k < n; k += 256) {
        const int64_t e = 3 * (int64_t)(first + k);
        acc[0] += bf[e]; acc[1] += bf[e + 1]; acc[2] += bf[e + 2];
        acc[3] += bt[e]; acc[4] += bt[e + 1]; acc[5] += bt[e + 2];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        for (int k = 0; k < 6; ++k) acc[k] += __shfl_down(acc[k], m, 64);
    const int wave = tid >> 6;
    if ((tid & 63) == 0)
        for (int k = 0; k < 6; ++k) part[wave][k] = acc[k];
    __syncthreads();
    Body& o = ba.bodies[b];
    if (tid == 0) {
        double F[3], T[3];
        for (int k = 0; k < 3; ++k) {
            F[k] = (part[0][k] + part[1][k]) + (part[2][k] + part[3][k]);
            T[k] = (part[0][3 + k] + part[1][3 + k]) + (part[2][3 + k] + part[3][3 + k]);
        }
        if (has_wca) {
            for (int k = 0; k < 3; ++k) {
                F[k] += cst[7 + k];
                T[k] += cst[10 + k];
            }
        }
        const double mass = cst[0], dt = cst[6];
        const double inertia[3] = {cst[1], cst[2], cst[3]};
        // second half kick with this step's force and body-frame torque, from the step's pose
        const Pose& P = cur;
        double vel[3], om[3], Tb[3];
        for (int ax = 0; ax < 3; ++ax) {
            vel[ax] = P.vel[ax];
            om[ax] = P.omega[ax];
            Tb[ax] = P.rot[ax] * T[0] + P.rot[3 + ax] * T[1] + P.rot[6 + ax] * T[2];
        }
        if (!fixed) {
            const double hh = 0.5 * dt;
            for (int ax = 0; ax < 3; ++ax) vel[ax] += hh * F[ax] / mass;
            half_kick(om, inertia, Tb, dt);
        }
        for (int ax = 0; ax < 3; ++ax) {
            o.pos[ax] = P.pos[ax];
            o.vel[ax] = st[ax] = vel[ax];
            o.omega[ax] = st[3 + ax] = om[ax];
            o.force[ax] = st[6 + ax] = F[ax];
            o.torque[ax] = st[9 + ax] = Tb[ax];
        }
        for (int k = 0; k < 4; ++k) o.quat[k] = P.quat[k];
        // the prediction reads the state back from LDS (fewer live registers)
        asm volatile("" ::: "memory");
        first_half(cur.pos, cur.quat, st, st + 3, st + 6, st + 9, cst[0], cst + 1, cst[6],
                   fixed != 0, next.pos, next.quat, next.vel, next.omega);
        complete_pose(next);
    }
    __syncthreads();
    if (tid < kPoseWords)
        reinterpret_cast<double*>(&o.pose[parity ^ 1])[tid] = reinterpret_cast<const double*>(&next)[tid];
    const RecPose RP = uniform_rec_pose(next);
    for (int q = 0, k = tid; k < n; ++q, k += 256) {
        double off[3];
        if (q < kPre) {
            for (int ax = 0; ax < 3; ++ax) off[ax] = pre_off[q][ax][tid];
        } else {
            const Bead& bd = ba.beads[first + k];
            for (int ax = 0; ax < 3; ++ax) off[ax] = bd.off[ax];
        }
        double r[3];
        write_bead_pose(RP, fixed != 0, off, ba.recs[first + k], r);
    }
}

// The node update of one tile group.  With FORCES the nodes consume the spread force of the
// coupling.  The first n_lead workgroups (0, or a multiple of 8 so that blockIdx % 8 still
// picks the XCD of the node tiles) finish the bodies: they read only the per-bead forces of
// the coupling and write only body records, which no node thread touches.  Every other workgroup updates PER consecutive tiles (a
// tuning choice; the XCD-aware order deals runs of them to each XCD).
// FP32: 72 registers give 7 wavefronts per SIMD (the FP32 paths fit without spills; FP64 is
// left to the compiler)
template <typename Real, bool MASKED, bool THERMAL, bool FORCES, bool NARROW, bool NT, int PER>
__global__ __launch_bounds__(kNodeBlock) __attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? 7 : 1)))
void node_step_kernel(const StepArgs<Real> a, const BodyArgs ba, int n_lead)
{
    const int64_t step = current_step(a.step_ptr, a.step_arg);
    int b = blockIdx.x;
    if (b < n_lead) {
        // the last MD step of this fluid step
        if (b < ba.n_bodies)
            body_finish(ba, b, (int)((step * ba.substeps + ba.substeps - 1) & 1));
        return;
    }
    b -= n_lead;
    __shared__ RowDesc tile_rows[MASKED ? kNodeBlock : 1];
    if constexpr (PER == 1) {
        const NodeTile t = a.tiles[xcd_tile(b, gridDim.x - n_lead)];
        const ReplicaDesc R = a.reps[t.replica];
        const int64_t local = t.begin + threadIdx.x;
        int x, y, z;
        RowDesc self;
        locate_tile<MASKED>(R, a.rows, t, local, tile_rows, x, y, z, self);
        if ((int)threadIdx.x >= t.count) return;
        update_node<Real, MASKED, THERMAL, FORCES, NARROW, NT>(a, R, local, x, y, z, self, step);
    } else {
        const int first = xcd_tile(b, gridDim.x - n_lead) * PER;
        for (int q = 0; q < PER; ++q) {
            const int ti = first + q;
            if (ti >= a.n_tiles) break;               // uniform over the workgroup
            if (MASKED && q > 0) __syncthreads();     // the previous tile's rows are no longer read
            const NodeTile t = a.tiles[ti];
            const ReplicaDesc R = a.reps[t.replica];
            const int64_t local = t.begin + threadIdx.x;
            int x, y, z;
            RowDesc self;
            locate_tile<MASKED>(R, a.rows, t, local, tile_rows, x, y, z, self);
            if ((int)threadIdx.x < t.count)
                update_node<Real, MASKED, THERMAL, FORCES, NARROW, NT>(a, R, local, x, y, z, self,
                                                                     step);
        }
    }
}

template <typename K>
int node_wg_lds(K kernel)
{
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel)) != hipSuccess) return 0;
    return (int)fa.sharedSizeBytes;
}

// LDS bytes one workgroup may allocate on the current device
inline int max_wg_lds()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 64 * 1024;
    return v;
}

// launch with dynamic LDS that caps the workgroups resident per CU at wg_per_cu (0: no cap;
// the request is clamped to what one workgroup may allocate)
template <typename K, typename... Args>
void launch_node_capped(K kernel, dim3 grid, hipStream_t s, const LaunchEvents& ev, int wg_per_cu,
                        Args... args)
{
    size_t dyn = 0;
    if (wg_per_cu > 0) {
        static const int limit = max_wg_lds();
        const int stat = node_wg_lds(kernel);
        const int want = std::min(kLdsPerCu / wg_per_cu, limit) - stat;
        dyn = want > 0 ? (size_t)want : 0;
    }
    if (ev.start)
        hipExtLaunchKernelGGL(kernel, grid, dim3(kNodeBlock), dyn, s, ev.start, ev.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, dim3(kNodeBlock), dyn, s, args...);
}

template <typename Real, bool MASKED, bool THERMAL, bool NARROW, int PER>
void launch_node_p(const StepArgs<Real>& a, bool forces, const BodyArgs& ba, int n_lead,
                   hipStream_t s, const LaunchEvents& ev)
{
    const dim3 grid((a.n_tiles + PER - 1) / PER + n_lead);
    const int cap = a.wg_per_cu;
    if (a.stream_stores) {
        if (forces)
            launch_node_capped(node_step_kernel<Real, MASKED, THERMAL, true, NARROW, true, PER>,
                               grid, s, ev, cap, a, ba, n_lead);
        else
            launch_node_capped(node_step_kernel<Real, MASKED, THERMAL, false, NARROW, true, PER>,
                               grid, s, ev, cap, a, ba, n_lead);
    } else {
        if (forces)
            launch_node_capped(node_step_kernel<Real, MASKED, THERMAL, true, NARROW, false, PER>,
                               grid, s, ev, cap, a, ba, n_lead);
        else
            launch_node_capped(node_step_kernel<Real, MASKED, THERMAL, false, NARROW, false, PER>,
                               grid, s, ev, cap, a, ba, n_lead);
    }
}

template <typename Real, bool MASKED, bool THERMAL, bool NARROW>
void launch_node_t(const StepArgs<Real>& a, bool forces, const BodyArgs* bodies, hipStream_t s,
                   const LaunchEvents& ev)
{
    BodyArgs ba{};
    if (bodies) ba = *bodies;
    const int n_lead = ba.n_bodies > 0 ? (ba.n_bodies + 7) & ~7 : 0;
    if (a.tiles_per_wg == kWideTiles)
        launch_node_p<Real, MASKED, THERMAL, NARROW, kWideTiles>(a, forces, ba, n_lead, s, ev);
    else
        launch_node_p<Real, MASKED, THERMAL, NARROW, 1>(a, forces, ba, n_lead, s, ev);
}

// 32-bit offsets pay in FP32 (+2 % on a pore, +1 % on a batch); FP64 keeps 64-bit indices
template <typename Real, bool MASKED, bool THERMAL>
void launch_node_w(const StepArgs<Real>& a, bool forces, const BodyArgs* bodies, hipStream_t s,
                   const LaunchEvents& ev)
{
    if constexpr (sizeof(Real) == 4) {
        if (a.narrow) {
            launch_node_t<Real, MASKED, THERMAL, true>(a, forces, bodies, s, ev);
            return;
        }
    }
    launch_node_t<Real, MASKED, THERMAL, false>(a, forces, bodies, s, ev);
}

template <typename Real>
void launch_node_step(const StepArgs<Real>& a, bool masked, bool forces, const BodyArgs* bodies,
                      hipStream_t s, const LaunchEvents& ev)
{
    if (a.n_tiles <= 0 && !(bodies && bodies->n_bodies > 0)) return;
    if (masked) {
        if (a.thermal) launch_node_w<Real, true, true>(a, forces, bodies, s, ev);
        else launch_node_w<Real, true, false>(a, forces, bodies, s, ev);
    } else {
        if (a.thermal) launch_node_w<Real, false, true>(a, forces, bodies, s, ev);
        else launch_node_w<Real, false, false>(a, forces, bodies, s, ev);
    }
}

// ------------------------------------------------------------------ bead coupling


// Thread t handles corner t & 7 of bead t >> 3.  The dependent loads are kept to three
// rounds: the bead's record of the step (position, velocity, friction, replica geometry) ->
// the 9 row descriptors around the corner node -> its 19 populations.  Within a workgroup
// (32 beads) the stencil nodes are deduplicated through an LDS hash table keyed by node:
// the first lane to claim a node pulls its populations once and publishes (drho, j); the
// lanes' force contributions are summed as fixed-point words in LDS and the node's owner
// adds each sum to the node with one device atomic per word.  Integer sums do not depend on
// their order, so the result is the same as one atomic per lane.

// LDS of one coupling workgroup: the node hash table, the nodes' moments and the force sums.
// A workgroup's lanes claim at most kCoupleBlock distinct nodes, so kCoupleBlock slots always
// suffice; FP32 takes twice that (shorter probes), FP64 takes kCoupleBlock so that its larger
// entries leave room for 4 instead of 3 workgroups per CU (the batch's FP64 coupling 248 ->
// 236 us).
template <typename Real>
struct CoupleLds {
    static constexpr int TS = (sizeof(Real) == 8 ? 1 : 2) * kCoupleBlock;   // power of two
    static constexpr int NW = sizeof(Real) == 8 ? 6 : 3; // fixed-point words per node
    unsigned long long key[TS];
    Real mom[4][TS];
    unsigned long long acc[NW][TS];
};

// the coupling of bead block cb of ncb (32 beads)
template <typename Real>
__device__ __forceinline__ void couple_beads(const StepArgs<Real>& a, const CoupleArgs& c, int cb,
                                             int ncb, CoupleLds<Real>& L)
{
    constexpr int TS = CoupleLds<Real>::TS;
    constexpr int NW = CoupleLds<Real>::NW;
    constexpr unsigned long long EMPTY = ~0ull;
    unsigned long long* key = L.key;
    Real (*mom)[TS] = L.mom;
    unsigned long long (*acc)[TS] = L.acc;
    for (int k = threadIdx.x; k < TS; k += kCoupleBlock) {
        key[k] = EMPTY;
        for (int w = 0; w < NW; ++w) acc[w][k] = 0;
    }

    // consecutive bead blocks (neighbouring beads of one body, sharing stencil rows) stay on
    // one XCD and its L2
    const int tid = xcd_tile(cb, ncb) * kCoupleBlock + threadIdx.x;
    const int bead = tid >> 3, corner = tid & 7;
    const bool active = bead < c.n_beads;   // the 8 lanes of a bead share this
    const int64_t step = current_step(a.step_ptr, a.step_arg);
    // the record spread over the bead's 8 lanes; the geometry is gathered now, the dynamics
    // after the stencil's populations are in
    const uint4 rq = reinterpret_cast<const uint4*>(c.recs + (active ? bead : 0))[corner];
    const int nx = (int)rec_word<LBRB_REC_WORD(nx)>(rq);
    const int ny = (int)rec_word<LBRB_REC_WORD(ny)>(rq);
    const int nz = (int)rec_word<LBRB_REC_WORD(nz)>(rq);
    const int mword = (int)rec_word<LBRB_REC_WORD(masked)>(rq);
    const int masked = mword & 0xFF;
    const bool swap = (mword >> 8) != 0;   // storage axes x and z exchanged
    const double r[3] = {rec_f64<LBRB_REC_WORD(r[0])>(rq), rec_f64<LBRB_REC_WORD(r[1])>(rq),
                         rec_f64<LBRB_REC_WORD(r[2])>(rq)};
    const int row_base = (int)rec_word<LBRB_REC_WORD(row_base)>(rq);
    const int64_t base = (int64_t)(((uint64_t)rec_word<LBRB_REC_WORD(base) + 1>(rq) << 32) |
                                   rec_word<LBRB_REC_WORD(base)>(rq));

    // corner of the trilinear stencil handled by this lane, in box coordinates (so the weights
    // and the corner sums do not depend on the storage axes)
    double fr[3];
    int i0[3];
    i0[0] = wrap_floor(r[0] - 0.5, nx, fr[0]);
    i0[1] = wrap_floor(r[1] - 0.5, ny, fr[1]);
    i0[2] = wrap_floor(r[2] - 0.5, nz, fr[2]);
    const int ox = corner & 1, oy = (corner >> 1) & 1, oz = corner >> 2;
    const int px = i0[0] + ox == nx ? 0 : i0[0] + ox;
    const int py = i0[1] + oy == ny ? 0 : i0[1] + oy;
    const int pz = i0[2] + oz == nz ? 0 : i0[2] + oz;
    const double w = (ox ? fr[0] : 1.0 - fr[0]) * (oy ? fr[1] : 1.0 - fr[1]) *
                     (oz ? fr[2] : 1.0 - fr[2]);

    // the node in storage coordinates and sides
    const int sx = swap ? pz : px, sz = swap ? px : pz;
    const int snx = swap ? nz : nx, snz = swap ? nx : nz;

    // the node's local index (-1: boundary node or no bead)
    int64_t local = -1;
    Rows9 rw;
    if (active) {
        if (masked) {
            load_rows9(a.rowinfo, row_base, ny, snz, py, sz, rw);
            const int off = sx - rw.lo[4];
            local = (unsigned)off < (unsigned)rw.ln[4] ? rw.st[4] + off : -1;
            // a hole is a boundary node: no velocity sampled, no force spread
            if (masked == 2 && local >= 0 && a.hole[base + local] != 0) local = -1;
        } else {
            local = px + (int64_t)nx * (py + (int64_t)ny * pz);
        }
    }
    const int64_t g = base + local;
    __syncthreads();   // the table is cleared

    // claim the node's slot
    int slot = -1;
    bool owner = false;
    if (local >= 0) {
        slot = (int)(((uint32_t)g * 2654435761u) >> 23) & (TS - 1);
        while (true) {
            const unsigned long long prev = atomicCAS(&key[slot], EMPTY, (unsigned long long)g);
            if (prev == EMPTY) { owner = true; break; }
            if (prev == (unsigned long long)g) break;
            slot = (slot + 1) & (TS - 1);
        }
    }
    // the owner pulls the node's populations (pre-collision of this step)
    if (owner) {
        Real d[Q];
        if (masked) {
            pull_rows<Real, 1>(a.src, base, snx, rw, sx, local, d, swap);
        } else {
            ReplicaDesc R{};
            R.nx = nx; R.ny = ny; R.nz = nz;
            R.base = base;
            const RowDesc self{0, 0, nx, 0};
            pull<Real, false>(a.src, a.N, R, a.rowinfo, px, py, pz, local, self, d);
        }
        Real drho, j[3];
        density_momentum<Real>(d, drho, j);
        mom[0][slot] = drho;
        for (int ax = 0; ax < 3; ++ax) mom[1 + ax][slot] = j[ax];
    }
    __syncthreads();

    double wu[3] = {0.0, 0.0, 0.0};
    if (local >= 0) {
        const double wr = w / ((double)a.cp.rho0 + (double)mom[0][slot]);
        for (int ax = 0; ax < 3; ++ax)
            wu[ax] = wr * ((double)mom[1 + ax][slot] + 0.5 * (double)a.gext[ax]);
    }
    // sum over the 8 corner lanes (same association on every lane)
#pragma unroll
    for (int m = 1; m < 8; m <<= 1)
        for (int ax = 0; ax < 3; ++ax) wu[ax] += __shfl_xor(wu[ax], m, 8);

    const double gamma = rec_f64<LBRB_REC_WORD(gamma)>(rq);
    const double v[3] = {rec_f64<LBRB_REC_WORD(v[0])>(rq), rec_f64<LBRB_REC_WORD(v[1])>(rq),
                         rec_f64<LBRB_REC_WORD(v[2])>(rq)};
    double F[3];
    for (int ax = 0; ax < 3; ++ax) F[ax] = -gamma * (v[ax] - wu[ax]);
    if (c.kT > 0.0) {
        const U4 blk = noise_block((uint64_t)step, rec_word<LBRB_REC_WORD(noise_idx)>(rq), 1u,
                                   c.md_step, rec_word<LBRB_REC_WORD(key0)>(rq),
                                   rec_word<LBRB_REC_WORD(key1)>(rq));
        const double amp = rec_f64<LBRB_REC_WORD(noise_amp)>(rq);
        F[0] += amp * uniform16<double>(blk.x);
        F[1] += amp * uniform16<double>(blk.x >> 16);
        F[2] += amp * uniform16<double>(blk.y);
    }

    if (local >= 0) {
        bool overflow = false;
        for (int ax = 0; ax < 3; ++ax) {
            const double val = -(w * (c.spread_h * F[ax]));
            const bool bad = !(fabs(val) < 16.0);
            overflow |= bad;
            long long hi, lo;
            spread_words<Real>(bad ? 0.0 : val, hi, lo);
            atomicAdd(&acc[ax][slot], (unsigned long long)hi);
            if constexpr (NW == 6) atomicAdd(&acc[3 + ax][slot], (unsigned long long)lo);
        }
        if (overflow) atomicOr(&c.hdr->err_flags, 1u);
    }
    const double dv[3] = {rec_f64<LBRB_REC_WORD(dv[0])>(rq), rec_f64<LBRB_REC_WORD(dv[1])>(rq),
                          rec_f64<LBRB_REC_WORD(dv[2])>(rq)};
    if (active && corner == 0) {
        for (int ax = 0; ax < 3; ++ax) c.bead_force[3 * bead + ax] = F[ax];
        c.bead_torque[3 * bead + 0] = dv[1] * F[2] - dv[2] * F[1];
        c.bead_torque[3 * bead + 1] = dv[2] * F[0] - dv[0] * F[2];
        c.bead_torque[3 * bead + 2] = dv[0] * F[1] - dv[1] * F[0];
    }
    __syncthreads();
    // one device atomic per node and word
    if (owner) {
        unsigned long long* gw = (unsigned long long*)(a.gforce + g * spread_stride<Real>());
        for (int wd = 0; wd < NW; ++wd) {
            const unsigned long long v = acc[wd][slot];
            if (v != 0) atomicAdd(gw + wd, v);
        }
        a.flags[g] = 1;
    }
}

// The coupling launch.  With excluded volume (WCA), the first n_wca workgroups (a multiple of
// 8, so that the bead workgroups keep their XCD pattern) compute each body's WCA force and
// torque for the same MD step instead (wca_block); they use the coupling's LDS.
// Without it the kernel is compiled without that code (its registers stay those of the
// coupling alone).  In FP32 the LDS admits 6 workgroups per CU; the coupling alone fits the
// 80 registers of 6 waves per SIMD without spilling, so it is compiled for that occupancy.
template <typename Real, bool WCA>
__global__ __launch_bounds__(kCoupleBlock)
__attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 && !WCA ? 6 : 1)))
void couple_kernel(const StepArgs<Real> a, const CoupleArgs c, const BodyArgs ba, int n_wca)
{
    __shared__ CoupleLds<Real> L;
    static_assert(sizeof(L) >= sizeof(WcaLds), "excluded-volume LDS fits in the coupling's");
    if (WCA && (int)blockIdx.x < n_wca) {
        if ((int)blockIdx.x < ba.n_bodies) {
            const int64_t step = current_step(a.step_ptr, a.step_arg);
            wca_block(ba, blockIdx.x, (int)((step * ba.substeps + c.md_step) & 1),
                      *reinterpret_cast<WcaLds*>(&L));
        }
        return;
    }
    couple_beads<Real>(a, c, blockIdx.x - n_wca, gridDim.x - n_wca, L);
}

template <typename Real>
void launch_couple(const StepArgs<Real>& a, const CoupleArgs& c, hipStream_t s,
                   const LaunchEvents& ev, const BodyArgs* wca)
{
    if (c.n_beads <= 0) return;
    BodyArgs ba{};
    int n_wca = 0;
    if (wca && wca->wca_ft && wca->n_bodies > 0) {
        ba = *wca;
        n_wca = (ba.n_bodies + 7) & ~7;
    }
    const int threads = c.n_beads * kBeadLanes;
    const dim3 grid((threads + kCoupleBlock - 1) / kCoupleBlock + n_wca);
    if (n_wca > 0)
        launch_timed(couple_kernel<Real, true>, grid, dim3(kCoupleBlock), s, ev, a, c, ba, n_wca);
    else
        launch_timed(couple_kernel<Real, false>, grid, dim3(kCoupleBlock), s, ev, a, c, ba, 0);
}

// Reverse pass: the coupling recompute of the next reverse step (forward step n-1, from its
// own state) in the same launch as the bead pass of reverse step n.  The two touch disjoint
// data: the coupling writes the spread force and flags of step n-1 (the node pass of step n
// has consumed those of step n) and its bead forces into the other of two buffers; the bead
// pass reads step n's bead forces, the force adjoints and adds into the population adjoint.
// The first n_cb workgroups couple (with the coupling's XCD pattern); each later workgroup
// runs the bead pass on its first wave.  FREE: the bead pass of the body passes, which takes
// the bead positions from the step's stored poses while the records hold step n-1's.
template <typename Real, bool FREE>
__global__ __launch_bounds__(kCoupleBlock) void couple_adj_bead_kernel(const StepArgs<Real> a,
                                                                      const CoupleArgs c,
                                                                      const AdjArgs<Real> A,
                                                                      int n_cb)
{
    __shared__ CoupleLds<Real> L;
    if ((int)blockIdx.x < n_cb) {
        couple_beads<Real>(a, c, blockIdx.x, n_cb, L);
        return;
    }
    if ((int)threadIdx.x < kAdjBeadBlock)
        adj_bead_lanes<Real, FREE>(A, ((int)blockIdx.x - n_cb) * kAdjBeadBlock + (int)threadIdx.x);
}

template <typename Real>
void launch_couple_adj_bead(const StepArgs<Real>& a, const CoupleArgs& c, const AdjArgs<Real>& A,
                            hipStream_t s)
{
    if (c.n_beads <= 0) return;
    const int n_cb = (c.n_beads * kBeadLanes + kCoupleBlock - 1) / kCoupleBlock;
    const int n_ab = (A.n_beads * kBeadLanes + kAdjBeadBlock - 1) / kAdjBeadBlock;
    if (A.body_adj)
        hipLaunchKernelGGL((couple_adj_bead_kernel<Real, true>), dim3(n_cb + n_ab),
                           dim3(kCoupleBlock), 0, s, a, c, A, n_cb);
    else
        hipLaunchKernelGGL((couple_adj_bead_kernel<Real, false>), dim3(n_cb + n_ab),
                           dim3(kCoupleBlock), 0, s, a, c, A, n_cb);
}

// pose of the coming step and its bead records, one workgroup per body
__global__ __launch_bounds__(256) void body_predict_kernel(const BodyArgs ba, int parity)
{
    __shared__ Pose next;
    Body& B = ba.bodies[blockIdx.x];
    if (threadIdx.x == 0) {
        predict_pose(B, B.pose[parity]);
        next = B.pose[parity];
    }
    __syncthreads();
    const RecConst C = rec_const(B);
    const int first = B.first_bead, n = B.n_beads;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const Bead bd = ba.beads[first + k];
        double r[3];
        write_bead_const(C, bd.user, ba.recs[first + k]);
        write_bead_pose(next, C.fixed != 0, bd.off, ba.recs[first + k], r);
    }
}

void launch_body_predict(const BodyArgs& b, int parity, hipStream_t s)
{
    if (b.n_bodies <= 0) return;
    hipLaunchKernelGGL(body_predict_kernel, dim3(b.n_bodies), dim3(256), 0, s, b, parity);
}

// the pose part of every bead record from a stored pose of its body, one thread per bead
__global__ __launch_bounds__(256) void records_from_poses_kernel(const Body* bodies, int par,
                                                                 const Bead* beads, BeadRec* recs,
                                                                 int n_beads)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n_beads) return;
    const Bead bd = beads[k];
    const Body& B = bodies[bd.body];
    double r[3];
    write_bead_pose(B.pose[par], B.fixed != 0, bd.off, recs[k], r);
}

void launch_records_from_poses(const Body* bodies, int par, const Bead* beads, BeadRec* recs,
                               int n_beads, hipStream_t s)
{
    if (n_beads <= 0) return;
    hipLaunchKernelGGL(records_from_poses_kernel, dim3((n_beads + 255) / 256), dim3(256), 0, s,
                       bodies, par, beads, recs, n_beads);
}

// finish every body after MD step k of the fluid step (one workgroup per body)
__global__ __launch_bounds__(256) void body_substep_kernel(const BodyArgs ba,
                                                           const int64_t* step_ptr,
                                                           int64_t step_arg, int k)
{
    const int64_t step = current_step(step_ptr, step_arg);
    body_finish(ba, blockIdx.x, (int)((step * ba.substeps + k) & 1));
}

void launch_body_substep(const BodyArgs& b, const int64_t* step_ptr, int64_t step_arg, int k,
                         hipStream_t s)
{
    if (b.n_bodies <= 0) return;
    hipLaunchKernelGGL(body_substep_kernel, dim3(b.n_bodies), dim3(256), 0, s, b, step_ptr,
                       step_arg, k);
}

__global__ void set_step_kernel(int64_t* p, int64_t v) { *p = v; }

void launch_set_step(int64_t* step_ptr, int64_t value, hipStream_t s)
{
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(1), 0, s, step_ptr, value);
}

// ------------------------------------------------------------------ initial state

template <typename Real>
__global__ __launch_bounds__(kNodeBlock) void init_equilibrium_kernel(
    Real* f, int64_t N, const ReplicaDesc* reps, const NodeTile* tiles, Real rho0, double ux,
    double uy, double uz)
{
    const NodeTile t = tiles[blockIdx.x];
    if ((int)threadIdx.x >= t.count) return;
    const ReplicaDesc R = reps[t.replica];
    const int64_t g = R.base + t.begin + threadIdx.x;
    const double r0 = (double)rho0, uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cu = cx_of(i) * ux + cy_of(i) * uy + cz_of(i) * uz;
        f[pop_at(i, g)] = (Real)(weight_of(i) * r0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
}

template <typename Real>
void launch_init_equilibrium(Real* f, int64_t N, const ReplicaDesc* reps, const NodeTile* tiles,
                             int32_t n_tiles, Real rho0, const double u0[3], hipStream_t s)
{
    if (n_tiles <= 0) return;
    hipLaunchKernelGGL((init_equilibrium_kernel<Real>), dim3(n_tiles), dim3(kNodeBlock), 0, s, f, N,
                       reps, tiles, rho0, u0[0], u0[1], u0[2]);
}

// ------------------------------------------------------------------ observables

template <typename Real, bool MASKED>
__global__ __launch_bounds__(kNodeBlock) void observe_kernel(const StepArgs<Real> a,
                                                             const NodeTile* tiles, Real* fields,
                                                             double* partials, double* pops)
{
    __shared__ double part[kNodeBlock / 64][5];
    const NodeTile t = tiles[blockIdx.x];
    const ReplicaDesc R = a.reps[t.replica];
    double acc[5] = {0, 0, 0, 0, 0};
    // holes are boundary nodes: zero fields and populations, not in the sums
    const bool node = (int)threadIdx.x < t.count &&
                      !(MASKED && R.masked == 2 && a.hole[R.base + t.begin + threadIdx.x] != 0);
    if (node) {
        const int64_t local = t.begin + threadIdx.x;
        int x, y, z;
        RowDesc self;
        locate<MASKED>(R, a.rows, t.row_lo, t.row_hi, local, x, y, z, self);
        Real d[Q];
        pull<Real, MASKED>(a.src, a.N, R, a.rowinfo, x, y, z, local, self, d);
        Real drho, j[3];
        density_momentum<Real>(d, drho, j);
        const int64_t dense = box_index(R, x, y, z);   // outputs in the box's own order
        if (fields) {
            const Real rho = a.cp.rho0 + drho;
            Real* o = fields + 4 * dense;
            o[0] = rho;
            for (int ax = 0; ax < 3; ++ax) o[1 + ax] = (j[ax] + (Real)0.5 * a.gext[ax]) / rho;
        }
        if (pops) {
            for (int i = 0; i < Q; ++i)
                pops[(int64_t)i * R.n_nodes + dense] = (double)d[i] + weight_of(i) * (double)a.cp.rho0;
        }
        acc[0] = (double)drho;
        acc[1] = (double)j[0]; acc[2] = (double)j[1]; acc[3] = (double)j[2];
        bool fin = isfinite((double)drho) && isfinite((double)j[0]) && isfinite((double)j[1]) &&
                   isfinite((double)j[2]);
        for (int i = 0; i < Q; ++i) fin = fin && isfinite((double)d[i]);
        acc[4] = fin ? 0.0 : 1.0;
    }
    if (!partials) return;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        for (int k = 0; k < 5; ++k) acc[k] += __shfl_down(acc[k], m, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 5; ++k) part[threadIdx.x >> 6][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k)
            partials[5 * (int64_t)blockIdx.x + k] = (part[0][k] + part[1][k]) + (part[2][k] + part[3][k]);
}

template <typename Real>
void launch_observe(const StepArgs<Real>& a, bool masked, int32_t tile0, int32_t n_tiles,
                    Real* fields, double* partials, double* pops_out, hipStream_t s)
{
    if (n_tiles <= 0) return;
    const NodeTile* tiles = a.tiles + tile0;
    if (masked)
        hipLaunchKernelGGL((observe_kernel<Real, true>), dim3(n_tiles), dim3(kNodeBlock), 0, s, a,
                           tiles, fields, partials, pops_out);
    else
        hipLaunchKernelGGL((observe_kernel<Real, false>), dim3(n_tiles), dim3(kNodeBlock), 0, s, a,
                           tiles, fields, partials, pops_out);
}

// explicit instantiations
template void launch_couple_adj_bead<float>(const StepArgs<float>&, const CoupleArgs&,
                                           const AdjArgs<float>&, hipStream_t);
template void launch_couple_adj_bead<double>(const StepArgs<double>&, const CoupleArgs&,
                                            const AdjArgs<double>&, hipStream_t);
template void launch_couple<float>(const StepArgs<float>&, const CoupleArgs&, hipStream_t,
                                   const LaunchEvents&, const BodyArgs*);
template void launch_couple<double>(const StepArgs<double>&, const CoupleArgs&, hipStream_t,
                                    const LaunchEvents&, const BodyArgs*);
template void launch_node_step<float>(const StepArgs<float>&, bool, bool, const BodyArgs*,
                                      hipStream_t, const LaunchEvents&);
template void launch_node_step<double>(const StepArgs<double>&, bool, bool, const BodyArgs*,
                                       hipStream_t, const LaunchEvents&);
template void launch_init_equilibrium<float>(float*, int64_t, const ReplicaDesc*, const NodeTile*,
                                             int32_t, float, const double*, hipStream_t);
template void launch_init_equilibrium<double>(double*, int64_t, const ReplicaDesc*,
                                              const NodeTile*, int32_t, double, const double*,
                                              hipStream_t);
template void launch_observe<float>(const StepArgs<float>&, bool, int32_t, int32_t, float*,
                                    double*, double*, hipStream_t);
template void launch_observe<double>(const StepArgs<double>&, bool, int32_t, int32_t, double*,
                                     double*, double*, hipStream_t);

}  // namespace lbrb
