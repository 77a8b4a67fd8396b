// lbrb_construct.hip -- raspberry construction by constrained relaxation (rb_relax_shells).
//
// Sec. 2.1 and its SI: the beads of a shell are spread evenly over an ellipsoid
// x^2/a^2 + y^2/b^2 + z^2/c^2 = 1 by damped MD under a WCA repulsion between beads and a
// harmonic restraint U = k |r - r_s|^2 towards the closest surface point r_s.  From the
// normal condition r - r_s = (t/2) grad S(r_s), x_s = x a^2 / (t + a^2) per axis, and the
// surface equation becomes F(t) = sum (x a / (t + a^2))^2 - 1 = 0, decreasing in t on
// (-min a^2, inf), solved by bisection.
//
// One workgroup of 1024 threads per shell: the shell's positions live in LDS for the whole
// launch, each thread owns up to kPer beads (their velocities in registers), and a step is
// "forces from the LDS positions, barrier, kick and drift, barrier" -- no grid-wide
// synchronisation.  Sixteen wavefronts per shell keep the LDS reads of the pair loop in
// flight.  Up to kShellsPerLaunch shells go in one launch as a by-value argument.
//
// Pairs: a Verlet list per bead (the beads within the cut plus a skin, in ascending index
// order, in LDS), rebuilt once any bead has moved more than half the skin since the last
// build.  Walking the list in order adds exactly the nonzero pair terms of the all-pairs loop
// in the same order, so the WCA sums are the all-pairs sums bit for bit.  The list capacity
// per bead is the shell's share of kNbSlots (24 for 2048 beads, 90 for 543: thin oblate
// shells have beads of both faces within the list radius); a bead with more candidates walks
// all pairs.  Closest point: Newton on a nearly linear transform of
// F(t) inside the shrinking bisection bracket, started from the bead's parameter of the
// previous step (one to three iterations where the bisection took about sixty).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "../../include/lbrb.h"

namespace {

constexpr int kBlock = 1024;
constexpr int kMaxBeads = 2048;                 // per shell (48 KB of LDS)
constexpr int kPer = kMaxBeads / kBlock;        // beads per thread
constexpr int kShellsPerLaunch = 64;
constexpr int kNbSlots = kMaxBeads * 24;        // list entries per shell (96 KB of LDS)
constexpr int kNbMax = 128;                     // list capacity per bead at most
constexpr double kSkin = 0.4;                   // list radius: the WCA cut plus kSkin

struct Shell {
    double axes[3];
    int32_t first, count;
};
struct ShellBatch {
    Shell s[kShellsPerLaunch];
};
struct RelaxArgs {
    double k2;          // 2 k
    double s2, rc2;     // sigma^2, (2^(1/6) sigma)^2
    double eps24;       // 24 eps
    double dt, m;
    double g;           // eta dt / 2
};

// closest point of the ellipsoid (semi-axes a, squares a2) to x: the root of F(t) on
// (-min a^2, max a |x| + 1], F decreasing there.  S = F + 1 is a sum of c_k / (t + a_k^2)^2,
// so G = 1/sqrt(S) - 1 is nearly linear in t (linear on a sphere): Newton on G from t (the
// previous step's root), inside the bracket that every evaluation shrinks; a step that leaves
// the bracket becomes the midpoint.  It stops once a step is within the rounding noise of
// S (64 ulp of max a^2 in t; S itself carries a relative error near 1e-16).  t returns the
// root.
__device__ void closest(const double a[3], const double a2[3], double amin2, double amax,
                        const double x[3], double& t, double rs[3])
{
    double lo = -amin2;
    double hi = amax * sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) + 1.0;
    const double tol = 64.0 * DBL_EPSILON * (amax * amax);
    if (!(t > lo && t < hi)) t = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        double S = 0.0, dS = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double ir = 1.0 / (t + a2[k]);
            const double v = x[k] * a[k] * ir;
            S += v * v;
            dS -= 2.0 * v * v * ir;
        }
        if (S == 1.0) break;
        if (S > 1.0) lo = t;
        else hi = t;
        const double rsq = 1.0 / sqrt(S);
        double tn = t + 2.0 * (rsq - 1.0) * S / (rsq * dS);
        if (!(fabs(tn - t) > tol)) {
            if (tn > lo && tn < hi) t = tn;
            break;
        }
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (!(tn > lo && tn < hi)) break;
        t = tn;
    }
    for (int k = 0; k < 3; ++k) rs[k] = x[k] * a2[k] / (t + a2[k]);
}

// WCA force of the pair (i, j) on i, added to f (nothing at or beyond the cut)
__device__ __forceinline__ void pair_force(const double xi[3], const double (*X)[3], int j,
                                           const RelaxArgs& p, double f[3])
{
    const double d[3] = {xi[0] - X[j][0], xi[1] - X[j][1], xi[2] - X[j][2]};
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(r2 < p.rc2)) return;
    const double ir2 = 1.0 / r2;
    const double u = p.s2 * ir2, u6 = u * u * u;
    const double coef = p.eps24 * (2.0 * u6 * u6 - u6) * ir2;
    for (int k = 0; k < 3; ++k) f[k] += coef * d[k];
}

__global__ __launch_bounds__(kBlock) void relax_kernel(const ShellBatch B, double* pos,
                                                       double* vel, const RelaxArgs p,
                                                       int n_steps)
{
    __shared__ double X[kMaxBeads][3];
    __shared__ uint16_t nb[kNbSlots];
    const Shell S = B.s[blockIdx.x];
    const int n = S.count;
    double a[3], a2[3], amin2 = INFINITY, amax = 0.0;
    for (int k = 0; k < 3; ++k) {
        a[k] = S.axes[k];
        a2[k] = a[k] * a[k];
        amin2 = fmin(amin2, a2[k]);
        amax = fmax(amax, a[k]);
    }
    const int cap = min(kNbMax, kNbSlots / max(n, 1));   // list entries per bead
    const double rl = sqrt(p.rc2) + kSkin, rl2 = rl * rl;
    const double move2 = 0.25 * kSkin * kSkin;       // (skin / 2)^2
    double* P = pos + 3 * (int64_t)S.first;
    double* V = vel + 3 * (int64_t)S.first;
    double v[kPer][3], xb[kPer][3], t[kPer];
    int cnt[kPer];                                   // list length; cap + 1: walk all pairs
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int i = threadIdx.x + q * kBlock;
        t[q] = 0.0;
        cnt[q] = 0;
        for (int k = 0; k < 3; ++k) {
            v[q][k] = i < n ? V[3 * i + k] : 0.0;
            xb[q][k] = 0.0;
            if (i < n) X[i][k] = P[3 * i + k];
        }
    }
    __syncthreads();
    bool rebuild = true;
    for (int step = 0; step < n_steps; ++step) {
        if (rebuild) {
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int i = threadIdx.x + q * kBlock;
                if (i >= n) continue;
                const double xi[3] = {X[i][0], X[i][1], X[i][2]};
                int c = 0;
                for (int j = 0; j < n; ++j) {
                    if (j == i) continue;
                    const double d0 = xi[0] - X[j][0], d1 = xi[1] - X[j][1], d2 = xi[2] - X[j][2];
                    if (!(d0 * d0 + d1 * d1 + d2 * d2 < rl2)) continue;
                    if (c < cap) nb[i * cap + c] = (uint16_t)j;
                    ++c;
                }
                cnt[q] = c <= cap ? c : cap + 1;
                for (int k = 0; k < 3; ++k) xb[q][k] = xi[k];
            }
        }
        double f[kPer][3];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int i = threadIdx.x + q * kBlock;
            f[q][0] = f[q][1] = f[q][2] = 0.0;
            if (i >= n) continue;
            const double xi[3] = {X[i][0], X[i][1], X[i][2]};
            if (cnt[q] <= cap) {
                for (int m = 0; m < cnt[q]; ++m) pair_force(xi, X, nb[i * cap + m], p, f[q]);
            } else {
                for (int j = 0; j < n; ++j)
                    if (j != i) pair_force(xi, X, j, p, f[q]);
            }
            double rs[3];
            closest(a, a2, amin2, amax, xi, t[q], rs);
            for (int k = 0; k < 3; ++k) f[q][k] -= p.k2 * (xi[k] - rs[k]);
        }
        __syncthreads();
        bool moved = false;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int i = threadIdx.x + q * kBlock;
            if (i >= n) continue;
            double dd = 0.0;
            for (int k = 0; k < 3; ++k) {
                v[q][k] = ((1.0 - p.g) * v[q][k] + p.dt * f[q][k] / p.m) / (1.0 + p.g);
                X[i][k] += p.dt * v[q][k];
                const double e = X[i][k] - xb[q][k];
                dd += e * e;
            }
            moved = moved || !(dd <= move2);
        }
        rebuild = __syncthreads_or(moved) != 0;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int i = threadIdx.x + q * kBlock;
        if (i >= n) continue;
        for (int k = 0; k < 3; ++k) {
            P[3 * i + k] = X[i][k];
            V[3 * i + k] = v[q][k];
        }
    }
}

}  // namespace

extern "C" int rb_relax_shells(int32_t n_shells, const double* axes, const int32_t* counts,
                               double* dev_pos, double* dev_vel, const rb_relax_params* prm,
                               int32_t n_steps, void* stream)
{
    if (n_shells < 1 || !axes || !counts || !dev_pos || !dev_vel || !prm || n_steps < 0)
        return LB_ERR_ARG;
    const rb_relax_params& q = *prm;
    if (!(q.dt > 0.0) || !(q.mass > 0.0) || !(q.sigma > 0.0) || !(q.epsilon >= 0.0) ||
        !(q.k_surface >= 0.0) || !(q.damping >= 0.0) || !std::isfinite(q.dt) ||
        !std::isfinite(q.mass) || !std::isfinite(q.sigma) || !std::isfinite(q.epsilon) ||
        !std::isfinite(q.k_surface) || !std::isfinite(q.damping))
        return LB_ERR_ARG;
    for (int32_t s = 0; s < n_shells; ++s) {
        if (counts[s] < 1 || counts[s] > kMaxBeads) return LB_ERR_ARG;
        for (int k = 0; k < 3; ++k)
            if (!(axes[3 * s + k] > 0.0) || !std::isfinite(axes[3 * s + k])) return LB_ERR_ARG;
    }
    RelaxArgs p{};
    p.k2 = 2.0 * q.k_surface;
    p.s2 = q.sigma * q.sigma;
    p.rc2 = std::pow(2.0, 1.0 / 3.0) * q.sigma * q.sigma;
    p.eps24 = 24.0 * q.epsilon;
    p.dt = q.dt;
    p.m = q.mass;
    p.g = 0.5 * q.damping * q.dt;
    int64_t first = 0;
    for (int32_t s0 = 0; s0 < n_shells; s0 += kShellsPerLaunch) {
        ShellBatch B{};
        const int nb = std::min<int32_t>(kShellsPerLaunch, n_shells - s0);
        for (int k = 0; k < nb; ++k) {
            Shell& S = B.s[k];
            for (int a = 0; a < 3; ++a) S.axes[a] = axes[3 * (s0 + k) + a];
            S.first = (int32_t)first;
            S.count = counts[s0 + k];
            first += counts[s0 + k];
        }
        if (first > INT32_MAX) return LB_ERR_ARG;
        if (n_steps > 0)
            hipLaunchKernelGGL(relax_kernel, dim3(nb), dim3(kBlock), 0, (hipStream_t)stream, B,
                               dev_pos, dev_vel, p, n_steps);
        if (hipGetLastError() != hipSuccess) return LB_ERR_HIP;
    }
    return LB_OK;
}
