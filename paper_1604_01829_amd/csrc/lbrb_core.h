// lbrb_core.h -- per-node and per-body arithmetic of the raspberry / lattice-Boltzmann step,
// shared by the gfx950 kernels (and compilable for the host so it can be unit-tested there).
//
// Lattice: D3Q19, velocities ordered rest; +-x; +-y; +-z; (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0);
// (1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1); (0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1), so that every odd
// index i has its opposite at i+1.  Weights 1/3, 1/18, 1/36.
//
// Collision (the multiple-relaxation-time scheme named in Sec. 1.1 of the paper): moments in
// the orthogonal D3Q19 basis of Duenweg, Schiller & Ladd; mass and momentum conserved (the
// momentum gains the force density); the bulk, shear, odd and even kinetic modes relax with
// their own rates towards the second-order equilibrium (kinetic modes towards zero); the
// force enters through u = (j + F/2)/rho and the second-moment source u F + F u with weight
// (1 + gamma_k)/2; thermal noise is added to every non-conserved mode with the
// fluctuation-dissipation amplitude sqrt(mu rho0 b_k (1 - gamma_k^2)), mu = kT/c_s^2.
// The forward transform is written on sums and differences of opposite populations, which
// halves the adds compared with a dense 19x19 product.
#ifndef LBRB_CORE_H
#define LBRB_CORE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#define LBRB_HD __host__ __device__ __forceinline__

namespace lbrb {

constexpr int Q = 19;

// velocity components of direction i (see the order above)
LBRB_HD int cx_of(int i)
{
    constexpr int t[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[i];
}
LBRB_HD int cy_of(int i)
{
    constexpr int t[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[i];
}
LBRB_HD int cz_of(int i)
{
    constexpr int t[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[i];
}
LBRB_HD int opposite_of(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// the direction with the x and z components of direction i exchanged
LBRB_HD int swap_xz_of(int i)
{
    constexpr int t[Q] = {0, 5, 6, 3, 4, 1, 2, 15, 16, 18, 17, 11, 12, 14, 13, 7, 8, 10, 9};
    return t[i];
}
LBRB_HD double weight_of(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror & Shaw (SC'11): ten rounds of two 32x32->64 products on counter
// words 0 and 2, a swap of the halves and a key xor; the key advances by two Weyl
// constants between rounds.
struct U4 { uint32_t x, y, z, w; };

LBRB_HD U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 16-bit integer h -> (2h + 1 - 2^16) / 2^17 in (-1/2, 1/2); exact in FP32 and FP64.
template <typename Real>
LBRB_HD Real uniform16(uint32_t h)
{
    return (Real)((int)(2u * (h & 0xFFFFu) + 1u) - 65536) * (Real)(1.0 / 131072.0);
}

// Noise counter layout: (step low word, index within the box, domain << 16 | block,
// step high word); key = the box's 64-bit seed.  Domain 0 = fluid nodes (two blocks per
// node give 16 half-words; modes 4..18 use half-words 0..14), domain 1 = beads (one block,
// half-words 0..2 for x, y, z).
LBRB_HD U4 noise_block(uint64_t step, uint32_t index, uint32_t domain, uint32_t block,
                       uint32_t k0, uint32_t k1)
{
    U4 c;
    c.x = (uint32_t)step;
    c.y = index;
    c.z = (domain << 16) | block;
    c.w = (uint32_t)(step >> 32);
    return philox4x32_10(c, k0, k1);
}

// ------------------------------------------------------------------ collision
// Per-precision constants of one relaxation setting, filled on the host.
template <typename Real>
struct CollideParams {
    Real rho0;
    Real g_bulk, g_shear, g_odd, g_even;     // gamma_k = 1 - 1/tau_k
    Real h_bulk, h_shear;                     // (1 + gamma_k) / 2 for the force source
    Real a_noise[Q];                          // sqrt(12 mu rho0 b_k (1 - gamma_k^2)), k >= 4
};

// One node: d[i] = f_i - w_i rho0 (pre-collision, shifted) in, post-collision shifted out.
// F = force density on the node.  U = 15 uniforms in (-1/2,1/2) for modes 4..18, or null.
template <typename Real>
LBRB_HD void collide(const CollideParams<Real>& P, Real d[Q], const Real F[3], const Real* U)
{
    // sums and differences of opposite pairs
    const Real sx = d[1] + d[2], dx = d[1] - d[2];
    const Real sy = d[3] + d[4], dy = d[3] - d[4];
    const Real sz = d[5] + d[6], dz = d[5] - d[6];
    const Real s7 = d[7] + d[8], d7 = d[7] - d[8];
    const Real s9 = d[9] + d[10], d9 = d[9] - d[10];
    const Real s11 = d[11] + d[12], d11 = d[11] - d[12];
    const Real s13 = d[13] + d[14], d13 = d[13] - d[14];
    const Real s15 = d[15] + d[16], d15 = d[15] - d[16];
    const Real s17 = d[17] + d[18], d17 = d[17] - d[18];

    const Real sax = sx + sy + sz;                    // axis pairs
    const Real sxy = s7 + s9, sxz = s11 + s13, syz = s15 + s17;
    const Real sdg = sxy + sxz + syz;                 // diagonal pairs

    // conserved modes (the shift w_i rho0 only enters mode 0)
    const Real drho = d[0] + sax + sdg;
    const Real jx = dx + d7 + d9 + d11 + d13;
    const Real jy = dy + d7 - d9 + d15 + d17;
    const Real jz = dz + d11 - d13 + d15 - d17;

    // non-conserved modes 4..18
    Real m[Q];
    m[4] = sdg - d[0];
    m[5] = (Real)2 * sx - sy - sz + sxy + sxz - (Real)2 * syz;
    m[6] = sy - sz + sxy - sxz;
    m[7] = s7 - s9;
    m[8] = s15 - s17;
    m[9] = s11 - s13;
    m[10] = d7 + d9 + d11 + d13 - (Real)2 * dx;
    m[11] = d7 - d9 + d15 + d17 - (Real)2 * dy;
    m[12] = d11 - d13 + d15 - d17 - (Real)2 * dz;
    m[13] = d7 + d9 - d11 - d13;
    m[14] = d9 - d7 + d15 + d17;
    m[15] = d11 - d13 - d15 + d17;
    m[16] = d[0] - (Real)2 * sax + sdg;
    m[17] = sy + sz - (Real)2 * sx + sxy + sxz - (Real)2 * syz;
    m[18] = sz - sy + sxy - sxz;

    const Real rho = P.rho0 + drho;
    const Real irho = (Real)1 / rho;
    const Real ux = (jx + (Real)0.5 * F[0]) * irho;
    const Real uy = (jy + (Real)0.5 * F[1]) * irho;
    const Real uz = (jz + (Real)0.5 * F[2]) * irho;

    // equilibrium of the stress modes and the force source
    const Real e4 = rho * (ux * ux + uy * uy + uz * uz);
    const Real e5 = rho * ((Real)2 * ux * ux - uy * uy - uz * uz);
    const Real e6 = rho * (uy * uy - uz * uz);
    const Real e7 = rho * ux * uy, e8 = rho * uy * uz, e9 = rho * uz * ux;
    const Real S4 = (Real)2 * (ux * F[0] + uy * F[1] + uz * F[2]);
    const Real S5 = (Real)2 * ((Real)2 * ux * F[0] - uy * F[1] - uz * F[2]);
    const Real S6 = (Real)2 * (uy * F[1] - uz * F[2]);
    const Real S7 = ux * F[1] + uy * F[0];
    const Real S8 = uy * F[2] + uz * F[1];
    const Real S9 = uz * F[0] + ux * F[2];

    m[4] = e4 + P.g_bulk * (m[4] - e4) + P.h_bulk * S4;
    m[5] = e5 + P.g_shear * (m[5] - e5) + P.h_shear * S5;
    m[6] = e6 + P.g_shear * (m[6] - e6) + P.h_shear * S6;
    m[7] = e7 + P.g_shear * (m[7] - e7) + P.h_shear * S7;
    m[8] = e8 + P.g_shear * (m[8] - e8) + P.h_shear * S8;
    m[9] = e9 + P.g_shear * (m[9] - e9) + P.h_shear * S9;
#pragma unroll
    for (int k = 10; k < 16; ++k) m[k] *= P.g_odd;
#pragma unroll
    for (int k = 16; k < 19; ++k) m[k] *= P.g_even;
    if (U) {
#pragma unroll
        for (int k = 4; k < 19; ++k) m[k] += P.a_noise[k] * U[k - 4];
    }

    // back to populations: f_i = w_i sum_k e_k(c_i) m_k / b_k, shifted by w_i rho0
    const Real a0 = drho;
    const Real a1 = (Real)3 * (jx + F[0]), a2 = (Real)3 * (jy + F[1]), a3 = (Real)3 * (jz + F[2]);
    const Real a4 = (Real)1.5 * m[4], a5 = (Real)0.75 * m[5], a6 = (Real)2.25 * m[6];
    const Real a7 = (Real)9 * m[7], a8 = (Real)9 * m[8], a9 = (Real)9 * m[9];
    const Real a10 = (Real)1.5 * m[10], a11 = (Real)1.5 * m[11], a12 = (Real)1.5 * m[12];
    const Real a13 = (Real)4.5 * m[13], a14 = (Real)4.5 * m[14], a15 = (Real)4.5 * m[15];
    const Real a16 = (Real)0.5 * m[16], a17 = (Real)0.75 * m[17], a18 = (Real)2.25 * m[18];

    const Real w0 = (Real)(1.0 / 3.0), w1 = (Real)(1.0 / 18.0), w2 = (Real)(1.0 / 36.0);
    d[0] = w0 * (a0 - a4 + a16);
    {
        const Real e = a0 + (Real)2 * a5 - (Real)2 * a16 - (Real)2 * a17;
        const Real o = a1 - (Real)2 * a10;
        d[1] = w1 * (e + o); d[2] = w1 * (e - o);
    }
    {
        const Real e = a0 - a5 + a6 - (Real)2 * a16 + a17 - a18;
        const Real o = a2 - (Real)2 * a11;
        d[3] = w1 * (e + o); d[4] = w1 * (e - o);
    }
    {
        const Real e = a0 - a5 - a6 - (Real)2 * a16 + a17 + a18;
        const Real o = a3 - (Real)2 * a12;
        d[5] = w1 * (e + o); d[6] = w1 * (e - o);
    }
    const Real exy = a0 + a4 + a5 + a6 + a16 + a17 + a18;   // common part of the xy pairs
    const Real exz = a0 + a4 + a5 - a6 + a16 + a17 - a18;   // xz pairs
    const Real eyz = a0 + a4 - (Real)2 * a5 + a16 - (Real)2 * a17;  // yz pairs
    {
        const Real e = exy + a7, o = a1 + a2 + a10 + a11 + a13 - a14;
        d[7] = w2 * (e + o); d[8] = w2 * (e - o);
    }
    {
        const Real e = exy - a7, o = a1 - a2 + a10 - a11 + a13 + a14;
        d[9] = w2 * (e + o); d[10] = w2 * (e - o);
    }
    {
        const Real e = exz + a9, o = a1 + a3 + a10 + a12 - a13 + a15;
        d[11] = w2 * (e + o); d[12] = w2 * (e - o);
    }
    {
        const Real e = exz - a9, o = a1 - a3 + a10 - a12 - a13 - a15;
        d[13] = w2 * (e + o); d[14] = w2 * (e - o);
    }
    {
        const Real e = eyz + a8, o = a2 + a3 + a11 + a12 + a14 - a15;
        d[15] = w2 * (e + o); d[16] = w2 * (e - o);
    }
    {
        const Real e = eyz - a8, o = a2 - a3 + a11 - a12 + a14 + a15;
        d[17] = w2 * (e + o); d[18] = w2 * (e - o);
    }
}

// ------------------------------------------------------------------ collision adjoint
// Orthogonal basis vector e_k at velocity c_i and its norm b_k = sum_i w_i e_k(c_i)^2.
LBRB_HD double basis_e(int k, int i)
{
    const double cx = cx_of(i), cy = cy_of(i), cz = cz_of(i), c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0: return 1.0;
    case 1: return cx;
    case 2: return cy;
    case 3: return cz;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * cx * cx - c2;
    case 6: return cy * cy - cz * cz;
    case 7: return cx * cy;
    case 8: return cy * cz;
    case 9: return cz * cx;
    case 10: return (3.0 * c2 - 5.0) * cx;
    case 11: return (3.0 * c2 - 5.0) * cy;
    case 12: return (3.0 * c2 - 5.0) * cz;
    case 13: return (cy * cy - cz * cz) * cx;
    case 14: return (cz * cz - cx * cx) * cy;
    case 15: return (cx * cx - cy * cy) * cz;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * cx * cx - c2);
    default: return (2.0 * c2 - 3.0) * (cy * cy - cz * cz);
    }
}
LBRB_HD double basis_b(int k)
{
    constexpr double b[Q] = {1.0, 1.0 / 3, 1.0 / 3, 1.0 / 3, 2.0 / 3, 4.0 / 3, 4.0 / 9, 1.0 / 9,
                             1.0 / 9, 1.0 / 9, 2.0 / 3, 2.0 / 3, 2.0 / 3, 2.0 / 9, 2.0 / 9, 2.0 / 9,
                             2.0, 4.0 / 3, 4.0 / 9};
    return b[k];
}

// Vector-Jacobian product of the deterministic collision: given lam (adjoint of the
// post-collision populations) return the adjoints of the pre-collision populations (in lam,
// overwritten) and of the force density (lamF).  d: shifted pre-collision populations.
// The derivative runs backwards through: back-transform, relaxation towards the equilibrium
// of (rho, u) plus the force source, u = (j + F/2)/rho, and the forward transform.
template <typename Real>
LBRB_HD void collide_vjp(const CollideParams<Real>& P, const Real d[Q], const Real F[3], Real lam[Q],
                         Real lamF[3])
{
    Real m[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        Real acc = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) acc += (Real)basis_e(k, i) * d[i];
        m[k] = acc;
    }
    const Real rho = P.rho0 + m[0];
    const Real u[3] = {(m[1] + (Real)0.5 * F[0]) / rho, (m[2] + (Real)0.5 * F[1]) / rho,
                       (m[3] + (Real)0.5 * F[2]) / rho};
    const Real ux = u[0], uy = u[1], uz = u[2];
    Real ls[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        Real acc = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) acc += (Real)(basis_e(k, i) * weight_of(i)) * lam[i];
        ls[k] = acc * (Real)(1.0 / basis_b(k));
    }
    Real lm[Q];
    lm[0] = ls[0];
    Real lrho = 0, lu[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) { lm[1 + a] = ls[1 + a]; lamF[a] = ls[1 + a]; }
    // relaxation rates per mode
#pragma unroll
    for (int k = 4; k < Q; ++k) {
        const Real g = k == 4 ? P.g_bulk : (k <= 9 ? P.g_shear : (k <= 15 ? P.g_odd : P.g_even));
        lm[k] = g * ls[k];
    }
    // stress modes: equilibrium (via rho and u) and force source (via u and F)
    const Real Ab = ((Real)1 - P.g_bulk) * ls[4], Bb = P.h_bulk * ls[4];
    Real A[10], B[10];
    for (int k = 5; k <= 9; ++k) { A[k] = ((Real)1 - P.g_shear) * ls[k]; B[k] = P.h_shear * ls[k]; }
    // k = 4: e = rho u.u, S = 2 u.F
    lrho += Ab * (ux * ux + uy * uy + uz * uz);
    for (int a = 0; a < 3; ++a) { lu[a] += Ab * (Real)2 * rho * u[a] + Bb * (Real)2 * F[a]; lamF[a] += Bb * (Real)2 * u[a]; }
    // k = 5: e = rho (2ux^2 - uy^2 - uz^2), S = 2 (2 ux Fx - uy Fy - uz Fz)
    lrho += A[5] * ((Real)2 * ux * ux - uy * uy - uz * uz);
    lu[0] += A[5] * (Real)4 * rho * ux + B[5] * (Real)4 * F[0];
    lu[1] -= A[5] * (Real)2 * rho * uy + B[5] * (Real)2 * F[1];
    lu[2] -= A[5] * (Real)2 * rho * uz + B[5] * (Real)2 * F[2];
    lamF[0] += B[5] * (Real)4 * ux; lamF[1] -= B[5] * (Real)2 * uy; lamF[2] -= B[5] * (Real)2 * uz;
    // k = 6: e = rho (uy^2 - uz^2), S = 2 (uy Fy - uz Fz)
    lrho += A[6] * (uy * uy - uz * uz);
    lu[1] += A[6] * (Real)2 * rho * uy + B[6] * (Real)2 * F[1];
    lu[2] -= A[6] * (Real)2 * rho * uz + B[6] * (Real)2 * F[2];
    lamF[1] += B[6] * (Real)2 * uy; lamF[2] -= B[6] * (Real)2 * uz;
    // k = 7: e = rho ux uy, S = ux Fy + uy Fx
    lrho += A[7] * ux * uy;
    lu[0] += A[7] * rho * uy + B[7] * F[1]; lu[1] += A[7] * rho * ux + B[7] * F[0];
    lamF[0] += B[7] * uy; lamF[1] += B[7] * ux;
    // k = 8: e = rho uy uz, S = uy Fz + uz Fy
    lrho += A[8] * uy * uz;
    lu[1] += A[8] * rho * uz + B[8] * F[2]; lu[2] += A[8] * rho * uy + B[8] * F[1];
    lamF[1] += B[8] * uz; lamF[2] += B[8] * uy;
    // k = 9: e = rho uz ux, S = uz Fx + ux Fz
    lrho += A[9] * uz * ux;
    lu[0] += A[9] * rho * uz + B[9] * F[2]; lu[2] += A[9] * rho * ux + B[9] * F[0];
    lamF[0] += B[9] * uz; lamF[2] += B[9] * ux;
    // u = (j + F/2) / rho
    const Real irho = (Real)1 / rho;
    for (int a = 0; a < 3; ++a) {
        lm[1 + a] += lu[a] * irho;
        lamF[a] += (Real)0.5 * lu[a] * irho;
        lrho -= lu[a] * u[a] * irho;
    }
    lm[0] += lrho;
    // m = E f
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        Real acc = 0;
#pragma unroll
        for (int k = 0; k < Q; ++k) acc += (Real)basis_e(k, i) * lm[k];
        lam[i] = acc;
    }
}

// density and momentum of shifted populations
template <typename Real>
LBRB_HD void density_momentum(const Real d[Q], Real& drho, Real j[3])
{
    Real r = 0, x = 0, y = 0, z = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        r += d[i];
        x += (Real)cx_of(i) * d[i];
        y += (Real)cy_of(i) * d[i];
        z += (Real)cz_of(i) * d[i];
    }
    drho = r; j[0] = x; j[1] = y; j[2] = z;
}

// ------------------------------------------------------------------ rigid bodies (FP64)
// Pose of a body for one step: its state after the first half kick, the drift and the
// rotation, with the rotation matrix and the lab-frame angular velocity.
struct Pose {
    double pos[3], quat[4], vel[3], omega[3];
    double rot[9];
    double omega_lab[3];
};

// Geometry of the replica a body lives in, copied into the body record so that the
// coupling reaches it without another dependent load.
struct BodyBox {
    int32_t nx, ny, nz, masked;      // the box's own sides (not the storage's)
    int64_t base;                    // global index of the replica's local node 0
    int32_t row_base;
    uint32_t key0, key1;             // Philox key of the replica
    int32_t swap;                    // the replica is stored with axes x and z exchanged
};

struct Body {
    double pos[3], quat[4], vel[3], omega[3];
    double force[3], torque[3];      // last MD step's sum (lab) and body-frame torque
    double mass, inertia[3], gamma;
    double noise_amp;                // sqrt(2 kT gamma / dt) sqrt(12): bead noise per uniform
    double dt;                       // MD step in fluid steps (1 / MD steps per fluid step)
    double ev_radius;                // Lennard-Jones radius of the excluded-volume sites
    double ev_reach;                 // largest |offset| of those sites
    int32_t first_ev, n_ev;          // excluded-volume site range
    int32_t fixed, replica;
    int32_t first_bead, n_beads;     // global bead range
    int32_t first_bead_in_replica;   // index of the first bead within its replica
    int32_t pad;
    BodyBox box;
    Pose pose[2];                    // the pose used by MD step S (counted over the run) is
                                     // pose[S & 1]
};

LBRB_HD void quat_to_matrix(const double q[4], double m[3][3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    m[0][0] = 1.0 - 2.0 * (y * y + z * z);
    m[0][1] = 2.0 * (x * y - w * z);
    m[0][2] = 2.0 * (x * z + w * y);
    m[1][0] = 2.0 * (x * y + w * z);
    m[1][1] = 1.0 - 2.0 * (x * x + z * z);
    m[1][2] = 2.0 * (y * z - w * x);
    m[2][0] = 2.0 * (x * z - w * y);
    m[2][1] = 2.0 * (y * z + w * x);
    m[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

// half kick of the angular velocity with a body-frame torque over an MD step dt: Euler's
// equations, explicit
LBRB_HD void half_kick(double omega[3], const double inertia[3], const double torque_b[3],
                       double dt)
{
    const double Lx = inertia[0] * omega[0], Ly = inertia[1] * omega[1], Lz = inertia[2] * omega[2];
    const double cxw = omega[1] * Lz - omega[2] * Ly;
    const double cyw = omega[2] * Lx - omega[0] * Lz;
    const double czw = omega[0] * Ly - omega[1] * Lx;
    const double hh = 0.5 * dt;
    omega[0] += hh * (torque_b[0] - cxw) / inertia[0];
    omega[1] += hh * (torque_b[1] - cyw) / inertia[1];
    omega[2] += hh * (torque_b[2] - czw) / inertia[2];
}

// First half of an MD step dt for a free body: V += dt F/(2M), omega half kick,
// R += dt V, q <- q (x) (cos(dt|w|/2), sin(dt|w|/2) w/|w|), renormalised.  Inputs: the state
// after the previous step (pos0, quat0, vel0, omega0) and that step's force and body-frame
// torque; outputs may not alias them.
LBRB_HD void first_half(const double pos0[3], const double quat0[4], const double vel0[3],
                        const double omega0[3], const double force[3], const double torque[3],
                        double mass, const double inertia[3], double dt, bool fixed,
                        double pos[3], double quat[4], double vel[3], double omega[3])
{
    for (int a = 0; a < 3; ++a) { pos[a] = pos0[a]; vel[a] = vel0[a]; omega[a] = omega0[a]; }
    for (int a = 0; a < 4; ++a) quat[a] = quat0[a];
    if (fixed) return;
    const double hh = 0.5 * dt;
    for (int a = 0; a < 3; ++a) vel[a] += hh * force[a] / mass;
    half_kick(omega, inertia, torque, dt);
    for (int a = 0; a < 3; ++a) pos[a] += dt * vel[a];
    const double wn = sqrt(omega[0] * omega[0] + omega[1] * omega[1] + omega[2] * omega[2]);
    if (wn > 0.0) {
        const double h = hh * wn, s = sin(h) / wn, c = cos(h);
        const double p[4] = {c, s * omega[0], s * omega[1], s * omega[2]};
        const double* q = quat;
        double n[4];
        n[0] = q[0] * p[0] - q[1] * p[1] - q[2] * p[2] - q[3] * p[3];
        n[1] = q[0] * p[1] + q[1] * p[0] + q[2] * p[3] - q[3] * p[2];
        n[2] = q[0] * p[2] - q[1] * p[3] + q[2] * p[0] + q[3] * p[1];
        n[3] = q[0] * p[3] + q[1] * p[2] - q[2] * p[1] + q[3] * p[0];
        const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2] + n[3] * n[3]);
        for (int a = 0; a < 4; ++a) quat[a] = n[a] / nn;
    }
}

// rotation matrix and lab-frame angular velocity of a pose whose quaternion and body-frame
// angular velocity are set
LBRB_HD void complete_pose(Pose& p)
{
    double m[3][3];
    quat_to_matrix(p.quat, m);
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) p.rot[3 * r + k] = m[r][k];
        p.omega_lab[r] = m[r][0] * p.omega[0] + m[r][1] * p.omega[1] + m[r][2] * p.omega[2];
    }
}

// Fill a pose from the state of a body (the first half of a step).
LBRB_HD void predict_pose(const Body& b, Pose& p)
{
    first_half(b.pos, b.quat, b.vel, b.omega, b.force, b.torque, b.mass, b.inertia, b.dt,
               b.fixed != 0, p.pos, p.quat, p.vel, p.omega);
    complete_pose(p);
}

}  // namespace lbrb

#endif
