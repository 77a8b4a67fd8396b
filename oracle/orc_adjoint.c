/*
 * orc_adjoint.c -- reverse-mode derivative of the step sequence, FP64, plain loops.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Objective over a window of T steps starting from the current state:
 *     J = sum_n sum_b  a(n, b) . F_b(n)
 * where F_b(n) is the summed bead force of body b in step n and a(n, b) are given weights
 * (a = (1/T, 0, 0) for every step gives the time-averaged drag along x).  Derivatives are
 * taken with respect to each body's bead friction gamma_b and each bead's body-frame offset.
 *
 * Scope: a deterministic or a thermal fluid (for kT > 0 the derivative is pathwise: the noise
 * draws of every step are those of the forward run, counter-based, and the bead noise
 * amplitude sqrt(2 kT gamma / h) is differentiated in gamma; the fluid's noise enters the
 * collision additively and leaves its Jacobian unchanged), one or several MD steps per fluid step (the MD
 * steps of a fluid step all read the same populations and each spreads -h times its bead
 * forces), WCA excluded volume (Sec. 2.1 inner layers, Sec. 2.3 pore beads); boundary masks
 * allowed; bodies fixed or free.  F_b(n) is the force of the last MD step of fluid step n
 * (the body force a fluid step leaves, excluded volume included).  The window's initial state (populations and
 * body states, including the force and torque of the step before the window) is held fixed.
 * The adjoint of one step is the transpose of each of its parts, taken in reverse order:
 *   streaming with halfway bounce-back  ->  lambda*_i(y) = lambda_i(y + c_i) if y + c_i is a
 *                                           fluid node, else lambda_opp(i)(y);
 *   collision f* = C(f, F)               ->  vector-Jacobian product of the mode-space collision
 *                                           (orc_collide_vjp below, pinned by finite differences);
 *   spreading g = -sum w F_k             ->  adjoint of F_k gets -sum_c w_c lambda_F(x_c);
 *   friction F_k = gamma u_k             ->  d gamma += lambda_Fk . u_k, lambda_uk = gamma lambda_Fk;
 *   interpolation u_k = sum w_c u(x_c)   ->  lambda_u(x_c) += w_c lambda_uk, and the position
 *                                           derivative of the weights;
 *   node velocity u = (j + g/2)/rho      ->  lambda_f_i += (c_i - u) . lambda_u / rho;
 * and for a free body (Sec. 1.2 virtual sites, Sec. 2.3 integrator) the transposes of
 *   bead kinematics r_k = R + Q(q) b_k, v_k = V + Q(q)(omega x b_k);
 *   force and torque sums F = sum F_k, tau = Q^T sum (r_k - R) x F_k;
 *   the second half kick V += h F/2M, omega += h (tau - omega x I omega) / 2I;
 *   the first half kick with the previous step's F and tau, the drift R += h V and the
 *   rotation q <- (q (x) (cos(h|w|/2), sin(h|w|/2) w/|w|)) / norm;
 * with the adjoint of the body state carried from step to step; and of the WCA pair forces
 * f(x_k - y_j) between a body's sites x_k = R + Q o_k and the static sites or the other
 * bodies' sites y_j, through the pair force's Jacobian
 *   df/dd = c I + 2 c' d d^T,  f = c(|d|^2) d,  c = 24 eps (2 s^12 - s^6)/|d|^2,  s = sigma/|d|,
 * to the positions and rotations of both bodies.  The rotation matrix is differentiated entry
 * by entry in the quaternion's components.
 * Every pre-collision state of the window is kept in memory (19 * N doubles per step), and
 * every body state before each fluid step; the reverse of a fluid step first recomputes its
 * MD steps (poses, bead forces, body states) from the state before it.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* accessors of the box defined in orc_lbrb.c */
int orc_box_dims(const orc_sim* s, int dims[3]);
const double* orc_box_f(const orc_sim* s);
void orc_box_set_f(orc_sim* s, const double* f);
const uint8_t* orc_box_mask(const orc_sim* s);
int orc_box_body(const orc_sim* s, int b, const double** offsets, int* n_beads, double pos[3],
                 double quat[4], double* gamma, int* fixed);
double orc_box_kT(const orc_sim* s);
int orc_box_md_steps(const orc_sim* s);
int orc_box_ev(const orc_sim* s, int b, const double** offsets, int* n, double* radius);
int orc_box_sites(const orc_sim* s, const double** pos, const double** radius, int* n);
int orc_box_bead_uniforms(const orc_sim* s, int64_t step, int bead, int k_md, double out[3]);
int orc_box_body_mass(const orc_sim* s, int b, double* mass, double inertia[3]);
int orc_box_first_half(const orc_sim* s, int b, const double state[19], double h, double out[13]);
int orc_box_second_half(const orc_sim* s, int b, const double in[19], double h, double out[19]);

/* the basis, its norms and the weights, read once into tables (the same values) */
static double AE[19][19], AB[19], AW[19];
static int tables_ready = 0;
static void adj_tables(void)
{
    if (tables_ready) return;
    for (int k = 0; k < 19; ++k) {
        AB[k] = orc_basis_norm(k);
        AW[k] = orc_weight(k);
        for (int i = 0; i < 19; ++i) AE[k][i] = orc_basis(k, i);
    }
    tables_ready = 1;
}

static double E_(int k, int i) { return AE[k][i]; }

void orc_collide_vjp(const orc_params* p, const double f_in[19], const double F[3],
                     const double lam_out[19], double lam_in[19], double lam_F[3])
{
    double m[19], b[19], w[19], lam_ms[19], lam_m[19];
    adj_tables();
    for (int k = 0; k < 19; ++k) {
        b[k] = AB[k];
        double acc = 0.0;
        for (int i = 0; i < 19; ++i) acc += E_(k, i) * f_in[i];
        m[k] = acc;
    }
    for (int i = 0; i < 19; ++i) w[i] = AW[i];
    const double rho = m[0];
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (m[1 + a] + 0.5 * F[a]) / rho;
    const double ux = u[0], uy = u[1], uz = u[2];
    const double meq[10] = {0, 0, 0, 0, rho * (ux * ux + uy * uy + uz * uz),
                            rho * (2 * ux * ux - uy * uy - uz * uz), rho * (uy * uy - uz * uz),
                            rho * ux * uy, rho * uy * uz, rho * uz * ux};
    /* back-transform f*_i = w_i sum_k e_ki m*_k / b_k: adjoint of m*_k */
    for (int k = 0; k < 19; ++k) {
        double acc = 0.0;
        for (int i = 0; i < 19; ++i) acc += E_(k, i) * w[i] * lam_out[i];
        lam_ms[k] = acc / b[k];
    }
    double lam_rho = 0.0, lam_u[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) lam_F[a] = 0.0;
    for (int k = 0; k < 19; ++k) lam_m[k] = 0.0;
    /* m*_0 = m_0 ; j* = j + F */
    lam_m[0] += lam_ms[0];
    for (int a = 0; a < 3; ++a) { lam_m[1 + a] += lam_ms[1 + a]; lam_F[a] += lam_ms[1 + a]; }
    /* m*_k = meq_k + g_k (m_k - meq_k) + (1+g_k)/2 S_k  (k = 4..9);  m*_k = g_k m_k (k >= 10) */
    for (int k = 4; k < 19; ++k) {
        double tau;
        if (k == 4) tau = p->tau_bulk;
        else if (k <= 9) tau = p->tau_shear;
        else if (k <= 15) tau = p->tau_odd;
        else tau = p->tau_even;
        const double g = 1.0 - 1.0 / tau;
        lam_m[k] += g * lam_ms[k];
        if (k > 9) continue;
        const double A = (1.0 - g) * lam_ms[k], B = 0.5 * (1.0 + g) * lam_ms[k];
        double de[3], dSu[3], dSF[3];
        switch (k) {
        case 4:
            de[0] = 2 * rho * ux; de[1] = 2 * rho * uy; de[2] = 2 * rho * uz;
            dSu[0] = 2 * F[0]; dSu[1] = 2 * F[1]; dSu[2] = 2 * F[2];
            dSF[0] = 2 * ux; dSF[1] = 2 * uy; dSF[2] = 2 * uz;
            break;
        case 5:
            de[0] = 4 * rho * ux; de[1] = -2 * rho * uy; de[2] = -2 * rho * uz;
            dSu[0] = 4 * F[0]; dSu[1] = -2 * F[1]; dSu[2] = -2 * F[2];
            dSF[0] = 4 * ux; dSF[1] = -2 * uy; dSF[2] = -2 * uz;
            break;
        case 6:
            de[0] = 0; de[1] = 2 * rho * uy; de[2] = -2 * rho * uz;
            dSu[0] = 0; dSu[1] = 2 * F[1]; dSu[2] = -2 * F[2];
            dSF[0] = 0; dSF[1] = 2 * uy; dSF[2] = -2 * uz;
            break;
        case 7:
            de[0] = rho * uy; de[1] = rho * ux; de[2] = 0;
            dSu[0] = F[1]; dSu[1] = F[0]; dSu[2] = 0;
            dSF[0] = uy; dSF[1] = ux; dSF[2] = 0;
            break;
        case 8:
            de[0] = 0; de[1] = rho * uz; de[2] = rho * uy;
            dSu[0] = 0; dSu[1] = F[2]; dSu[2] = F[1];
            dSF[0] = 0; dSF[1] = uz; dSF[2] = uy;
            break;
        default: /* 9 */
            de[0] = rho * uz; de[1] = 0; de[2] = rho * ux;
            dSu[0] = F[2]; dSu[1] = 0; dSu[2] = F[0];
            dSF[0] = uz; dSF[1] = 0; dSF[2] = ux;
            break;
        }
        lam_rho += A * meq[k] / rho;
        for (int a = 0; a < 3; ++a) {
            lam_u[a] += A * de[a] + B * dSu[a];
            lam_F[a] += B * dSF[a];
        }
    }
    /* u = (j + F/2) / rho */
    for (int a = 0; a < 3; ++a) {
        lam_m[1 + a] += lam_u[a] / rho;
        lam_F[a] += 0.5 * lam_u[a] / rho;
        lam_rho -= lam_u[a] * u[a] / rho;
    }
    lam_m[0] += lam_rho;
    /* m = E f */
    for (int i = 0; i < 19; ++i) {
        double acc = 0.0;
        for (int k = 0; k < 19; ++k) acc += E_(k, i) * lam_m[k];
        lam_in[i] = acc;
    }
}

/* rotation matrix body -> lab of a unit quaternion (w,x,y,z) */
static void rotmat(const double q[4], double m[3][3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    m[0][0] = 1 - 2 * (y * y + z * z); m[0][1] = 2 * (x * y - w * z); m[0][2] = 2 * (x * z + w * y);
    m[1][0] = 2 * (x * y + w * z); m[1][1] = 1 - 2 * (x * x + z * z); m[1][2] = 2 * (y * z - w * x);
    m[2][0] = 2 * (x * z - w * y); m[2][1] = 2 * (y * z + w * x); m[2][2] = 1 - 2 * (x * x + y * y);
}

static int wrapi(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }

/* velocity of a fluid node from pre-collision populations f (19*N, [i][node]) */
static void node_u(const double* f, int64_t N, int64_t x, const double gext[3], double* rho_out,
                   double u[3])
{
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < 19; ++i) {
        const double fi = f[i * N + x];
        rho += fi;
        for (int a = 0; a < 3; ++a) j[a] += orc_velocity(i, a) * fi;
    }
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * gext[a]) / rho;
    *rho_out = rho;
}

/* A(w) d = d x (I w) + w x (I d), the derivative of w x I w along d; out = A(w)^T m         */
static void euler_vjp(const double w[3], const double I[3], const double m[3], double out[3])
{
    const double Iw[3] = {I[0] * w[0], I[1] * w[1], I[2] * w[2]};
    double a[3], b[3];
    /* m . (d x Iw) = d . (Iw x m) */
    a[0] = Iw[1] * m[2] - Iw[2] * m[1];
    a[1] = Iw[2] * m[0] - Iw[0] * m[2];
    a[2] = Iw[0] * m[1] - Iw[1] * m[0];
    /* m . (w x I d) = (I d) . (m x w) */
    b[0] = m[1] * w[2] - m[2] * w[1];
    b[1] = m[2] * w[0] - m[0] * w[2];
    b[2] = m[0] * w[1] - m[1] * w[0];
    for (int k = 0; k < 3; ++k) out[k] = a[k] + I[k] * b[k];
}

static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* partial derivatives of the rotation matrix entries with respect to q = (w, x, y, z)      */
static void rotmat_partials(const double q[4], double d[4][3][3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double dw[3][3] = {{0, -2 * z, 2 * y}, {2 * z, 0, -2 * x}, {-2 * y, 2 * x, 0}};
    const double dx[3][3] = {{0, 2 * y, 2 * z}, {2 * y, -4 * x, -2 * w}, {2 * z, 2 * w, -4 * x}};
    const double dy[3][3] = {{-4 * y, 2 * x, 2 * w}, {2 * x, 0, 2 * z}, {-2 * w, 2 * z, -4 * y}};
    const double dz[3][3] = {{-4 * z, -2 * w, 2 * x}, {2 * w, -4 * z, 2 * y}, {2 * x, 2 * y, 0}};
    memcpy(d[0], dw, sizeof dw);
    memcpy(d[1], dx, sizeof dx);
    memcpy(d[2], dy, sizeof dy);
    memcpy(d[3], dz, sizeof dz);
}

/* WCA pair at separation d with sigma: adds the force on the first site to F; with J given,
 * also returns c and c' (the derivative of c with respect to |d|^2) in J[0], J[1]; returns 0
 * beyond the cutoff 2^(1/6) sigma (no force)                                               */
static int wca_pair_j(double eps, double sigma, const double d[3], double F[3], double J[2])
{
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(r2 < pow(2.0, 1.0 / 3.0) * sigma * sigma)) return 0;
    const double s2 = sigma * sigma / r2, s6 = s2 * s2 * s2, s12 = s6 * s6;
    const double c = 24.0 * eps * (2.0 * s12 - s6) / r2;
    for (int k = 0; k < 3; ++k) F[k] += c * d[k];
    if (J) {
        J[0] = c;
        J[1] = 24.0 * eps * (-14.0 * s12 + 4.0 * s6) / (r2 * r2);
    }
    return 1;
}

static void min_image3(const int dims[3], const double a[3], const double b[3], double d[3])
{
    for (int k = 0; k < 3; ++k) {
        d[k] = a[k] - b[k];
        d[k] -= dims[k] * round(d[k] / dims[k]);
    }
}

/* body layout of orc_body_state: pos 0, quat 3, vel 7, omega 10, force 13, torque 16       */
enum { S_POS = 0, S_QUAT = 3, S_VEL = 7, S_OM = 10, S_F = 13, S_T = 16, S_N = 19 };

/* lab position x and arm d = Q o of a site at body-frame offset o, pose P (centre, quaternion) */
static void site_of(const double* P, const double o[3], double d[3], double x[3])
{
    double R[3][3];
    rotmat(P + S_QUAT, R);
    for (int a = 0; a < 3; ++a) {
        d[a] = R[a][0] * o[0] + R[a][1] * o[1] + R[a][2] * o[2];
        x[a] = P[S_POS + a] + d[a];
    }
}

/* WCA force and lab torque on every body (6 per body) at the poses P (13 words per body):
 * each excluded-volume site of a body against the static sites and the other bodies' sites */
static void wca_forces(const orc_sim* s, double eps, const int dims[3], int n_bodies,
                       const double* P, double* out)
{
    const double *wpos, *wrad;
    int nw;
    orc_box_sites(s, &wpos, &wrad, &nw);
    for (int b = 0; b < 6 * n_bodies; ++b) out[b] = 0.0;
    if (!(eps > 0.0)) return;
    for (int b = 0; b < n_bodies; ++b) {
        const double* ob; int nb; double rb;
        orc_box_ev(s, b, &ob, &nb, &rb);
        for (int k = 0; k < nb; ++k) {
            double d[3], x[3], F[3] = {0, 0, 0}, dd[3];
            site_of(P + 13 * (size_t)b, ob + 3 * k, d, x);
            for (int w = 0; w < nw; ++w) {
                min_image3(dims, x, wpos + 3 * w, dd);
                wca_pair_j(eps, rb + wrad[w], dd, F, NULL);
            }
            for (int c = 0; c < n_bodies; ++c) {
                const double* oc; int nc; double rc;
                orc_box_ev(s, c, &oc, &nc, &rc);
                if (c == b) continue;
                for (int j = 0; j < nc; ++j) {
                    double dj[3], y[3];
                    site_of(P + 13 * (size_t)c, oc + 3 * j, dj, y);
                    min_image3(dims, x, y, dd);
                    wca_pair_j(eps, rb + rc, dd, F, NULL);
                }
            }
            double T[3];
            cross3(d, F, T);
            for (int a = 0; a < 3; ++a) { out[6 * b + a] += F[a]; out[6 * b + 3 + a] += T[a]; }
        }
    }
}

/* per-body adjoint words of one reverse MD step */
enum { RA_F = 0, RA_TB = 3, RA_TAU = 6, RA_VM = 9, RA_WM = 12, RA_RC = 15, RA_QC = 18, RA_Q = 22,
       RA_N = 31 };

int orc_adjoint(orc_sim* s, const orc_params* p, int n_steps, int n_bodies, const double* dJ_dF,
                double* J_out, double* dJ_dgamma, double* dJ_doffsets)
{
    int dims[3];
    orc_box_dims(s, dims);
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const int64_t N = (int64_t)nx * ny * nz;
    const uint8_t* mask = orc_box_mask(s);
    const int m = orc_box_md_steps(s);
    if (n_steps < 0) return -1;
    const double kT = orc_box_kT(s);
    const int64_t step0 = orc_step_count(s);
    const double h = 1.0 / m;   /* MD step */
    adj_tables();   /* before the parallel node loop */

    int total_beads = 0;
    for (int b = 0; b < n_bodies; ++b) {
        const double* off; int nb; double pos[3], q[4], gamma; int fixed;
        if (orc_box_body(s, b, &off, &nb, pos, q, &gamma, &fixed) != 0) return -1;
        total_beads += nb;
    }

    /* forward pass, keeping every pre-collision state and every body state before each fluid
     * step (and after the last) */
    const size_t nbs = (size_t)(n_bodies > 0 ? n_bodies : 1);
    const size_t ntb = (size_t)(total_beads > 0 ? total_beads : 1);
    double* states = (double*)malloc(sizeof(double) * 19 * N * (size_t)(n_steps + 1));
    double* bst = (double*)malloc(sizeof(double) * S_N * nbs * (size_t)(n_steps + 1));
    double* bead_F = (double*)malloc(sizeof(double) * 3 * ntb * (size_t)m);   /* per MD step */
    double* sub = (double*)malloc(sizeof(double) * S_N * nbs * (size_t)(m + 1));
    double* pose = (double*)malloc(sizeof(double) * 13 * nbs * (size_t)m);
    double* wca = (double*)malloc(sizeof(double) * 6 * nbs);
    /* per body, reverse of one MD step: adjoints of the body force and lab torque, of the
     * pose (centre, quaternion, rotation matrix) and of the step's velocities */
    double* RA = (double*)malloc(sizeof(double) * RA_N * nbs);
    if (!states || !bst || !bead_F || !sub || !pose || !wca || !RA) {
        free(states); free(bst); free(bead_F); free(sub); free(pose); free(wca); free(RA);
        return -1;
    }
    double J = 0.0;
    for (int n = 0; n <= n_steps; ++n) {
        for (int b = 0; b < n_bodies; ++b) orc_body_state(s, b, bst + ((size_t)n * nbs + b) * S_N);
        if (n == n_steps) break;
        memcpy(states + (size_t)n * 19 * N, orc_box_f(s), sizeof(double) * 19 * N);
        orc_step(s, 1);
        for (int b = 0; b < n_bodies; ++b) {
            double st[19];
            orc_body_state(s, b, st);
            for (int a = 0; a < 3; ++a) J += dJ_dF[((size_t)n * n_bodies + b) * 3 + a] * st[S_F + a];
        }
    }
    memcpy(states + (size_t)n_steps * 19 * N, orc_box_f(s), sizeof(double) * 19 * N);
    if (J_out) *J_out = J;

    /* backward pass */
    double* lam = (double*)calloc((size_t)19 * N, sizeof(double));     /* adjoint of f^{n+1} */
    double* lam_n = (double*)calloc((size_t)19 * N, sizeof(double));   /* adjoint of f^n */
    double* lam_F = (double*)calloc((size_t)3 * N, sizeof(double));
    double* lam_u = (double*)calloc((size_t)3 * N, sizeof(double));
    double* g = (double*)calloc((size_t)3 * N, sizeof(double));
    double* bstate = (double*)calloc(S_N * nbs, sizeof(double));   /* adjoint of the body state */
    for (int b = 0; b < n_bodies; ++b) dJ_dgamma[b] = 0.0;
    for (int k = 0; k < 3 * total_beads; ++k) dJ_doffsets[k] = 0.0;
#define SUB(b, k) (sub + ((size_t)(k) * nbs + (b)) * S_N)
#define POSE(b, k) (pose + ((size_t)(k) * nbs + (b)) * 13)
    for (int n = n_steps - 1; n >= 0; --n) {
        const double* f = states + (size_t)n * 19 * N;
        /* the MD steps of fluid step n again: poses, bead forces, body states, spread force */
        memset(g, 0, sizeof(double) * 3 * N);
        for (int b = 0; b < n_bodies; ++b) memcpy(SUB(b, 0), bst + ((size_t)n * nbs + b) * S_N, sizeof(double) * S_N);
        for (int k = 0; k < m; ++k) {
            /* every body's pose of MD step k, then the WCA forces between them */
            for (int b = 0; b < n_bodies; ++b) orc_box_first_half(s, b, SUB(b, k), h, POSE(b, k));
            wca_forces(s, p->wca_epsilon, dims, n_bodies, pose + (size_t)k * nbs * 13, wca);
            for (int b = 0, kb = 0; b < n_bodies; ++b) {
                const double* off; int nb; double pos0[3], q0[4], gamma; int fixed;
                orc_box_body(s, b, &off, &nb, pos0, q0, &gamma, &fixed);
                double* P = POSE(b, k);
                double R[3][3];
                rotmat(P + S_QUAT, R);
                double Fs[3] = {0, 0, 0}, Ts[3] = {0, 0, 0};
                for (int j = 0; j < nb; ++j, ++kb) {
                    const double* bk = off + 3 * j;
                    double d[3], r[3], v[3] = {0, 0, 0}, e[3];
                    cross3(P + S_OM, bk, e);
                    for (int a = 0; a < 3; ++a) {
                        d[a] = R[a][0] * bk[0] + R[a][1] * bk[1] + R[a][2] * bk[2];
                        r[a] = P[S_POS + a] + d[a];
                        if (!fixed) v[a] = P[S_VEL + a] + R[a][0] * e[0] + R[a][1] * e[1] + R[a][2] * e[2];
                    }
                    int64_t idx[8]; double w[8], uk[3] = {0, 0, 0};
                    orc_trilinear(nx, ny, nz, r, idx, w);
                    for (int c = 0; c < 8; ++c) {
                        if (mask[idx[c]]) continue;
                        double rho, u[3];
                        node_u(f, N, idx[c], p->g_ext, &rho, u);
                        for (int a = 0; a < 3; ++a) uk[a] += w[c] * u[a];
                    }
                    double* F = bead_F + 3 * ((size_t)k * ntb + kb);
                    for (int a = 0; a < 3; ++a) F[a] = -gamma * (v[a] - uk[a]);
                    if (kT > 0.0) {   /* the forward run's bead noise of this MD step */
                        const double amp = sqrt(2.0 * kT * gamma / h) * sqrt(12.0);
                        double un[3];
                        orc_box_bead_uniforms(s, step0 + n, kb, k, un);
                        for (int a = 0; a < 3; ++a) F[a] += amp * un[a];
                    }
                    for (int c = 0; c < 8; ++c) {
                        if (mask[idx[c]]) continue;
                        for (int a = 0; a < 3; ++a) g[3 * idx[c] + a] -= w[c] * (h * F[a]);
                    }
                    double dxF[3];
                    cross3(d, F, dxF);
                    for (int a = 0; a < 3; ++a) { Fs[a] += F[a]; Ts[a] += dxF[a]; }
                }
                /* the state the MD step leaves: its pose, the second half kick */
                for (int a = 0; a < 3; ++a) {
                    Fs[a] += wca[6 * b + a];
                    Ts[a] += wca[6 * b + 3 + a];
                }
                double mid[S_N];
                memcpy(mid, P, sizeof(double) * 13);
                for (int a = 0; a < 3; ++a) {
                    mid[S_F + a] = Fs[a];
                    mid[S_T + a] = R[0][a] * Ts[0] + R[1][a] * Ts[1] + R[2][a] * Ts[2];
                }
                orc_box_second_half(s, b, mid, h, SUB(b, k + 1));
            }
        }
        /* streaming transpose and collision VJP (each node writes only its own entries) */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int64_t here = x + (int64_t)nx * (y + (int64_t)ny * z);
                    if (mask[here]) {
                        for (int i = 0; i < 19; ++i) lam_n[i * N + here] = 0.0;
                        for (int a = 0; a < 3; ++a) lam_F[3 * here + a] = 0.0;
                        continue;
                    }
                    double ls[19], fin[19], F[3], lin[19], lF[3];
                    for (int i = 0; i < 19; ++i) {
                        const int dx = wrapi(x + orc_velocity(i, 0), nx);
                        const int dy = wrapi(y + orc_velocity(i, 1), ny);
                        const int dz = wrapi(z + orc_velocity(i, 2), nz);
                        const int64_t dst = dx + (int64_t)nx * (dy + (int64_t)ny * dz);
                        ls[i] = mask[dst] ? lam[orc_opposite(i) * N + here] : lam[i * N + dst];
                        fin[i] = f[i * N + here];
                    }
                    for (int a = 0; a < 3; ++a) F[a] = p->g_ext[a] + g[3 * here + a];
                    orc_collide_vjp(p, fin, F, ls, lin, lF);
                    for (int i = 0; i < 19; ++i) lam_n[i * N + here] = lin[i];
                    for (int a = 0; a < 3; ++a) lam_F[3 * here + a] = lF[a];
                }
        /* coupling, excluded volume and body transpose, MD steps in reverse order */
        memset(lam_u, 0, sizeof(double) * 3 * N);
        for (int k = m - 1; k >= 0; --k) {
            /* (1) per body: the second half kick and the torque's rotation into the body frame */
            for (int b = 0; b < n_bodies; ++b) {
                const double* off; int nb; double pos0[3], q0[4], gamma; int fixed;
                orc_box_body(s, b, &off, &nb, pos0, q0, &gamma, &fixed);
                double mass, I[3];
                orc_box_body_mass(s, b, &mass, I);
                const double* P = POSE(b, k);
                const double* out = SUB(b, k + 1);
                const double* ab = bstate + S_N * (size_t)b;   /* adjoint of `out` */
                double* A = RA + RA_N * (size_t)b;
                memset(A, 0, sizeof(double) * RA_N);
                /* the objective takes the force of the last MD step of the fluid step */
                for (int a = 0; a < 3; ++a)
                    A[RA_F + a] = k == m - 1 ? dJ_dF[((size_t)n * n_bodies + b) * 3 + a] : 0.0;
                if (fixed) continue;
                double R[3][3], mu[3], em[3], T[3];
                rotmat(P + S_QUAT, R);
                for (int a = 0; a < 3; ++a) {
                    A[RA_F + a] += ab[S_F + a] + 0.5 * h * ab[S_VEL + a] / mass;
                    mu[a] = 0.5 * h * ab[S_OM + a] / I[a];
                    A[RA_TAU + a] = ab[S_T + a] + mu[a];
                    A[RA_VM + a] = ab[S_VEL + a];
                    A[RA_RC + a] = ab[S_POS + a];
                }
                for (int a = 0; a < 4; ++a) A[RA_QC + a] = ab[S_QUAT + a];
                euler_vjp(P + S_OM, I, mu, em);
                for (int a = 0; a < 3; ++a) A[RA_WM + a] = ab[S_OM + a] - em[a];
                /* tau = Q^T T with T the lab torque: T = Q tau */
                for (int a = 0; a < 3; ++a) {
                    T[a] = R[a][0] * out[S_T] + R[a][1] * out[S_T + 1] + R[a][2] * out[S_T + 2];
                    A[RA_TB + a] = R[a][0] * A[RA_TAU] + R[a][1] * A[RA_TAU + 1] + R[a][2] * A[RA_TAU + 2];
                }
                for (int a = 0; a < 3; ++a)
                    for (int c = 0; c < 3; ++c) A[RA_Q + 3 * a + c] += T[a] * A[RA_TAU + c];
            }
            /* (2) per body: its beads (coupling, spreading, kinematics) */
            for (int b = 0, kb = 0; b < n_bodies; ++b) {
                const double* off; int nb; double pos0[3], q0[4], gamma; int fixed;
                orc_box_body(s, b, &off, &nb, pos0, q0, &gamma, &fixed);
                const double* P = POSE(b, k);
                double* A = RA + RA_N * (size_t)b;
                const double* Fbar = A + RA_F;
                const double* Tbar = A + RA_TB;
                double R[3][3];
                rotmat(P + S_QUAT, R);
                for (int j = 0; j < nb; ++j, ++kb) {
                    const double* bk = off + 3 * j;
                    double d[3], r[3], e[3], v[3] = {0, 0, 0};
                    cross3(P + S_OM, bk, e);
                    for (int a = 0; a < 3; ++a) {
                        d[a] = R[a][0] * bk[0] + R[a][1] * bk[1] + R[a][2] * bk[2];
                        r[a] = P[S_POS + a] + d[a];
                        if (!fixed) v[a] = P[S_VEL + a] + R[a][0] * e[0] + R[a][1] * e[1] + R[a][2] * e[2];
                    }
                    int64_t idx[8]; double w[8];
                    orc_trilinear(nx, ny, nz, r, idx, w);
                    /* fractional position inside the cell, for the weight gradients */
                    double fr[3];
                    for (int a = 0; a < 3; ++a) { const double sa = r[a] - 0.5; fr[a] = sa - floor(sa); }
                    const double* Fk = bead_F + 3 * ((size_t)k * ntb + kb);
                    /* adjoint of the bead force: the objective and the body sums, the torque
                     * sum T = sum d x F, and the spreading g -= w h F */
                    double lFk[3], uc[8][3], uk[3] = {0, 0, 0}, TxD[3];
                    cross3(Tbar, d, TxD);
                    for (int a = 0; a < 3; ++a) lFk[a] = Fbar[a] + TxD[a];
                    for (int c = 0; c < 8; ++c) {
                        for (int a = 0; a < 3; ++a) uc[c][a] = 0.0;
                        if (mask[idx[c]]) continue;
                        double rho;
                        node_u(f, N, idx[c], p->g_ext, &rho, uc[c]);
                        for (int a = 0; a < 3; ++a) {
                            uk[a] += w[c] * uc[c][a];
                            lFk[a] -= w[c] * h * lam_F[3 * idx[c] + a];
                        }
                    }
                    /* F_k = -gamma (v_k - u_k) + sqrt(2 kT gamma / h) xi_k: the noise term
                     * F_k + gamma (v_k - u_k) scales with sqrt(gamma) */
                    double luk[3], lv[3];
                    for (int a = 0; a < 3; ++a) {
                        dJ_dgamma[b] += lFk[a] * (uk[a] - v[a]);
                        if (kT > 0.0 && gamma > 0.0)
                            dJ_dgamma[b] += lFk[a] * (Fk[a] + gamma * (v[a] - uk[a])) / (2.0 * gamma);
                        luk[a] = gamma * lFk[a];
                        lv[a] = -gamma * lFk[a];
                    }
                    /* interpolation and spreading weights at r */
                    double rbar[3] = {0, 0, 0};
                    for (int c = 0; c < 8; ++c) {
                        if (mask[idx[c]]) continue;
                        const int o[3] = {c & 1, (c >> 1) & 1, c >> 2};
                        double gw[3];
                        for (int a = 0; a < 3; ++a) {
                            double prod = o[a] ? 1.0 : -1.0;
                            for (int e2 = 0; e2 < 3; ++e2)
                                if (e2 != a) prod *= o[e2] ? fr[e2] : 1.0 - fr[e2];
                            gw[a] = prod;
                        }
                        double su = 0.0, sF = 0.0;
                        for (int a = 0; a < 3; ++a) {
                            su += uc[c][a] * luk[a];
                            sF += h * Fk[a] * lam_F[3 * idx[c] + a];
                            lam_u[3 * idx[c] + a] += w[c] * luk[a];
                        }
                        for (int a = 0; a < 3; ++a) rbar[a] += gw[a] * (su - sF);
                    }
                    /* r = R + d, d = Q b, and d enters T = sum d x F */
                    double dbar[3], FxT[3];
                    cross3(Fk, Tbar, FxT);
                    for (int a = 0; a < 3; ++a) dbar[a] = rbar[a] + (fixed ? 0.0 : FxT[a]);
                    double* ob = dJ_doffsets + 3 * (size_t)kb;
                    for (int a = 0; a < 3; ++a)
                        ob[a] += R[0][a] * dbar[0] + R[1][a] * dbar[1] + R[2][a] * dbar[2];
                    if (fixed) continue;
                    for (int a = 0; a < 3; ++a) {
                        A[RA_RC + a] += rbar[a];
                        for (int c = 0; c < 3; ++c) A[RA_Q + 3 * a + c] += dbar[a] * bk[c];
                    }
                    /* v = V_m + Q e, e = w_m x b */
                    double ebar[3], bxe[3], exw[3];
                    for (int a = 0; a < 3; ++a) {
                        A[RA_VM + a] += lv[a];
                        for (int c = 0; c < 3; ++c) A[RA_Q + 3 * a + c] += lv[a] * e[c];
                        ebar[a] = R[0][a] * lv[0] + R[1][a] * lv[1] + R[2][a] * lv[2];
                    }
                    cross3(bk, ebar, bxe);
                    cross3(ebar, P + S_OM, exw);
                    for (int a = 0; a < 3; ++a) { A[RA_WM + a] += bxe[a]; ob[a] += exw[a]; }
                }
            }
            /* (3) WCA pairs: the force f(x - y) on site x = R_b + Q_b o of body b enters F_b and
             * T_b; its adjoint g = Fbar_b + Tbar_b x d reaches both sites' positions through
             * df/dd, and the arm d through the torque */
            if (p->wca_epsilon > 0.0) {
                const double eps = p->wca_epsilon;
                const double *wpos, *wrad;
                int nw;
                orc_box_sites(s, &wpos, &wrad, &nw);
                for (int b = 0; b < n_bodies; ++b) {
                    const double* ob; int nbv; double rb;
                    orc_box_ev(s, b, &ob, &nbv, &rb);
                    const double *off; int nbd; double pos0[3], q0[4], gamma; int fixed_b;
                    orc_box_body(s, b, &off, &nbd, pos0, q0, &gamma, &fixed_b);
                    double* A = RA + RA_N * (size_t)b;
                    for (int kk = 0; kk < nbv; ++kk) {
                        double d[3], x[3], gk[3], TxD[3];
                        site_of(POSE(b, k), ob + 3 * kk, d, x);
                        cross3(A + RA_TB, d, TxD);
                        for (int a = 0; a < 3; ++a) gk[a] = A[RA_F + a] + TxD[a];
                        /* partners: static sites (c = -1), then the other bodies' sites */
                        for (int c = -1; c < n_bodies; ++c) {
                            if (c == b) continue;
                            const double* oc = NULL; int nc = 0; double rc = 0.0;
                            int fixed_c = 1;
                            if (c >= 0) {
                                orc_box_ev(s, c, &oc, &nc, &rc);
                                const double *offc; int nbc; double pc[3], qc[4], gc;
                                orc_box_body(s, c, &offc, &nbc, pc, qc, &gc, &fixed_c);
                            } else {
                                nc = nw;
                            }
                            for (int j = 0; j < nc; ++j) {
                                double y[3], dj[3] = {0, 0, 0}, dd[3], f[3] = {0, 0, 0}, Jc[2];
                                double sigma;
                                if (c < 0) {
                                    for (int a = 0; a < 3; ++a) y[a] = wpos[3 * j + a];
                                    sigma = rb + wrad[j];
                                } else {
                                    site_of(POSE(c, k), oc + 3 * j, dj, y);
                                    sigma = rb + rc;
                                }
                                min_image3(dims, x, y, dd);
                                if (!wca_pair_j(eps, sigma, dd, f, Jc)) continue;
                                /* dbar = (c I + 2 c' dd dd^T) g */
                                const double dg = dd[0] * gk[0] + dd[1] * gk[1] + dd[2] * gk[2];
                                double db[3];
                                for (int a = 0; a < 3; ++a) db[a] = Jc[0] * gk[a] + 2.0 * Jc[1] * dg * dd[a];
                                if (!fixed_b) {
                                    double fxt[3];
                                    cross3(f, A + RA_TB, fxt);
                                    for (int a = 0; a < 3; ++a) {
                                        A[RA_RC + a] += db[a];
                                        for (int e2 = 0; e2 < 3; ++e2)
                                            A[RA_Q + 3 * a + e2] += (db[a] + fxt[a]) * ob[3 * kk + e2];
                                    }
                                }
                                if (c >= 0 && !fixed_c) {
                                    double* Ac = RA + RA_N * (size_t)c;
                                    for (int a = 0; a < 3; ++a) {
                                        Ac[RA_RC + a] -= db[a];
                                        for (int e2 = 0; e2 < 3; ++e2)
                                            Ac[RA_Q + 3 * a + e2] -= db[a] * oc[3 * j + e2];
                                    }
                                }
                            }
                        }
                    }
                }
            }
            /* (4) per body: rotation matrix, quaternion rotation, drift, first half kick */
            for (int b = 0; b < n_bodies; ++b) {
                const double* off; int nb; double pos0[3], q0[4], gamma; int fixed;
                orc_box_body(s, b, &off, &nb, pos0, q0, &gamma, &fixed);
                if (fixed) continue;
                double mass, I[3];
                orc_box_body_mass(s, b, &mass, I);
                const double* P = POSE(b, k);
                const double* in = SUB(b, k);   /* before MD step k */
                double* ab = bstate + S_N * (size_t)b;
                double* A = RA + RA_N * (size_t)b;
                double* Rcbar = A + RA_RC;
                double* qcbar = A + RA_QC;
                double* Vmbar = A + RA_VM;
                double* wmbar = A + RA_WM;
                double dQ[4][3][3];
                rotmat_partials(P + S_QUAT, dQ);
                for (int j = 0; j < 4; ++j)
                    for (int a = 0; a < 3; ++a)
                        for (int c = 0; c < 3; ++c) qcbar[j] += A[RA_Q + 3 * a + c] * dQ[j][a][c];
                /* first half: q_c = p/|p|, p = q_in (x) dq(w_m) (q_c = q_in when w_m = 0) */
                const double* qi = in + S_QUAT;
                const double* wm = P + S_OM;
                double qibar[4];
                const double wn = sqrt(wm[0] * wm[0] + wm[1] * wm[1] + wm[2] * wm[2]);
                if (wn > 0.0) {
                    const double ang = 0.5 * h * wn;
                    const double dq[4] = {cos(ang), sin(ang) * wm[0] / wn, sin(ang) * wm[1] / wn,
                                          sin(ang) * wm[2] / wn};
                    double pq[4];
                    pq[0] = qi[0] * dq[0] - qi[1] * dq[1] - qi[2] * dq[2] - qi[3] * dq[3];
                    pq[1] = qi[0] * dq[1] + qi[1] * dq[0] + qi[2] * dq[3] - qi[3] * dq[2];
                    pq[2] = qi[0] * dq[2] - qi[1] * dq[3] + qi[2] * dq[0] + qi[3] * dq[1];
                    pq[3] = qi[0] * dq[3] + qi[1] * dq[2] - qi[2] * dq[1] + qi[3] * dq[0];
                    const double np = sqrt(pq[0] * pq[0] + pq[1] * pq[1] + pq[2] * pq[2] + pq[3] * pq[3]);
                    const double* qc = P + S_QUAT;
                    const double qq = qc[0] * qcbar[0] + qc[1] * qcbar[1] + qc[2] * qcbar[2] + qc[3] * qcbar[3];
                    double pb[4];
                    for (int a = 0; a < 4; ++a) pb[a] = (qcbar[a] - qc[a] * qq) / np;
                    /* product rule of the quaternion product, component by component */
                    qibar[0] = pb[0] * dq[0] + pb[1] * dq[1] + pb[2] * dq[2] + pb[3] * dq[3];
                    qibar[1] = -pb[0] * dq[1] + pb[1] * dq[0] - pb[2] * dq[3] + pb[3] * dq[2];
                    qibar[2] = -pb[0] * dq[2] + pb[1] * dq[3] + pb[2] * dq[0] - pb[3] * dq[1];
                    qibar[3] = -pb[0] * dq[3] - pb[1] * dq[2] + pb[2] * dq[1] + pb[3] * dq[0];
                    double dqbar[4];
                    dqbar[0] = pb[0] * qi[0] + pb[1] * qi[1] + pb[2] * qi[2] + pb[3] * qi[3];
                    dqbar[1] = -pb[0] * qi[1] + pb[1] * qi[0] + pb[2] * qi[3] - pb[3] * qi[2];
                    dqbar[2] = -pb[0] * qi[2] - pb[1] * qi[3] + pb[2] * qi[0] + pb[3] * qi[1];
                    dqbar[3] = -pb[0] * qi[3] + pb[1] * qi[2] - pb[2] * qi[1] + pb[3] * qi[0];
                    /* dq = (cos(h n/2), s(n) w) with n = |w|, s(n) = sin(h n/2)/n */
                    const double sn = sin(ang) / wn;
                    const double dsn = (0.5 * h * cos(ang) / wn - sin(ang) / (wn * wn));
                    const double wdq = wm[0] * dqbar[1] + wm[1] * dqbar[2] + wm[2] * dqbar[3];
                    for (int a = 0; a < 3; ++a)
                        wmbar[a] += -sin(ang) * 0.5 * h * (wm[a] / wn) * dqbar[0] + sn * dqbar[1 + a] +
                                    dsn * (wm[a] / wn) * wdq;
                } else {
                    for (int a = 0; a < 4; ++a) qibar[a] = qcbar[a];
                }
                /* drift R_c = R_in + h V_m; kick V_m = V_in + h F_prev/2M;
                 * w_m = w_in + h (tau_prev - w_in x I w_in)/2I */
                double mu2[3], em2[3];
                for (int a = 0; a < 3; ++a) {
                    Vmbar[a] += h * Rcbar[a];
                    mu2[a] = 0.5 * h * wmbar[a] / I[a];
                }
                euler_vjp(in + S_OM, I, mu2, em2);
                for (int a = 0; a < 3; ++a) {
                    ab[S_POS + a] = Rcbar[a];
                    ab[S_VEL + a] = Vmbar[a];
                    ab[S_OM + a] = wmbar[a] - em2[a];
                    ab[S_F + a] = 0.5 * h * Vmbar[a] / mass;
                    ab[S_T + a] = mu2[a];
                }
                for (int a = 0; a < 4; ++a) ab[S_QUAT + a] = qibar[a];
            }
        }
#undef SUB
#undef POSE
        /* node velocities depend on f^n (every MD step of the fluid step samples them) */
        for (int64_t x = 0; x < N; ++x) {
            if (mask[x]) continue;
            const double lu[3] = {lam_u[3 * x], lam_u[3 * x + 1], lam_u[3 * x + 2]};
            if (lu[0] == 0.0 && lu[1] == 0.0 && lu[2] == 0.0) continue;
            double rho, u[3];
            node_u(f, N, x, p->g_ext, &rho, u);
            for (int i = 0; i < 19; ++i) {
                double acc = 0.0;
                for (int a = 0; a < 3; ++a) acc += (orc_velocity(i, a) - u[a]) * lu[a];
                lam_n[i * N + x] += acc / rho;
            }
        }
        double* t = lam; lam = lam_n; lam_n = t;
    }
    /* the box ends at the last state of the window */
    orc_box_set_f(s, states + (size_t)n_steps * 19 * N);
    free(states); free(bst); free(bead_F); free(sub); free(pose); free(wca); free(RA); free(lam);
    free(lam_n); free(lam_F); free(lam_u); free(g); free(bstate);
    return 0;
}
