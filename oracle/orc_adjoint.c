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
 * Scope: every body fixed (bead velocities zero, positions constant over the window) and a
 * deterministic fluid (kT = 0); boundary masks allowed.  The adjoint of one step is the
 * transpose of each of its parts, taken in reverse order:
 *   streaming with halfway bounce-back  ->  lambda*_i(y) = lambda_i(y + c_i) if y + c_i is a
 *                                           fluid node, else lambda_opp(i)(y);
 *   collision f* = C(f, F)               ->  vector-Jacobian product of the mode-space collision
 *                                           (orc_collide_vjp below, pinned by finite differences);
 *   spreading g = -sum w F_k             ->  adjoint of F_k gets -sum_c w_c lambda_F(x_c);
 *   friction F_k = gamma u_k             ->  d gamma += lambda_Fk . u_k, lambda_uk = gamma lambda_Fk;
 *   interpolation u_k = sum w_c u(x_c)   ->  lambda_u(x_c) += w_c lambda_uk, and the position
 *                                           derivative of the weights;
 *   node velocity u = (j + g/2)/rho      ->  lambda_f_i += (c_i - u) . lambda_u / rho.
 * Every pre-collision state of the window is kept in memory (19 * N doubles per step).
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
int orc_box_plain_md(const orc_sim* s);

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

int orc_adjoint(orc_sim* s, const orc_params* p, int n_steps, int n_bodies, const double* dJ_dF,
                double* J_out, double* dJ_dgamma, double* dJ_doffsets)
{
    int dims[3];
    orc_box_dims(s, dims);
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const int64_t N = (int64_t)nx * ny * nz;
    const uint8_t* mask = orc_box_mask(s);
    if (orc_box_kT(s) != 0.0 || !orc_box_plain_md(s) || n_steps < 0) return -1;
    adj_tables();   /* before the parallel node loop */

    /* bodies: fixed, constant bead positions */
    int total_beads = 0;
    for (int b = 0; b < n_bodies; ++b) {
        const double* off; int nb; double pos[3], q[4], gamma; int fixed;
        if (orc_box_body(s, b, &off, &nb, pos, q, &gamma, &fixed) != 0 || !fixed) return -1;
        total_beads += nb;
    }

    /* forward pass, keeping every pre-collision state and the bead forces */
    double* states = (double*)malloc(sizeof(double) * 19 * N * (size_t)(n_steps + 1));
    double* bead_F = (double*)malloc(sizeof(double) * 3 * (size_t)total_beads * (n_steps + 1));
    if (!states || !bead_F) { free(states); free(bead_F); return -1; }
    double J = 0.0;
    for (int n = 0; n < n_steps; ++n) {
        memcpy(states + (size_t)n * 19 * N, orc_box_f(s), sizeof(double) * 19 * N);
        orc_step(s, 1);
        int k0 = 0;
        for (int b = 0; b < n_bodies; ++b) {
            double st[19];
            orc_body_state(s, b, st);
            const double* off; int nb; double pos[3], q[4], gamma; int fixed;
            orc_box_body(s, b, &off, &nb, pos, q, &gamma, &fixed);
            for (int a = 0; a < 3; ++a) J += dJ_dF[((size_t)n * n_bodies + b) * 3 + a] * st[13 + a];
            k0 += nb;
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
    double* dr = (double*)calloc((size_t)3 * total_beads, sizeof(double));
    for (int b = 0; b < n_bodies; ++b) dJ_dgamma[b] = 0.0;
    for (int n = n_steps - 1; n >= 0; --n) {
        const double* f = states + (size_t)n * 19 * N;
        /* spread force of step n, recomputed from f^n */
        memset(g, 0, sizeof(double) * 3 * N);
        for (int b = 0, kb = 0; b < n_bodies; ++b) {
            const double* off; int nb; double pos[3], q[4], gamma; int fixed;
            orc_box_body(s, b, &off, &nb, pos, q, &gamma, &fixed);
            double R[3][3];
            rotmat(q, R);
            for (int k = 0; k < nb; ++k, ++kb) {
                double r[3];
                for (int a = 0; a < 3; ++a)
                    r[a] = pos[a] + R[a][0] * off[3 * k] + R[a][1] * off[3 * k + 1] + R[a][2] * off[3 * k + 2];
                int64_t idx[8]; double w[8], uk[3] = {0, 0, 0};
                orc_trilinear(nx, ny, nz, r, idx, w);
                for (int c = 0; c < 8; ++c) {
                    if (mask[idx[c]]) continue;
                    double rho, u[3];
                    node_u(f, N, idx[c], p->g_ext, &rho, u);
                    for (int a = 0; a < 3; ++a) uk[a] += w[c] * u[a];
                }
                for (int a = 0; a < 3; ++a) bead_F[3 * (size_t)kb + a] = gamma * uk[a];
                for (int c = 0; c < 8; ++c) {
                    if (mask[idx[c]]) continue;
                    for (int a = 0; a < 3; ++a) g[3 * idx[c] + a] -= w[c] * gamma * uk[a];
                }
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
        /* coupling transpose */
        memset(lam_u, 0, sizeof(double) * 3 * N);
        for (int b = 0, kb = 0; b < n_bodies; ++b) {
            const double* off; int nb; double pos[3], q[4], gamma; int fixed;
            orc_box_body(s, b, &off, &nb, pos, q, &gamma, &fixed);
            double R[3][3];
            rotmat(q, R);
            for (int k = 0; k < nb; ++k, ++kb) {
                double r[3];
                for (int a = 0; a < 3; ++a)
                    r[a] = pos[a] + R[a][0] * off[3 * k] + R[a][1] * off[3 * k + 1] + R[a][2] * off[3 * k + 2];
                int64_t idx[8]; double w[8];
                orc_trilinear(nx, ny, nz, r, idx, w);
                /* fractional position inside the cell, for the weight gradients */
                double d[3];
                for (int a = 0; a < 3; ++a) { const double sa = r[a] - 0.5; d[a] = sa - floor(sa); }
                double lFk[3], uc[8][3], uk[3] = {0, 0, 0};
                for (int a = 0; a < 3; ++a) lFk[a] = dJ_dF[((size_t)n * n_bodies + b) * 3 + a];
                for (int c = 0; c < 8; ++c) {
                    for (int a = 0; a < 3; ++a) uc[c][a] = 0.0;
                    if (mask[idx[c]]) continue;
                    double rho;
                    node_u(f, N, idx[c], p->g_ext, &rho, uc[c]);
                    for (int a = 0; a < 3; ++a) {
                        uk[a] += w[c] * uc[c][a];
                        lFk[a] -= w[c] * lam_F[3 * idx[c] + a];
                    }
                }
                const double* Fk = bead_F + 3 * (size_t)kb;
                for (int a = 0; a < 3; ++a) dJ_dgamma[b] += lFk[a] * uk[a];
                double luk[3];
                for (int a = 0; a < 3; ++a) luk[a] = gamma * lFk[a];
                for (int c = 0; c < 8; ++c) {
                    if (mask[idx[c]]) continue;
                    const int o[3] = {c & 1, (c >> 1) & 1, c >> 2};
                    double gw[3];
                    for (int a = 0; a < 3; ++a) {
                        double prod = o[a] ? 1.0 : -1.0;
                        for (int e = 0; e < 3; ++e)
                            if (e != a) prod *= o[e] ? d[e] : 1.0 - d[e];
                        gw[a] = prod;
                    }
                    double su = 0.0, sF = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        su += uc[c][a] * luk[a];
                        sF += Fk[a] * lam_F[3 * idx[c] + a];
                        lam_u[3 * idx[c] + a] += w[c] * luk[a];
                    }
                    for (int a = 0; a < 3; ++a) dr[3 * (size_t)kb + a] += gw[a] * (su - sF);
                }
            }
        }
        /* node velocities depend on f^n */
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
    /* offsets: r_k = R + Q b_k */
    for (int b = 0, kb = 0; b < n_bodies; ++b) {
        const double* off; int nb; double pos[3], q[4], gamma; int fixed;
        orc_box_body(s, b, &off, &nb, pos, q, &gamma, &fixed);
        double R[3][3];
        rotmat(q, R);
        for (int k = 0; k < nb; ++k, ++kb)
            for (int a = 0; a < 3; ++a)
                dJ_doffsets[3 * (size_t)kb + a] = R[0][a] * dr[3 * (size_t)kb] +
                                                  R[1][a] * dr[3 * (size_t)kb + 1] +
                                                  R[2][a] * dr[3 * (size_t)kb + 2];
    }
    /* the box ends at the last state of the window */
    orc_box_set_f(s, states + (size_t)n_steps * 19 * N);
    free(states); free(bead_F); free(lam); free(lam_n); free(lam_F); free(lam_u); free(g); free(dr);
    return 0;
}
