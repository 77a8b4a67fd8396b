/*
 * orc_lbrb.c -- one time step of the raspberry / lattice-Boltzmann method, FP64, plain loops.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * State of a box (lattice units, spacing 1, time step 1):
 *   f[i][node]  pre-collision populations f_i(x, n) ("after streaming"), i = 0..18,
 *               node = x + nx*(y + ny*z), node (x,y,z) centred at (x+1/2, y+1/2, z+1/2);
 *   mask[node]  1 = boundary (solid) node, 0 = fluid;
 *   bodies      raspberry centres (position R, unit quaternion q, velocity V, body-frame
 *               angular velocity w, mass M, principal inertia I, friction gamma, fixed flag,
 *               force F and body-frame torque T of the previous step) and the body-frame
 *               offsets b_k of their beads.
 *
 * One step n -> n+1, in this order (the paper's description of each part is cited inline);
 * steps 1-7 and 10 form one MD step of length h, repeated m = md_substeps times (h = 1/m)
 * on the frozen fluid before 8 and 9:
 *   1  free bodies: half kick with last MD step's force/torque, drift, quaternion rotation
 *   2  bead positions r_k = R + R(q) b_k and velocities v_k = V + R(q)(w x b_k)
 *   3  node velocities u = (j + g_ext/2)/rho from the current populations
 *   4  trilinear interpolation of u at each bead
 *   5  friction + bead noise F_k = -gamma (v_k - u_k) + f_s
 *   6  the opposite force -h F_k spread onto the same 8 nodes with the same weights
 *   7  body force F = sum F_k + WCA forces of its excluded-volume sites, torque
 *      T = sum (r_k - R) x F_k (+ the same for the sites), torque into the body frame
 *   8  collision of every fluid node in mode space with the force g_ext + spread force
 *   9  streaming with halfway bounce-back at boundary nodes
 *  10  free bodies: second half kick with this MD step's force/torque
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double pos[3], quat[4], vel[3], omega[3];
    double mass, inertia[3], gamma;
    int fixed;
    double force[3], torque_body[3];   /* of the last completed step */
    int n_beads;
    int64_t first_bead;                /* index of the first bead in the box's bead numbering */
    double* offsets;                   /* n_beads*3, body frame                               */
    double* bead_force;                /* n_beads*3, lab frame, last step                     */
    int n_ev;                          /* excluded-volume sites (not coupled to the fluid)    */
    double* ev_offsets;                /* n_ev*3, body frame                                  */
    double ev_radius;
} orc_body;

struct orc_sim {
    int nx, ny, nz;
    int64_t n;
    orc_params p;
    double* f;        /* 19*n, pre-collision */
    double* fpost;    /* 19*n, post-collision scratch */
    double* g;        /* 3*n spread force */
    uint8_t* mask;    /* 0 = fluid, k > 0 = boundary node of wall k */
    double uwall[256][3];   /* velocity of wall k (zero unless set) */
    int64_t step;
    int n_bodies, cap_bodies;
    orc_body* bodies;
    int64_t n_beads_total;
    int n_sites;          /* static WCA sites (pore beads) */
    double* site_pos;     /* n_sites*3, lab */
    double* site_radius;  /* n_sites */
};

/* ------------------------------------------------------------------------- helpers */

/* The lattice and basis functions of orc_lattice.c evaluated once into tables.            */
static double TE[19][19], TB[19], TW[19];
static int TC[19][3], TOPP[19], tables_ready = 0;

static void tables(void)
{
    if (tables_ready) return;
    for (int i = 0; i < 19; ++i) {
        TW[i] = orc_weight(i);
        TOPP[i] = orc_opposite(i);
        for (int a = 0; a < 3; ++a) TC[i][a] = orc_velocity(i, a);
    }
    for (int k = 0; k < 19; ++k) {
        TB[k] = orc_basis_norm(k);
        for (int i = 0; i < 19; ++i) TE[k][i] = orc_basis(k, i);
    }
    tables_ready = 1;
}

static int64_t node_index(const orc_sim* s, int x, int y, int z)
{
    return (int64_t)x + (int64_t)s->nx * ((int64_t)y + (int64_t)s->ny * (int64_t)z);
}

static int wrap(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }

static double tau_of_mode(const orc_params* p, int k)
{
    if (k == 4) return p->tau_bulk;
    if (k >= 5 && k <= 9) return p->tau_shear;
    if (k >= 10 && k <= 15) return p->tau_odd;
    return p->tau_even; /* 16..18 */
}

/* rotation matrix of a unit quaternion (w,x,y,z): body frame -> lab frame                 */
static void quat_matrix(const double q[4], double m[3][3])
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

static void mat_vec(const double m[3][3], const double v[3], double out[3])
{
    for (int a = 0; a < 3; ++a) out[a] = m[a][0] * v[0] + m[a][1] * v[1] + m[a][2] * v[2];
}

static void mat_t_vec(const double m[3][3], const double v[3], double out[3])
{
    for (int a = 0; a < 3; ++a) out[a] = m[0][a] * v[0] + m[1][a] * v[1] + m[2][a] * v[2];
}

static void cross(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* Hamilton product a (x) b                                                                 */
static void quat_mul(const double a[4], const double b[4], double out[4])
{
    out[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    out[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    out[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    out[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

/* four Philox words for (box seed, step, index, domain, block)                             */
static void draw(const orc_sim* s, int64_t step, uint32_t index, uint32_t domain,
                 uint32_t block, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)((uint64_t)step & 0xFFFFFFFFu), index,
                       (domain << 16) | block, (uint32_t)((uint64_t)step >> 32)};
    uint32_t key[2] = {(uint32_t)(s->p.seed & 0xFFFFFFFFu), (uint32_t)(s->p.seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* 16-bit half h of a block of Philox words: low half of word h/2 for even h, high for odd  */
static uint32_t half_of(const uint32_t words[4], int h)
{
    uint32_t w = words[h / 2];
    return (h % 2 == 0) ? (w & 0xFFFFu) : (w >> 16);
}

/* ------------------------------------------------------------------------- single node */

/* Equilibrium in mode space: mass, momentum, and the second moments of a Maxwellian at
 * second order in u (rho/3 delta + rho u u); kinetic (ghost) modes have zero equilibrium. */
static void equilibrium_modes(double rho, const double u[3], double meq[19])
{
    for (int k = 0; k < 19; ++k) meq[k] = 0.0;
    meq[0] = rho;
    meq[1] = rho * u[0];
    meq[2] = rho * u[1];
    meq[3] = rho * u[2];
    meq[4] = rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    meq[5] = rho * (2.0 * u[0] * u[0] - u[1] * u[1] - u[2] * u[2]);
    meq[6] = rho * (u[1] * u[1] - u[2] * u[2]);
    meq[7] = rho * u[0] * u[1];
    meq[8] = rho * u[1] * u[2];
    meq[9] = rho * u[2] * u[0];
}

static void modes_to_populations(const double m[19], double f[19])
{
    tables();
    for (int i = 0; i < 19; ++i) {
        double acc = 0.0;
        for (int k = 0; k < 19; ++k) acc += TE[k][i] * m[k] / TB[k];
        f[i] = TW[i] * acc;
    }
}

void orc_equilibrium(double rho, const double u[3], double f_out[19])
{
    double meq[19];
    equilibrium_modes(rho, u, meq);
    modes_to_populations(meq, f_out);
}

void orc_collide_node(const orc_params* p, const double f_in[19], const double F[3],
                      const double* unoise, double f_out[19])
{
    double m[19], meq[19], S[19], mpost[19];
    tables();
    for (int k = 0; k < 19; ++k) {
        double acc = 0.0;
        for (int i = 0; i < 19; ++i) acc += TE[k][i] * f_in[i];
        m[k] = acc;
    }
    const double rho = m[0];
    /* velocity including half the force (second-order forcing) */
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (m[1 + a] + 0.5 * F[a]) / rho;
    equilibrium_modes(rho, u, meq);

    /* source of the second moments: u F + F u, projected onto modes 4..9 */
    for (int k = 0; k < 19; ++k) S[k] = 0.0;
    S[4] = 2.0 * (u[0] * F[0] + u[1] * F[1] + u[2] * F[2]);
    S[5] = 2.0 * (2.0 * u[0] * F[0] - u[1] * F[1] - u[2] * F[2]);
    S[6] = 2.0 * (u[1] * F[1] - u[2] * F[2]);
    S[7] = u[0] * F[1] + u[1] * F[0];
    S[8] = u[1] * F[2] + u[2] * F[1];
    S[9] = u[2] * F[0] + u[0] * F[2];

    mpost[0] = m[0];
    for (int a = 0; a < 3; ++a) mpost[1 + a] = m[1 + a] + F[a];
    const double mu = 3.0 * p->kT; /* kT / c_s^2 */
    for (int k = 4; k < 19; ++k) {
        const double gk = 1.0 - 1.0 / tau_of_mode(p, k);
        double v = meq[k] + gk * (m[k] - meq[k]) + 0.5 * (1.0 + gk) * S[k];
        if (unoise) {
            const double phi = sqrt(mu * p->rho0 * TB[k] * (1.0 - gk * gk));
            v += phi * sqrt(12.0) * unoise[k];
        }
        mpost[k] = v;
    }
    modes_to_populations(mpost, f_out);
}

void orc_trilinear(int nx, int ny, int nz, const double r[3], int64_t idx[8], double w[8])
{
    const int dims[3] = {nx, ny, nz};
    int i0[3];
    double d[3];
    for (int a = 0; a < 3; ++a) {
        const double sa = r[a] - 0.5;
        const double fl = floor(sa);
        d[a] = sa - fl;
        i0[a] = wrap((int)(fl - floor(fl / dims[a]) * dims[a]), dims[a]);
    }
    int c = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int x = (i0[0] + dx) % nx, y = (i0[1] + dy) % ny, z = (i0[2] + dz) % nz;
                idx[c] = (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * (int64_t)z);
                w[c] = (dx ? d[0] : 1.0 - d[0]) * (dy ? d[1] : 1.0 - d[1]) *
                       (dz ? d[2] : 1.0 - d[2]);
                ++c;
            }
}

/* ------------------------------------------------------------------------- whole box */

/* pre-collision state from a post-collision one: pull along every link, reflecting links
 * whose upstream node is a boundary node back into the opposite population of the node. */
static void stream(orc_sim* s)
{
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const int64_t n = s->n;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t here = node_index(s, x, y, z);
                if (s->mask[here]) {
                    for (int i = 0; i < 19; ++i) s->f[i * n + here] = 0.0;
                    continue;
                }
                for (int i = 0; i < 19; ++i) {
                    const int sx = wrap(x - TC[i][0], nx);
                    const int sy = wrap(y - TC[i][1], ny);
                    const int sz = wrap(z - TC[i][2], nz);
                    const int64_t src = node_index(s, sx, sy, sz);
                    if (s->mask[src]) {
                        /* halfway bounce-back; a wall moving with velocity u_w adds
                         * 2 w_i rho0 (c_i . u_w) / c_s^2 to the reflected population */
                        const double* uw = s->uwall[s->mask[src]];
                        const double cu = TC[i][0] * uw[0] + TC[i][1] * uw[1] + TC[i][2] * uw[2];
                        s->f[i * n + here] = s->fpost[TOPP[i] * n + here] + 6.0 * TW[i] * s->p.rho0 * cu;
                    } else {
                        s->f[i * n + here] = s->fpost[i * n + src];
                    }
                }
            }
}

static void initialise_fluid(orc_sim* s)
{
    double feq[19];
    orc_equilibrium(s->p.rho0, s->p.u0, feq);
    for (int64_t x = 0; x < s->n; ++x)
        for (int i = 0; i < 19; ++i) s->fpost[i * s->n + x] = s->mask[x] ? 0.0 : feq[i];
    /* the fluid starts in equilibrium just before a streaming step */
    stream(s);
}

orc_sim* orc_create(int nx, int ny, int nz, const orc_params* p)
{
    if (nx < 1 || ny < 1 || nz < 1 || !p) return NULL;
    tables();
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->n = (int64_t)nx * ny * nz;
    s->p = *p;
    s->f = (double*)calloc((size_t)(19 * s->n), sizeof(double));
    s->fpost = (double*)calloc((size_t)(19 * s->n), sizeof(double));
    s->g = (double*)calloc((size_t)(3 * s->n), sizeof(double));
    s->mask = (uint8_t*)calloc((size_t)s->n, 1);
    if (!s->f || !s->fpost || !s->g || !s->mask) { orc_destroy(s); return NULL; }
    initialise_fluid(s);
    return s;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    for (int b = 0; b < s->n_bodies; ++b) {
        free(s->bodies[b].offsets);
        free(s->bodies[b].bead_force);
        free(s->bodies[b].ev_offsets);
    }
    free(s->bodies);
    free(s->site_pos);
    free(s->site_radius);
    free(s->f); free(s->fpost); free(s->g); free(s->mask);
    free(s);
}

int orc_set_mask(orc_sim* s, const uint8_t* mask)
{
    if (!s || !mask || s->step != 0) return -1;
    for (int64_t x = 0; x < s->n; ++x) s->mask[x] = mask[x];
    initialise_fluid(s);
    return 0;
}

int orc_set_wall_velocity(orc_sim* s, int wall, const double u[3])
{
    if (!s || !u || wall < 1 || wall > 255 || s->step != 0) return -1;
    for (int a = 0; a < 3; ++a) s->uwall[wall][a] = u[a];
    initialise_fluid(s);
    return 0;
}

int orc_add_body(orc_sim* s, const double* offsets, int n_beads, double mass,
                 const double inertia[3], const double pos[3], const double quat[4],
                 const double vel[3], const double omega_body[3], double gamma, int fixed)
{
    if (!s || n_beads < 1 || !offsets) return -1;
    if (!fixed && (!(mass > 0) || !(inertia[0] > 0) || !(inertia[1] > 0) || !(inertia[2] > 0)))
        return -1;
    if (s->n_bodies == s->cap_bodies) {
        int cap = s->cap_bodies ? 2 * s->cap_bodies : 8;
        orc_body* nb = (orc_body*)realloc(s->bodies, (size_t)cap * sizeof(orc_body));
        if (!nb) return -1;
        s->bodies = nb;
        s->cap_bodies = cap;
    }
    orc_body* b = &s->bodies[s->n_bodies];
    memset(b, 0, sizeof(*b));
    double qn = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    for (int a = 0; a < 3; ++a) {
        b->pos[a] = pos[a];
        b->vel[a] = fixed ? 0.0 : vel[a];
        b->omega[a] = fixed ? 0.0 : omega_body[a];
        b->inertia[a] = inertia[a];
    }
    for (int a = 0; a < 4; ++a) b->quat[a] = quat[a] / qn;
    b->mass = mass;
    b->gamma = gamma;
    b->fixed = fixed ? 1 : 0;
    b->n_beads = n_beads;
    b->first_bead = s->n_beads_total;
    b->offsets = (double*)malloc((size_t)n_beads * 3 * sizeof(double));
    b->bead_force = (double*)calloc((size_t)n_beads * 3, sizeof(double));
    memcpy(b->offsets, offsets, (size_t)n_beads * 3 * sizeof(double));
    s->n_beads_total += n_beads;
    return s->n_bodies++;
}

/* step 1: first half kick (previous force/torque), drift, rotation by the exponential of
 * the body-frame angular velocity (Sec. 2.3: velocity Verlet for the centre, quaternion
 * update from the angular velocity), over an MD step of length h.                          */
static void body_first_half(orc_body* b, double h)
{
    if (b->fixed) return;
    double Iw[3], wxIw[3];
    for (int a = 0; a < 3; ++a) b->vel[a] += 0.5 * h * b->force[a] / b->mass;
    for (int a = 0; a < 3; ++a) Iw[a] = b->inertia[a] * b->omega[a];
    cross(b->omega, Iw, wxIw);
    for (int a = 0; a < 3; ++a)
        b->omega[a] += 0.5 * h * (b->torque_body[a] - wxIw[a]) / b->inertia[a];
    for (int a = 0; a < 3; ++a) b->pos[a] += h * b->vel[a];
    const double wn = sqrt(b->omega[0] * b->omega[0] + b->omega[1] * b->omega[1] +
                           b->omega[2] * b->omega[2]);
    if (wn > 0.0) {
        const double ang = 0.5 * h * wn;   /* half the rotation angle */
        const double dq[4] = {cos(ang), sin(ang) * b->omega[0] / wn,
                              sin(ang) * b->omega[1] / wn, sin(ang) * b->omega[2] / wn};
        double qn[4];
        quat_mul(b->quat, dq, qn);
        const double nrm = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
        for (int a = 0; a < 4; ++a) b->quat[a] = qn[a] / nrm;
    }
}

/* step 10: second half kick with this MD step's force and body-frame torque               */
static void body_second_half(orc_body* b, double h)
{
    if (b->fixed) return;
    double Iw[3], wxIw[3];
    for (int a = 0; a < 3; ++a) b->vel[a] += 0.5 * h * b->force[a] / b->mass;
    for (int a = 0; a < 3; ++a) Iw[a] = b->inertia[a] * b->omega[a];
    cross(b->omega, Iw, wxIw);
    for (int a = 0; a < 3; ++a)
        b->omega[a] += 0.5 * h * (b->torque_body[a] - wxIw[a]) / b->inertia[a];
}

/* step 3: fluid velocity of a node from the current pre-collision populations             */
static void node_velocity(const orc_sim* s, int64_t x, double u[3])
{
    if (s->mask[x]) { u[0] = u[1] = u[2] = 0.0; return; }
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
        const double fi = s->f[i * s->n + x];
        rho += fi;
        for (int a = 0; a < 3; ++a) j[a] += TC[i][a] * fi;
    }
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * s->p.g_ext[a]) / rho;
}

/* steps 2-7 for one body in MD step k (length h) of the fluid step: returns the coupling
 * force (lab) and torque (lab) sums                                                         */
static void couple_body(orc_sim* s, orc_body* b, int k_md, double h, double Fsum[3],
                        double Tsum[3])
{
    double R[3][3];
    quat_matrix(b->quat, R);
    for (int a = 0; a < 3; ++a) Fsum[a] = Tsum[a] = 0.0;
    /* a force held over h carries the momentum variance 2 kT gamma h */
    const double amp = sqrt(2.0 * s->p.kT * b->gamma / h) * sqrt(12.0);
    for (int k = 0; k < b->n_beads; ++k) {
        const double* off = b->offsets + 3 * k;
        double d[3], r[3], v[3], wxb[3], rw[3];
        mat_vec(R, off, d);
        for (int a = 0; a < 3; ++a) r[a] = b->pos[a] + d[a];
        if (b->fixed) {
            v[0] = v[1] = v[2] = 0.0;
        } else {
            cross(b->omega, off, wxb);
            mat_vec(R, wxb, rw);
            for (int a = 0; a < 3; ++a) v[a] = b->vel[a] + rw[a];
        }
        /* fluid velocity interpolated between the 8 nearest nodes (eq. latticeboltzmannfriction) */
        int64_t idx[8];
        double w[8], uk[3] = {0.0, 0.0, 0.0};
        orc_trilinear(s->nx, s->ny, s->nz, r, idx, w);
        for (int c = 0; c < 8; ++c) {
            double un[3];
            node_velocity(s, idx[c], un);
            for (int a = 0; a < 3; ++a) uk[a] += w[c] * un[a];
        }
        /* friction plus a noise of variance 2 kT gamma per component */
        double F[3];
        uint32_t words[4] = {0, 0, 0, 0};
        if (s->p.kT > 0.0)
            draw(s, s->step, (uint32_t)(b->first_bead + k), 1u, (uint32_t)k_md, words);
        for (int a = 0; a < 3; ++a) {
            F[a] = -b->gamma * (v[a] - uk[a]);
            if (s->p.kT > 0.0) F[a] += amp * orc_uniform16(half_of(words, a));
        }
        /* the fluid receives the opposite momentum h F, on the same nodes with the same
         * weights (a force density over the unit fluid step)                               */
        for (int c = 0; c < 8; ++c) {
            if (s->mask[idx[c]]) continue;
            for (int a = 0; a < 3; ++a) s->g[3 * idx[c] + a] -= w[c] * (h * F[a]);
        }
        double dxF[3];
        cross(d, F, dxF);
        for (int a = 0; a < 3; ++a) {
            b->bead_force[3 * k + a] = F[a];
            Fsum[a] += F[a];
            Tsum[a] += dxF[a];
        }
    }
}

/* ---- WCA excluded volume (Sec. 2.1 inner layer, Sec. 2.3 pore beads) ---- */

/* separation a - b with each component taken to its nearest periodic image               */
static void min_image(const orc_sim* s, const double a[3], const double b[3], double d[3])
{
    const double L[3] = {(double)s->nx, (double)s->ny, (double)s->nz};
    for (int k = 0; k < 3; ++k) {
        d[k] = a[k] - b[k];
        d[k] -= L[k] * round(d[k] / L[k]);
    }
}

/* WCA pair at separation d (first site minus second) with sigma = r_a + r_b: adds the
 * force on the first site to F and returns the pair energy (0 beyond 2^(1/6) sigma).      */
static double wca_pair(double eps, double sigma, const double d[3], double F[3])
{
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double rc2 = pow(2.0, 1.0 / 3.0) * sigma * sigma;
    if (!(r2 < rc2)) return 0.0;
    const double s2 = sigma * sigma / r2, s6 = s2 * s2 * s2, s12 = s6 * s6;
    /* U = 4 eps (s12 - s6) + eps;  -dU/dr * (d / r) = 24 eps (2 s12 - s6) d / r^2          */
    const double coef = 24.0 * eps * (2.0 * s12 - s6) / r2;
    for (int k = 0; k < 3; ++k) F[k] += coef * d[k];
    return 4.0 * eps * (s12 - s6) + eps;
}

/* lab positions of a body's excluded-volume sites and their offsets from the centre      */
static void ev_sites(const orc_body* b, double* x, double* dv)
{
    double R[3][3];
    quat_matrix(b->quat, R);
    for (int k = 0; k < b->n_ev; ++k) {
        mat_vec(R, b->ev_offsets + 3 * k, dv + 3 * k);
        for (int a = 0; a < 3; ++a) x[3 * k + a] = b->pos[a] + dv[3 * k + a];
    }
}

/* WCA force and torque (lab, about the centre) on every body, 6 per body, and the total
 * energy with each pair counted once                                                      */
static double wca_all(const orc_sim* s, double* out)
{
    const double eps = s->p.wca_epsilon;
    double energy = 0.0;
    for (int b = 0; b < 6 * s->n_bodies; ++b) out[b] = 0.0;
    if (!(eps > 0.0)) return 0.0;
    for (int b = 0; b < s->n_bodies; ++b) {
        const orc_body* B = &s->bodies[b];
        if (B->n_ev == 0) continue;
        double* xb = (double*)malloc(sizeof(double) * 6 * (size_t)B->n_ev);
        double* db = xb + 3 * B->n_ev;
        ev_sites(B, xb, db);
        for (int k = 0; k < B->n_ev; ++k) {
            double F[3] = {0.0, 0.0, 0.0}, d[3];
            for (int w = 0; w < s->n_sites; ++w) {
                min_image(s, xb + 3 * k, s->site_pos + 3 * w, d);
                energy += wca_pair(eps, B->ev_radius + s->site_radius[w], d, F);
            }
            for (int o = 0; o < s->n_bodies; ++o) {
                const orc_body* O = &s->bodies[o];
                if (o == b || O->n_ev == 0) continue;
                double* xo = (double*)malloc(sizeof(double) * 6 * (size_t)O->n_ev);
                ev_sites(O, xo, xo + 3 * O->n_ev);
                for (int m = 0; m < O->n_ev; ++m) {
                    min_image(s, xb + 3 * k, xo + 3 * m, d);
                    energy += 0.5 * wca_pair(eps, B->ev_radius + O->ev_radius, d, F);
                }
                free(xo);
            }
            double T[3];
            cross(db + 3 * k, F, T);
            for (int a = 0; a < 3; ++a) {
                out[6 * b + a] += F[a];
                out[6 * b + 3 + a] += T[a];
            }
        }
        free(xb);
    }
    return energy;
}

int orc_wca_forces(const orc_sim* s, double* out)
{
    if (!s || !out) return -1;
    wca_all(s, out);
    return 0;
}

double orc_wca_energy(const orc_sim* s)
{
    if (!s) return 0.0;
    double* tmp = (double*)malloc(sizeof(double) * 6 * (size_t)(s->n_bodies > 0 ? s->n_bodies : 1));
    const double e = wca_all(s, tmp);
    free(tmp);
    return e;
}

int orc_set_excluded_volume(orc_sim* s, int body, const double* offsets, int n, double radius)
{
    if (!s || body < 0 || body >= s->n_bodies || n < 0 || (n > 0 && !offsets) ||
        !(radius >= 0.0) || s->step != 0)
        return -1;
    orc_body* b = &s->bodies[body];
    free(b->ev_offsets);
    b->ev_offsets = NULL;
    b->n_ev = 0;
    if (n > 0) {
        b->ev_offsets = (double*)malloc(sizeof(double) * 3 * (size_t)n);
        if (!b->ev_offsets) return -1;
        memcpy(b->ev_offsets, offsets, sizeof(double) * 3 * (size_t)n);
    }
    b->n_ev = n;
    b->ev_radius = radius;
    return 0;
}

int orc_add_wall_sites(orc_sim* s, const double* pos, int n, double radius)
{
    if (!s || n < 0 || (n > 0 && !pos) || !(radius >= 0.0) || s->step != 0) return -1;
    double* p = (double*)realloc(s->site_pos, sizeof(double) * 3 * (size_t)(s->n_sites + n + 1));
    if (!p) return -1;
    s->site_pos = p;
    double* r = (double*)realloc(s->site_radius, sizeof(double) * (size_t)(s->n_sites + n + 1));
    if (!r) return -1;
    s->site_radius = r;
    for (int k = 0; k < n; ++k) {
        for (int a = 0; a < 3; ++a) s->site_pos[3 * (s->n_sites + k) + a] = pos[3 * k + a];
        s->site_radius[s->n_sites + k] = radius;
    }
    s->n_sites += n;
    return 0;
}

static void collide_all(orc_sim* s)
{
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    const int64_t n = s->n;
    const int thermal = s->p.kT > 0.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t here = node_index(s, x, y, z);
                if (s->mask[here]) continue;
                double fin[19], fout[19], F[3], un[19];
                for (int i = 0; i < 19; ++i) fin[i] = s->f[i * n + here];
                for (int a = 0; a < 3; ++a) F[a] = s->p.g_ext[a] + s->g[3 * here + a];
                if (thermal) {
                    uint32_t w0[4], w1[4];
                    draw(s, s->step, (uint32_t)here, 0u, 0u, w0);
                    draw(s, s->step, (uint32_t)here, 0u, 1u, w1);
                    for (int k = 0; k < 4; ++k) un[k] = 0.0;
                    for (int k = 4; k < 19; ++k) {
                        const int h = k - 4;
                        un[k] = orc_uniform16(h < 8 ? half_of(w0, h) : half_of(w1, h - 8));
                    }
                }
                orc_collide_node(&s->p, fin, F, thermal ? un : NULL, fout);
                for (int i = 0; i < 19; ++i) s->fpost[i * n + here] = fout[i];
            }
}

int orc_step(orc_sim* s, int n_steps)
{
    if (!s || n_steps < 0) return -1;
    const int m = s->p.md_substeps > 1 ? s->p.md_substeps : 1;
    const double h = 1.0 / m;
    double* wca = (double*)malloc(sizeof(double) * 6 * (size_t)(s->n_bodies > 0 ? s->n_bodies : 1));
    if (!wca) return -1;
    for (int it = 0; it < n_steps; ++it) {
        memset(s->g, 0, (size_t)(3 * s->n) * sizeof(double));
        for (int k = 0; k < m; ++k) {
            for (int b = 0; b < s->n_bodies; ++b) body_first_half(&s->bodies[b], h);
            wca_all(s, wca);   /* at the poses of this MD step, before any body moves on */
            for (int b = 0; b < s->n_bodies; ++b) {
                orc_body* body = &s->bodies[b];
                double F[3], T[3], R[3][3], Tb[3];
                couple_body(s, body, k, h, F, T);
                for (int a = 0; a < 3; ++a) {
                    F[a] += wca[6 * b + a];
                    T[a] += wca[6 * b + 3 + a];
                }
                quat_matrix(body->quat, R);
                mat_t_vec(R, T, Tb);
                for (int a = 0; a < 3; ++a) {
                    body->force[a] = F[a];
                    body->torque_body[a] = Tb[a];
                }
            }
            for (int b = 0; b < s->n_bodies; ++b) body_second_half(&s->bodies[b], h);
        }
        collide_all(s);
        stream(s);
        s->step += 1;
    }
    free(wca);
    return 0;
}

int64_t orc_step_count(const orc_sim* s) { return s ? s->step : -1; }

void orc_fields(const orc_sim* s, double* rho_u)
{
    for (int64_t x = 0; x < s->n; ++x) {
        if (s->mask[x]) {
            for (int a = 0; a < 4; ++a) rho_u[4 * x + a] = 0.0;
            continue;
        }
        double rho = 0.0, u[3];
        for (int i = 0; i < 19; ++i) rho += s->f[i * s->n + x];
        node_velocity(s, x, u);
        rho_u[4 * x + 0] = rho;
        for (int a = 0; a < 3; ++a) rho_u[4 * x + 1 + a] = u[a];
    }
}

void orc_populations(const orc_sim* s, double* f)
{
    memcpy(f, s->f, (size_t)(19 * s->n) * sizeof(double));
}

void orc_set_populations(orc_sim* s, const double* f)
{
    for (int i = 0; i < 19; ++i)
        for (int64_t x = 0; x < s->n; ++x) s->f[i * s->n + x] = s->mask[x] ? 0.0 : f[i * s->n + x];
}

void orc_totals(const orc_sim* s, double out[8])
{
    for (int a = 0; a < 8; ++a) out[a] = 0.0;
    int finite = 1;
    const int64_t plane = (int64_t)s->nx * s->ny;
    for (int z = 0; z < s->nz; ++z) {
        double part[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t x = z * plane; x < (z + 1) * plane; ++x) {
            if (s->mask[x]) continue;
            for (int i = 0; i < 19; ++i) {
                const double fi = s->f[i * s->n + x];
                if (!isfinite(fi)) finite = 0;
                part[0] += fi;
                for (int a = 0; a < 3; ++a) part[1 + a] += TC[i][a] * fi;
            }
        }
        for (int a = 0; a < 4; ++a) out[a] += part[a];
    }
    for (int b = 0; b < s->n_bodies; ++b) {
        const orc_body* body = &s->bodies[b];
        if (body->fixed) continue;
        for (int a = 0; a < 3; ++a) out[4 + a] += body->mass * body->vel[a];
    }
    out[7] = finite ? 1.0 : 0.0;
}

int orc_body_state(const orc_sim* s, int body, double out[19])
{
    if (!s || body < 0 || body >= s->n_bodies) return -1;
    const orc_body* b = &s->bodies[body];
    for (int a = 0; a < 3; ++a) out[a] = b->pos[a];
    for (int a = 0; a < 4; ++a) out[3 + a] = b->quat[a];
    for (int a = 0; a < 3; ++a) out[7 + a] = b->vel[a];
    for (int a = 0; a < 3; ++a) out[10 + a] = b->omega[a];
    for (int a = 0; a < 3; ++a) out[13 + a] = b->force[a];
    for (int a = 0; a < 3; ++a) out[16 + a] = b->torque_body[a];
    return 0;
}

int orc_bead_forces(const orc_sim* s, int body, double* out)
{
    if (!s || body < 0 || body >= s->n_bodies) return -1;
    const orc_body* b = &s->bodies[body];
    memcpy(out, b->bead_force, (size_t)b->n_beads * 3 * sizeof(double));
    return 0;
}

/* ---- read access for the adjoint (orc_adjoint.c) ---- */
int orc_box_dims(const orc_sim* s, int dims[3])
{
    dims[0] = s->nx; dims[1] = s->ny; dims[2] = s->nz;
    return 0;
}
const double* orc_box_f(const orc_sim* s) { return s->f; }
void orc_box_set_f(orc_sim* s, const double* f) { memcpy(s->f, f, sizeof(double) * 19 * (size_t)s->n); }
const uint8_t* orc_box_mask(const orc_sim* s) { return s->mask; }
double orc_box_kT(const orc_sim* s) { return s->p.kT; }
/* MD steps per fluid step                                                                 */
int orc_box_md_steps(const orc_sim* s) { return s->p.md_substeps > 1 ? s->p.md_substeps : 1; }
/* body b's excluded-volume sites (body-frame offsets) and their radius                      */
int orc_box_ev(const orc_sim* s, int b, const double** offsets, int* n, double* radius)
{
    if (b < 0 || b >= s->n_bodies) return -1;
    *offsets = s->bodies[b].ev_offsets;
    *n = s->bodies[b].n_ev;
    *radius = s->bodies[b].ev_radius;
    return 0;
}
/* the uniforms (in (-1/2, 1/2)) of the bead noise that fluid step `step`, MD step k_md gives
 * bead `bead` (its index over all bodies in order), as couple_body draws them              */
int orc_box_bead_uniforms(const orc_sim* s, int64_t step, int bead, int k_md, double out[3])
{
    uint32_t words[4];
    draw(s, step, (uint32_t)bead, 1u, (uint32_t)k_md, words);
    for (int a = 0; a < 3; ++a) out[a] = orc_uniform16(half_of(words, a));
    return 0;
}
/* the static sites (lab positions, radii)                                                  */
int orc_box_sites(const orc_sim* s, const double** pos, const double** radius, int* n)
{
    *pos = s->site_pos;
    *radius = s->site_radius;
    *n = s->n_sites;
    return 0;
}
int orc_box_body_mass(const orc_sim* s, int b, double* mass, double inertia[3])
{
    if (b < 0 || b >= s->n_bodies) return -1;
    *mass = s->bodies[b].mass;
    for (int a = 0; a < 3; ++a) inertia[a] = s->bodies[b].inertia[a];
    return 0;
}
/* the first half of an MD step of length h (body_first_half) applied to a state of body b
 * in the layout of orc_body_state: out = position, quaternion, velocity and body-frame
 * angular velocity that the step's coupling uses                                          */
int orc_box_first_half(const orc_sim* s, int b, const double state[19], double h, double out[13])
{
    if (b < 0 || b >= s->n_bodies) return -1;
    orc_body t = s->bodies[b];
    for (int a = 0; a < 3; ++a) {
        t.pos[a] = state[a];
        t.vel[a] = state[7 + a];
        t.omega[a] = state[10 + a];
        t.force[a] = state[13 + a];
        t.torque_body[a] = state[16 + a];
    }
    for (int a = 0; a < 4; ++a) t.quat[a] = state[3 + a];
    body_first_half(&t, h);
    for (int a = 0; a < 3; ++a) {
        out[a] = t.pos[a];
        out[7 + a] = t.vel[a];
        out[10 + a] = t.omega[a];
    }
    for (int a = 0; a < 4; ++a) out[3 + a] = t.quat[a];
    return 0;
}
/* the second half of an MD step of length h (body_second_half) applied to body b: in and out
 * in the layout of orc_body_state; in holds the step's pose and velocities after the first
 * half, and the step's force and body-frame torque                                        */
int orc_box_second_half(const orc_sim* s, int b, const double in[19], double h, double out[19])
{
    if (b < 0 || b >= s->n_bodies) return -1;
    orc_body t = s->bodies[b];
    for (int a = 0; a < 3; ++a) {
        t.pos[a] = in[a];
        t.vel[a] = in[7 + a];
        t.omega[a] = in[10 + a];
        t.force[a] = in[13 + a];
        t.torque_body[a] = in[16 + a];
    }
    for (int a = 0; a < 4; ++a) t.quat[a] = in[3 + a];
    body_second_half(&t, h);
    for (int a = 0; a < 3; ++a) {
        out[a] = t.pos[a];
        out[7 + a] = t.vel[a];
        out[10 + a] = t.omega[a];
        out[13 + a] = t.force[a];
        out[16 + a] = t.torque_body[a];
    }
    for (int a = 0; a < 4; ++a) out[3 + a] = t.quat[a];
    return 0;
}
int orc_box_body(const orc_sim* s, int b, const double** offsets, int* n_beads, double pos[3],
                 double quat[4], double* gamma, int* fixed)
{
    if (b < 0 || b >= s->n_bodies) return -1;
    const orc_body* B = &s->bodies[b];
    *offsets = B->offsets;
    *n_beads = B->n_beads;
    for (int a = 0; a < 3; ++a) pos[a] = B->pos[a];
    for (int a = 0; a < 4; ++a) quat[a] = B->quat[a];
    *gamma = B->gamma;
    *fixed = B->fixed;
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the parallel loops from here on (the baseline is timed at 1 and at all) */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
