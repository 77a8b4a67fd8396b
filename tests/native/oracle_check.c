/*
 * oracle_check.c -- drives every entry point of the FP64 oracle (oracle/oracle.h) on small
 * boxes, for the AddressSanitizer / UndefinedBehaviorSanitizer build of tests/test_sanitizers.py
 * (test infrastructure: the oracle sources compiled together with this file).  The cases reach
 * the oracle's branches: a general mask (a pore, an obstacle whose rows hold several fluid runs,
 * a moving wall), the thermal fluid and beads, two MD steps per fluid step, excluded-volume and
 * wall sites, a body in contact with a periodic face, the reverse pass, shell relaxation and the
 * error returns.  Each case also checks what holds at any size (finite state, mass conserved by
 * the deterministic fluid without moving walls, the adjoint's J equal to the forward sum).
 * Exits 0 on success; the first failed check prints and exits 1.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

#define CHECK(cond, what)                                                            \
    do {                                                                             \
        if (!(cond)) {                                                               \
            fprintf(stderr, "FAIL %s:%d: %s (%s)\n", __FILE__, __LINE__, what, #cond); \
            exit(1);                                                                 \
        }                                                                            \
    } while (0)

static orc_params params(double kT, int md, double eps, unsigned long long seed)
{
    orc_params p;
    memset(&p, 0, sizeof p);
    p.rho0 = 1.0;
    p.tau_shear = 0.8;
    p.tau_bulk = 1.1;
    p.tau_odd = 0.9;
    p.tau_even = 1.2;
    p.kT = kT;
    p.g_ext[0] = 2e-6;
    p.g_ext[2] = -1e-6;
    p.seed = seed;
    p.md_substeps = md;
    p.wca_epsilon = eps;
    return p;
}

/* n points on a sphere of radius r (golden-angle spiral) */
static void sphere(int n, double r, double* off)
{
    const double ga = 3.14159265358979323846 * (3.0 - sqrt(5.0));
    for (int k = 0; k < n; ++k) {
        const double z = 1.0 - 2.0 * (k + 0.5) / n, s = sqrt(1.0 - z * z);
        off[3 * k] = r * s * cos(ga * k);
        off[3 * k + 1] = r * s * sin(ga * k);
        off[3 * k + 2] = r * z;
    }
}

static void add_sphere(orc_sim* s, double R, int n, const double pos[3], int fixed, double gamma)
{
    double* off = malloc(sizeof(double) * 3 * n);
    sphere(n, R, off);
    const double m = 30.0, I[3] = {50.0, 50.0, 50.0}, q[4] = {0.9, 0.1, -0.3, 0.3};
    const double v[3] = {1e-3, -2e-3, 5e-4}, w[3] = {2e-4, 0.0, -1e-4};
    double qn[4], nq = 0.0;
    for (int a = 0; a < 4; ++a) nq += q[a] * q[a];
    for (int a = 0; a < 4; ++a) qn[a] = q[a] / sqrt(nq);
    const int id = orc_add_body(s, off, n, m, I, pos, qn, v, w, gamma, fixed);
    CHECK(id >= 0, "orc_add_body");
    free(off);
}

static int finite_all(const double* v, size_t n)
{
    for (size_t k = 0; k < n; ++k)
        if (!isfinite(v[k])) return 0;
    return 1;
}

/* a 14 x 12 x 11 box: a pore wall (1), an obstacle (2) and a moving plate (3) */
static void masked_thermal_case(void)
{
    const int nx = 14, ny = 12, nz = 11, N = nx * ny * nz;
    orc_params p = params(1e-4, 2, 1.0, 99);
    orc_sim* s = orc_create(nx, ny, nz, &p);
    CHECK(s != NULL, "orc_create");
    unsigned char* mask = calloc((size_t)N, 1);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const double dy = y + 0.5 - ny / 2.0, dz = z + 0.5 - nz / 2.0;
                unsigned char v = 0;
                if (dy * dy + dz * dz > 25.0) v = 1;
                else if (x >= 9 && x <= 10 && y >= 5 && y <= 6) v = 2;
                else if (x == 2 && y < 4) v = 3;
                mask[x + nx * (y + ny * z)] = v;
            }
    CHECK(orc_set_mask(s, mask) == 0, "orc_set_mask");
    const double uw[3] = {0.0, 0.0, 1e-3};
    CHECK(orc_set_wall_velocity(s, 3, uw) == 0, "orc_set_wall_velocity");
    const double c0[3] = {5.5, 6.2, 5.4}, c1[3] = {12.9, 6.0, 0.3};   /* one across a face */
    add_sphere(s, 1.6, 24, c0, 0, 2.0);
    add_sphere(s, 1.2, 18, c1, 0, 1.0);
    double ev[3 * 6];
    sphere(6, 0.6, ev);
    CHECK(orc_set_excluded_volume(s, 0, ev, 6, 0.5) == 0, "excluded volume 0");
    CHECK(orc_set_excluded_volume(s, 1, ev, 6, 0.5) == 0, "excluded volume 1");
    double site[3 * 4] = {5.5, 1.2, 5.5, 0.2, 6.0, 9.9, 13.8, 11.6, 10.7, 7.0, 6.0, 1.0};
    CHECK(orc_add_wall_sites(s, site, 4, 0.5) == 0, "wall sites");
    double wf[12];
    CHECK(orc_wca_forces(s, wf) == 0 && finite_all(wf, 12), "orc_wca_forces");
    CHECK(isfinite(orc_wca_energy(s)), "orc_wca_energy");
    CHECK(orc_step(s, 6) == 0 && orc_step_count(s) == 6, "orc_step");
    /* after the first step the mask and sites are fixed */
    CHECK(orc_set_mask(s, mask) != 0, "mask after a step is refused");
    CHECK(orc_add_wall_sites(s, site, 1, 0.5) != 0, "sites after a step are refused");
    double tot[8];
    orc_totals(s, tot);
    CHECK(tot[7] == 1.0 && finite_all(tot, 7), "totals finite");
    double* fields = malloc(sizeof(double) * 4 * N);
    double* pops = malloc(sizeof(double) * 19 * N);
    orc_fields(s, fields);
    orc_populations(s, pops);
    CHECK(finite_all(fields, 4 * (size_t)N) && finite_all(pops, 19 * (size_t)N), "fields");
    orc_set_populations(s, pops);
    for (int b = 0; b < 2; ++b) {
        double st[19], bf[3 * 24];
        CHECK(orc_body_state(s, b, st) == 0 && finite_all(st, 19), "orc_body_state");
        CHECK(orc_bead_forces(s, b, bf) == 0 && finite_all(bf, 3 * (b ? 18 : 24)), "bead forces");
    }
    double st[19];
    CHECK(orc_body_state(s, 2, st) != 0 && orc_body_state(s, -1, st) != 0, "bad body index");
    CHECK(orc_step(s, 3) == 0, "more steps");
    orc_totals(s, tot);
    CHECK(tot[7] == 1.0, "finite after 9 steps");
    free(fields);
    free(pops);
    free(mask);
    orc_destroy(s);
}

/* deterministic fluid, plain walls: the total mass stays put */
static void deterministic_mass_case(void)
{
    const int nx = 9, ny = 10, nz = 8, N = nx * ny * nz;
    orc_params p = params(0.0, 1, 0.0, 5);
    orc_sim* s = orc_create(nx, ny, nz, &p);
    unsigned char* mask = calloc((size_t)N, 1);
    for (int z = 0; z < nz; ++z)
        for (int x = 0; x < nx; ++x) mask[x + nx * (0 + ny * z)] = 1;   /* one wall plane */
    CHECK(orc_set_mask(s, mask) == 0, "mask");
    const double c[3] = {4.2, 5.1, 3.9};
    add_sphere(s, 1.5, 20, c, 0, 1.5);
    double t0[8], t1[8];
    orc_totals(s, t0);
    CHECK(orc_step(s, 12) == 0, "steps");
    orc_totals(s, t1);
    CHECK(fabs(t1[0] - t0[0]) <= 1e-10 * t0[0], "mass conserved");
    free(mask);
    orc_destroy(s);
}

/* the reverse pass: J returned equals the forward sum of dJ_dF . F over the window */
static void adjoint_case(void)
{
    const int nx = 10, ny = 9, nz = 8, T = 5;
    orc_params p = params(0.0, 1, 0.0, 3);
    orc_sim* a = orc_create(nx, ny, nz, &p);
    orc_sim* b = orc_create(nx, ny, nz, &p);
    const double c[3] = {5.1, 4.4, 3.8};
    add_sphere(a, 1.5, 16, c, 1, 2.0);
    add_sphere(b, 1.5, 16, c, 1, 2.0);
    double w[3 * T];
    for (int k = 0; k < 3 * T; ++k) w[k] = 0.1 * (k % 5) - 0.2;
    double J = 0.0, dg = 0.0, doff[3 * 16];
    CHECK(orc_adjoint(a, &p, T, 1, w, &J, &dg, doff) == 0, "orc_adjoint");
    CHECK(isfinite(J) && isfinite(dg) && finite_all(doff, 48), "adjoint finite");
    double Jf = 0.0;
    for (int n = 0; n < T; ++n) {
        double st[19];
        CHECK(orc_step(b, 1) == 0 && orc_body_state(b, 0, st) == 0, "forward");
        for (int d = 0; d < 3; ++d) Jf += w[3 * n + d] * st[13 + d];
    }
    CHECK(fabs(J - Jf) <= 1e-12 * (fabs(Jf) + 1e-30), "J equals the forward sum");
    /* the general reverse pass: a thermal box, a free body next to a fixed one, two MD steps
     * per fluid step and WCA sites on both bodies and a few static sites; J again equals the
     * forward sum (same seed, same noise) and everything stays finite */
    orc_params pt = params(1e-4, 2, 1e-3, 3);
    orc_sim* t = orc_create(nx, ny, nz, &pt);
    orc_sim* tf = orc_create(nx, ny, nz, &pt);
    const double c2[3] = {2.0, 4.6, 4.1};
    const double ev[6] = {1.0, 0.0, 0.0, -1.0, 0.0, 0.0};
    const double sites[6] = {5.0, 1.2, 3.8, 5.3, 7.7, 3.9};
    orc_sim* both[2] = {t, tf};
    for (int k = 0; k < 2; ++k) {
        add_sphere(both[k], 1.5, 16, c, 0, 0.2);
        add_sphere(both[k], 1.0, 8, c2, 1, 0.2);
        CHECK(orc_set_excluded_volume(both[k], 0, ev, 2, 0.5) == 0, "excluded volume 0");
        CHECK(orc_set_excluded_volume(both[k], 1, ev, 2, 0.5) == 0, "excluded volume 1");
        CHECK(orc_add_wall_sites(both[k], sites, 2, 0.5) == 0, "wall sites");
    }
    double w2[6 * T], dg2[2], doff2[3 * 24];
    for (int k = 0; k < 6 * T; ++k) w2[k] = 0.1 * (k % 7) - 0.3;
    CHECK(orc_adjoint(t, &pt, T, 2, w2, &J, dg2, doff2) == 0, "general reverse pass");
    CHECK(isfinite(J) && finite_all(dg2, 2) && finite_all(doff2, 72), "general adjoint finite");
    Jf = 0.0;
    for (int n = 0; n < T; ++n) {
        CHECK(orc_step(tf, 1) == 0, "forward");
        for (int bb = 0; bb < 2; ++bb) {
            double st[19];
            CHECK(orc_body_state(tf, bb, st) == 0, "body state");
            for (int d = 0; d < 3; ++d) Jf += w2[6 * n + 3 * bb + d] * st[13 + d];
        }
    }
    CHECK(fabs(J - Jf) <= 1e-12 * (fabs(Jf) + 1e-30), "general J equals the forward sum");
    orc_destroy(tf);
    double lin[19], lout[19], lF[3], f[19], F[3] = {1e-4, -2e-4, 3e-5};
    const double u[3] = {0.01, -0.02, 0.005};
    orc_equilibrium(1.02, u, f);
    for (int i = 0; i < 19; ++i) lout[i] = 0.05 * i - 0.3;
    orc_collide_vjp(&p, f, F, lout, lin, lF);
    CHECK(finite_all(lin, 19) && finite_all(lF, 3), "orc_collide_vjp");
    orc_destroy(a);
    orc_destroy(b);
    orc_destroy(t);
}

static void tables_and_helpers(void)
{
    for (int i = 0; i < 19; ++i) {
        CHECK(orc_opposite(orc_opposite(i)) == i, "opposite");
        for (int a = 0; a < 3; ++a)
            CHECK(orc_velocity(i, a) == -orc_velocity(orc_opposite(i), a), "velocities");
        for (int k = 0; k < 19; ++k) CHECK(isfinite(orc_basis(k, i)), "basis");
    }
    for (int k = 0; k < 19; ++k) CHECK(orc_basis_norm(k) > 0.0, "basis norms");
    const unsigned int ctr[4] = {1u, 2u, 3u, 4u}, key[2] = {0xdeadbeefu, 7u};
    unsigned int out[4];
    orc_philox4x32_10(ctr, key, out);
    for (int k = 0; k < 4; ++k) {
        const double r = orc_uniform16(out[k]);
        CHECK(r > -0.5 && r < 0.5, "uniform16");
    }
    /* trilinear weights at interior, face and out-of-box points */
    const double pts[4][3] = {{3.3, 2.7, 1.1}, {0.0, 0.0, 0.0}, {-0.4, 7.9, 5.99}, {8.0, -3.2, 12.5}};
    for (int k = 0; k < 4; ++k) {
        int64_t idx[8];
        double w[8], sw = 0.0;
        orc_trilinear(8, 8, 6, pts[k], idx, w);
        for (int c = 0; c < 8; ++c) {
            CHECK(idx[c] >= 0 && idx[c] < 8 * 8 * 6, "trilinear index in the box");
            sw += w[c];
        }
        CHECK(fabs(sw - 1.0) < 1e-14, "trilinear weights sum to one");
    }
    double fin[19], fo[19];
    const double u[3] = {0.02, 0.0, -0.01}, F[3] = {0.0, 1e-3, 0.0};
    orc_params p = params(0.0, 1, 0.0, 1);
    orc_equilibrium(0.97, u, fin);
    orc_collide_node(&p, fin, F, NULL, fo);
    CHECK(finite_all(fo, 19), "orc_collide_node");
    double un[19];
    for (int i = 0; i < 19; ++i) un[i] = 0.03 * i - 0.27;
    p.kT = 1e-4;
    orc_collide_node(&p, fin, F, un, fo);
    CHECK(finite_all(fo, 19), "orc_collide_node, thermal");
}

static void relax_case(void)
{
    const double axes[3] = {4.0, 3.0, 2.5};
    const int n = 40;
    double pos[3 * 40], vel[3 * 40] = {0};
    sphere(n, 1.0, pos);
    for (int k = 0; k < n; ++k) {
        pos[3 * k] *= axes[0];
        pos[3 * k + 1] *= axes[1];
        pos[3 * k + 2] *= axes[2];
    }
    orc_relax_params rp = {10.0, 1.4, 0.1, 1000.0, 0.001, 1.0};
    const double e0 = orc_shell_energy(axes, n, pos, &rp);
    CHECK(orc_relax_shell(axes, n, pos, vel, &rp, 200) == 0, "orc_relax_shell");
    const double e1 = orc_shell_energy(axes, n, pos, &rp);
    CHECK(isfinite(e0) && isfinite(e1) && e1 <= e0 + 1e-12, "relaxation lowers the energy");
    const double x[3] = {6.0, -1.0, 0.5};
    double rs[3];
    const double t = orc_closest_point(axes, x, rs);
    double lhs = 0.0;
    for (int a = 0; a < 3; ++a) lhs += rs[a] * rs[a] / (axes[a] * axes[a]);
    CHECK(isfinite(t) && fabs(lhs - 1.0) < 1e-12, "closest point on the surface");
    CHECK(orc_relax_shell(axes, -1, pos, vel, &rp, 1) != 0, "bad shell refused");
}

int main(void)
{
    orc_set_num_threads(1);
    CHECK(orc_num_threads() >= 1, "threads");
    tables_and_helpers();
    masked_thermal_case();
    deterministic_mass_case();
    adjoint_case();
    relax_case();
    /* argument errors */
    orc_params bad = params(0.0, 1, 0.0, 1);
    bad.tau_shear = 0.4;
    orc_sim* s = orc_create(4, 4, 4, &bad);
    if (s) orc_destroy(s);
    CHECK(orc_create(0, 4, 4, &bad) == NULL, "empty box refused");
    printf("oracle_check: ok\n");
    return 0;
}
