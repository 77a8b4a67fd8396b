/*
 * orc_relax.c -- raspberry construction by constrained relaxation, FP64, plain loops.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Sec. 2.1 and its SI ("Details for ellipsoidal raspberry construction"): beads are spread
 * evenly over an ellipsoid x^2/a^2 + y^2/b^2 + z^2/c^2 = 1 by damped MD with two forces, a
 * harmonic restraint U = k |r - r_s|^2 towards the closest surface point r_s and a pairwise
 * WCA repulsion between the beads.  The closest point follows from the normal condition
 * r - r_s = (t/2) grad S(r_s), i.e. x = x_s (t/a^2 + 1) per axis, so x_s = x a^2 / (t + a^2);
 * putting that into the surface equation gives F(t) = sum (x a / (t + a^2))^2 - 1 = 0 (the
 * printed F(t) has a misplaced "+1" inside the squares), which is decreasing in t on
 * (-min a^2, inf) and is solved there by bisection.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>

/* F(t) for the point x, semi-axes a and their squares a2                                   */
static double surface_f(const double x[3], const double a[3], const double a2[3], double t)
{
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double v = x[k] * a[k] / (t + a2[k]);
        s += v * v;
    }
    return s - 1.0;
}

double orc_closest_point(const double axes[3], const double x[3], double rs[3])
{
    double a2[3], amin2 = INFINITY, amax = 0.0, rn = 0.0;
    for (int k = 0; k < 3; ++k) {
        a2[k] = axes[k] * axes[k];
        if (a2[k] < amin2) amin2 = a2[k];
        if (axes[k] > amax) amax = axes[k];
        rn += x[k] * x[k];
    }
    /* F > 0 just above -min a^2 (unless the point lies on that axis' plane) and F < 0 once
     * t > max a |x|, since each term is at most (x a / t)^2                                 */
    double lo = -amin2, hi = amax * sqrt(rn) + 1.0;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (surface_f(x, axes, a2, mid) > 0.0) lo = mid;
        else hi = mid;
    }
    const double t = 0.5 * (lo + hi);
    for (int k = 0; k < 3; ++k) rs[k] = x[k] * a2[k] / (t + a2[k]);
    return t;
}

/* forces on every bead of one shell: WCA from every other bead (j in order), then the
 * surface restraint                                                                        */
static void shell_forces(const double axes[3], int n, const double* pos,
                         const orc_relax_params* p, double* f)
{
    const double rc2 = pow(2.0, 1.0 / 3.0) * p->sigma * p->sigma;
    const double s2 = p->sigma * p->sigma;
    for (int i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3], r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                d[k] = pos[3 * i + k] - pos[3 * j + k];
                r2 += d[k] * d[k];
            }
            if (!(r2 < rc2)) continue;
            const double q = s2 / r2, q6 = q * q * q;
            const double coef = 24.0 * p->epsilon * (2.0 * q6 * q6 - q6) / r2;
            for (int k = 0; k < 3; ++k) fi[k] += coef * d[k];
        }
        double rs[3];
        orc_closest_point(axes, pos + 3 * i, rs);
        for (int k = 0; k < 3; ++k) f[3 * i + k] = fi[k] - 2.0 * p->k_surface * (pos[3 * i + k] - rs[k]);
    }
}

int orc_relax_shell(const double axes[3], int n, double* pos, double* vel,
                    const orc_relax_params* p, int n_steps)
{
    if (!axes || n < 1 || !pos || !vel || !p || n_steps < 0 || !(p->mass > 0.0) || !(p->dt > 0.0))
        return -1;
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!f) return -1;
    /* leapfrog with the friction -eta m v taken half before and half after the kick:
     * v(n+1/2) = ((1 - g) v(n-1/2) + dt F(n) / m) / (1 + g), g = eta dt / 2;  x += dt v     */
    const double g = 0.5 * p->damping * p->dt;
    for (int s = 0; s < n_steps; ++s) {
        shell_forces(axes, n, pos, p, f);
        for (int i = 0; i < 3 * n; ++i) {
            vel[i] = ((1.0 - g) * vel[i] + p->dt * f[i] / p->mass) / (1.0 + g);
            pos[i] += p->dt * vel[i];
        }
    }
    free(f);
    return 0;
}

double orc_shell_energy(const double axes[3], int n, const double* pos, const orc_relax_params* p)
{
    const double rc2 = pow(2.0, 1.0 / 3.0) * p->sigma * p->sigma;
    const double s2 = p->sigma * p->sigma;
    double e = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = i + 1; j < n; ++j) {
            double r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double d = pos[3 * i + k] - pos[3 * j + k];
                r2 += d * d;
            }
            if (!(r2 < rc2)) continue;
            const double q = s2 / r2, q6 = q * q * q;
            e += 4.0 * p->epsilon * (q6 * q6 - q6) + p->epsilon;
        }
        double rs[3], d2 = 0.0;
        orc_closest_point(axes, pos + 3 * i, rs);
        for (int k = 0; k < 3; ++k) d2 += (pos[3 * i + k] - rs[k]) * (pos[3 * i + k] - rs[k]);
        e += p->k_surface * d2;
    }
    return e;
}
