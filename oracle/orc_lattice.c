/*
 * orc_lattice.c -- D3Q19 velocity set, weights and the orthogonal mode basis.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper runs a multi-relaxation-time lattice Boltzmann fluid (Sec. 1.1) but names no
 * velocity set or basis.  The oracle uses the D3Q19 set with weights 1/3, 1/18, 1/36 and the
 * orthogonal moment basis of Duenweg, Schiller & Ladd, in which each basis vector is a
 * polynomial in the lattice velocity.  The norms b_k are not typed in: they are computed from
 * their definition b_k = sum_i w_i e_k(c_i)^2 so that a wrong polynomial shows up as a
 * failed orthogonality pin rather than as a consistent error.
 */
#include "oracle.h"

static const int VEL[19][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
};

int orc_velocity(int i, int axis) { return VEL[i][axis]; }

double orc_weight(int i)
{
    int c2 = VEL[i][0] * VEL[i][0] + VEL[i][1] * VEL[i][1] + VEL[i][2] * VEL[i][2];
    if (c2 == 0) return 1.0 / 3.0;
    if (c2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

int orc_opposite(int i)
{
    for (int j = 0; j < 19; ++j)
        if (VEL[j][0] == -VEL[i][0] && VEL[j][1] == -VEL[i][1] && VEL[j][2] == -VEL[i][2])
            return j;
    return -1;
}

/* e_k(c): 0 mass; 1-3 momentum; 4 bulk; 5-9 shear; 10-15 odd kinetic; 16-18 even kinetic */
double orc_basis(int k, int i)
{
    const double cx = VEL[i][0], cy = VEL[i][1], cz = VEL[i][2];
    const double c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0:  return 1.0;
    case 1:  return cx;
    case 2:  return cy;
    case 3:  return cz;
    case 4:  return c2 - 1.0;
    case 5:  return 3.0 * cx * cx - c2;
    case 6:  return cy * cy - cz * cz;
    case 7:  return cx * cy;
    case 8:  return cy * cz;
    case 9:  return cz * cx;
    case 10: return (3.0 * c2 - 5.0) * cx;
    case 11: return (3.0 * c2 - 5.0) * cy;
    case 12: return (3.0 * c2 - 5.0) * cz;
    case 13: return (cy * cy - cz * cz) * cx;
    case 14: return (cz * cz - cx * cx) * cy;
    case 15: return (cx * cx - cy * cy) * cz;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * cx * cx - c2);
    case 18: return (2.0 * c2 - 3.0) * (cy * cy - cz * cz);
    default: return 0.0;
    }
}

double orc_basis_norm(int k)
{
    double b = 0.0;
    for (int i = 0; i < 19; ++i) b += orc_weight(i) * orc_basis(k, i) * orc_basis(k, i);
    return b;
}
