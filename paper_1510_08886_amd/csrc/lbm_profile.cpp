// Slip velocity and Knudsen-layer analysis of a plane-channel velocity profile
// (Section VI of the paper: Eqs. defSlip, uNS, uNEQ). Host only.
#include <cmath>

#include "lbm_internal.h"

using namespace lbm;

extern "C" int lbm_profile_analysis(const double *u, int ny, lbm_profile_stats_t *stats,
                                    double *u_ns, double *u_neq) {
    if (!u || ny < 3 || (ny % 2 == 0 && ny < 4))
        return fail(LBM_E_INVALID, "lbm_profile_analysis: need u and ny >= 3 (>= 4 if even)");
    // Nodes at y_j = (j + 1/2) h, walls at y = 0 and y = ny h. The quadratic
    // through the nodes at distances h/2, 3h/2, 5h/2 from a wall takes the wall
    // value (15 u_0 - 10 u_1 + 3 u_2) / 8 (Lagrange weights at distance 0).
    const double lo = (15.0 * u[0] - 10.0 * u[1] + 3.0 * u[2]) / 8.0;
    const double hi = (15.0 * u[ny - 1] - 10.0 * u[ny - 2] + 3.0 * u[ny - 3]) / 8.0;
    const double u_wall = 0.5 * (lo + hi);
    double u_center;
    if (ny % 2) {
        u_center = u[ny / 2];
    } else {
        // cubic through the four middle nodes (at -3h/2, -h/2, h/2, 3h/2) at 0
        const int k = ny / 2;
        u_center = (-u[k - 2] + 9.0 * u[k - 1] + 9.0 * u[k] - u[k + 1]) / 16.0;
    }
    double mean = 0.0, z2 = 0.0;
    for (int j = 0; j < ny; ++j) {
        const double z = (j + 0.5) / ny - 0.5;
        mean += u[j];
        z2 += z * z;
    }
    mean /= ny;
    z2 /= ny;
    // parabola with the profile's centre value and node-averaged mass flow
    const double curv = (1.0 - mean / u_center) / z2;
    for (int j = 0; j < ny; ++j) {
        const double z = (j + 0.5) / ny - 0.5;
        const double ns = u_center * (1.0 - curv * z * z);
        if (u_ns) u_ns[j] = ns;
        if (u_neq) u_neq[j] = u[j] - ns;
    }
    if (stats) {
        stats->u_center = u_center;
        stats->u_wall = u_wall;
        stats->slip = u_wall / u_center;
        stats->mean = mean;
    }
    return LBM_OK;
}
