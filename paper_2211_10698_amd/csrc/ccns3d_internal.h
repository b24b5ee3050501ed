// Internal declarations of the three-dimensional projection (not part of
// the C interface).
#ifndef CCNS3D_INTERNAL_H
#define CCNS3D_INTERNAL_H

#include <string>
#include <vector>

#include "ccns3d.h"

namespace ccns {

// Coefficient fields of the 3-D projection in the dense (nz+2) x (ny+2) x
// (nx+2) layout, index [a] the face direction.
struct HostCoef3 {
    std::vector<double> c[3];  // Poisson face weights A^2 / M between pressure unknowns
    std::vector<double> g[3];  // corrector factors A / M where c > 0
    std::vector<double> a[3];  // A on the velocity unknowns, 0 elsewhere
    std::vector<double> dinv;  // inverse diagonal of -L on the pressure unknowns
    int n_active = 0;
};

bool grid3_valid(const ccns3_grid *g);

// Validates the capacities and derives the fields above (host, FP64).
ccns_status prepare3(const ccns3_grid &g, const ccns3_params &p, const double *caps, HostCoef3 &o, std::string &err);

}  // namespace ccns

#endif
