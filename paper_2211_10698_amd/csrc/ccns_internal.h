// Internal declarations of libccns (not part of the C interface).
#ifndef CCNS_INTERNAL_H
#define CCNS_INTERNAL_H

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ccns.h"

namespace ccns {

// Gauss-Kronrod 7/15 nodes and weights on [-1, 1].
inline constexpr double kXK[8] = {0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
                       0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
                       0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
                       0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
inline constexpr double kWK[8] = {0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
                       0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
                       0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
                       0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
inline constexpr double kWG[4] = {0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
                       0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

// Device layout of every field: `rows` = ny+2 rows of `pitch` elements
// (pitch a multiple of 64), element (j, i) at j*pitch + i, with the same
// index meaning as the dense host layout.
struct Layout {
    int nx = 0, ny = 0, rows = 0, pitch = 0;
    size_t n = 0;  // rows * pitch
};

Layout make_layout(int nx, int ny);

// Coefficient fields derived from the capacities on the host, in the dense
// (ny+2) x (nx+2) layout.  Every name is a field of the device workspace.
struct HostCoef {
    std::vector<double> cx, cy, dinv;         // Poisson face weights and inverse diagonal
    std::vector<double> gx, gy;               // corrector factors A/V on coupled faces
    std::vector<double> ax, ay;               // A^x, A^y (mass fluxes, divergence)
    std::vector<double> het;                  // cont(0, D) at cells
    std::vector<double> hbx, hby;             // (het_L + het_R)/4 at faces (convective bracket)
    std::vector<double> dx, dy;               // Dirichlet data
    std::vector<double> vu, vv;               // V^x, V^y on velocity unknowns, 0 elsewhere
    std::vector<double> bxx, bxy, byy, byx;   // viscous face weights
    std::vector<double> wxx, wyy;             // 1/W^xx, 1/W^yy (cells)
    std::vector<double> nxx, nxy, nyx, nyy;   // node strain weights
    std::vector<double> hdx, hdy;             // inverse Jacobi diagonal of H (faces)
    std::vector<double> vinv;                 // 1/V on pressure unknowns
    std::vector<double> utx, uty;             // D on non-unknown faces, 0 on unknowns
    std::vector<double> vur, vvr;             // V^x, V^y on every face (kinetic energy)
    std::vector<double> vdx, vdy;             // visc(strain(U~, D)) on unknown faces
    int n_active = 0;                         // pressure unknowns
    int n_uact = 0, n_vact = 0;               // velocity unknowns
    int n_out = 0;                            // outflow faces the projection corrects
    // force on the bodies: the cells and nodes whose capacities differ across
    // them (the cut ones), FORCE_W values each (see ForceCell / ForceNode)
    std::vector<double> fcell, fnode;
};

// Entries of the force tables (one row of FORCE_W doubles each).
enum ForceCell {
    FC_J, FC_I, FC_WPX, FC_WPY, FC_WVX, FC_WVY,          // weights of P and of the cell strains
    FC_WXX, FC_BXX_E, FC_BXX_W, FC_AXX,                  // S_xx = WXX (B_E (U-D)_E - B_W (U-D)_W + AXX (D_E - D_W))
    FC_WYY, FC_BYY_N, FC_BYY_S, FC_AYY
};
enum ForceNode {
    FN_J, FN_I, FN_WNX, FN_WNY,                          // weights of the node strains S_x, S_y
    FN_BXY_A, FN_BXY_B, FN_AXY,                          // g_x from the x-faces above and below
    FN_BYX_R, FN_BYX_L, FN_AYX,                          // g_y from the y-faces right and left
    FN_NXX, FN_NXY, FN_NYX, FN_NYY
};
constexpr int FORCE_W = 14;

// Validates the inputs and derives every coefficient field (host, FP64).
ccns_status prepare_coefficients(const ccns_grid &g, const ccns_params &prm, const double *caps,
                                 const double *dir, HostCoef &out, std::string &err);

// visc(strain(U, D)) with the Dirichlet terms, on the host (interior faces).
void host_viscous(const ccns_grid &g, const double *caps, const HostCoef &o, const double *Ux,
                  const double *Uy, std::vector<double> &vx, std::vector<double> &vy);

// One 2x2 agglomeration step of the Poisson weights (multigrid hierarchy).
void coarsen_poisson(int nx, int ny, const std::vector<double> &cx, const std::vector<double> &cy,
                     const std::vector<double> &dinv, int nxc, int nyc, std::vector<double> &cxc,
                     std::vector<double> &cyc, std::vector<double> &dinvc);

// Pseudo-inverse of a small symmetric positive semi-definite matrix.
std::vector<double> pseudo_inverse_spsd(std::vector<double> A, int n);

}  // namespace ccns

#endif
