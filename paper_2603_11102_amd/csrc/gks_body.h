// gks_body.h -- argument blocks of the actuator-line and immersed-boundary kernels (internal).
#pragma once

#include "gks_internal.h"

namespace gks {

struct AlmArgs {
    int n_act, nb, npb, corr;
    int tip;               // tip correction on (Section 4.4)
    double g1_axi, g1_tan; // g1 = exp(-c1 (N lambda - c2)) + 0.1 for the axial and tangential factors
    double hub[3];
    double omega, theta0, radius, u_inf, eps, cl_slope, alpha_clip, cd0, cd2, rho_ref, area;
    const double* r;      // device, npb
    const double* chord;  // device, npb
    const double* twist;  // device, npb
    const double* width;  // device, npb
    const double* scale;  // device, n_act, or null
    double* X;            // device, 3 n_act: point positions of the step
    double* fv;           // device, 3 n_act: force on the fluid per point
    double* out_alpha;    // device, n_act
    double* out_fx;
    double* out_ft;
    double* out_urel;
    double* out_phi;
    double* out_u;        // device, 3 n_act: sampled velocity
    int box_lo[3], box_n[3];
    GridDesc g;
    DevState* st;
};

struct IbmArgs {
    int npts, ncell, iters;
    double rho_ref;
    const double* xyz;    // device, 3 npts
    const double* dS;     // device, npts
    const int* cell;      // device, 3 ncell: (i, j, k) of every cell in some point's support
    const int* csr;       // device, ncell + 1
    const int* ent;       // device, point indices per cell (ascending)
    double* vbar;         // device, ncell
    const double* vel;    // device, 3 npts prescribed point velocities, or null (stationary points)
    double* vbar_vel;     // device, 3 ncell: v-bar = sum W V_p v_p / V-bar (zero when vel is null)
    double* partials;     // device, 3 * ceil(ncell / 256)
    GridDesc g;
    DevState* st;
};

// Tip-correction factor f = (2/pi) acos(min(1, exp(-g1 N (R - r) / (2 r sin phi)))) and df/dphi.
__device__ __forceinline__ double tip_factor(double g1, int N, double R, double r, double phi, double* dfdphi) {
    const double sp = sin(phi);
    const double K = g1 * N * (R - r) / (2.0 * r);
    const double E = exp(-K / sp);
    if (!(E < 1.0)) {
        if (dfdphi) *dfdphi = 0.0;
        return 0.0;
    }
    if (dfdphi) *dfdphi = -(2.0 / M_PI) * E * K * cos(phi) / (sp * sp * sqrt(1.0 - E * E));
    return (2.0 / M_PI) * acos(E);
}

template <typename real>
hipError_t launch_alm(Field4<real> f, const AlmArgs& a, hipStream_t s);
hipError_t launch_ibm_vbar(const IbmArgs& a, hipStream_t s);
hipError_t launch_alm_points_only(Field4<double> f, const AlmArgs& a, hipStream_t s);
template <typename real>
hipError_t launch_ibm(Field4<real> f, const IbmArgs& a, hipStream_t s);
int ibm_blocks(int ncell);

}  // namespace gks
