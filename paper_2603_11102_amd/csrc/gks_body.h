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
    int samp_lo[3], samp_n[3];  // cells that the velocity sampling of any point can reach over a revolution
    int line_n;            // line sampling: samples along the direction of motion (<= 1: point sampling)
    double line_half;      // half-length of the sampling segment
    GridDesc g;
    DevState* st;
};

// Sampling positions of the line sampling of an actuator point (the NTNU rotor of Section 4.4): the
// midpoints s_k = l ((2k + 1) / N - 1), k = 0 .. N - 1, of N equal parts of the segment [-l, l] along
// the blade's direction of motion.
__host__ __device__ inline double line_offset(const AlmArgs& a, int k) {
    return a.line_half * ((double)(2 * k + 1) / (double)a.line_n - 1.0);
}

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
    const int* ncell_dev; // device cell count when the supports are rebuilt on the device (moving body),
                          // else null; ncell is then the capacity 64 npts
    int moving;
    GridDesc g;
    DevState* st;
};

// Rigid motion of the immersed body and the buffers of the per-step rebinning on the device.
struct IbmMoveArgs {
    double c0[3], vel[3], omega[3], t0;
    const double* xyz0;  // device, 3 npts: positions at t0
    double* xyz;         // device, 3 npts: positions of the step (IbmArgs::xyz)
    double* pvel;        // device, 3 npts: velocities of the step (IbmArgs::vel)
    int* base;           // device, 3 npts: lowest support cell per axis (clamped into the run)
    int run_lo[3], run_hi[3];  // cells of the body's grid per axis (a stretched mesh: the run of cells
                               // of the body's width; otherwise all cells); supports must stay inside
    unsigned* key[2];    // device, 64 npts each: cell index of the (cell, point) pairs, ping-pong
    int* val[2];         // device, 64 npts each: point index of the pairs
    int* hist;           // device, 256 * tiles: digit counts per tile, digit-major
    int* dtot;           // device, 256: pairs per digit
    int* tcnt;           // device, tiles: cells starting in each tile, then their offsets
    int* counts;         // device, [0] cells, [1] pairs
    int* cell;           // device, 3 * 64 npts (IbmArgs::cell)
    int* csr;            // device, 64 npts + 1 (IbmArgs::csr)
    int* ent;            // device, 64 npts: points per cell, the output of the pair sort (IbmArgs::ent)
};
constexpr int RADIX_TILE = 2048;  // pairs per workgroup of the sort and compaction passes (8 rounds of 256)

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
hipError_t launch_ibm_move(const IbmArgs& a, const IbmMoveArgs& m, hipStream_t s);
hipError_t launch_alm_points_only(Field4<double> f, const AlmArgs& a, hipStream_t s);
template <typename real>
hipError_t launch_ibm(Field4<real> f, const IbmArgs& a, hipStream_t s);
int ibm_blocks(int ncell);

}  // namespace gks
