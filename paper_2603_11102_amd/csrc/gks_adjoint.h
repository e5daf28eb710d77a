// gks_adjoint.h -- discrete adjoint of the S2O4 step with the actuator-line body force (internal).
//
// The reverse sweep linearises the step exactly; the WENO nonlinear weights are either held at their
// forward values (frozen, the default) or differentiated too (exact). Per face direction and stage
// operator the transpose is computed in gather form, without atomics, in four passes over buffers in
// the adjoint workspace:
//   A  recompute the forward face pipeline, store the inputs of the tangential WENO evaluations (the
//      normal face values q^L, q^R and the t1 line values q^L_m, q^R_m) and the adjoints of the
//      Gauss-point inputs (q^L, q^R, dQ/dn, dQ/dt1, dQ/dt2) from the flux seeds;
//   B  transpose of the t2 sweep (gather over the five faces whose stencils hold a t1 line value),
//   C  then, row by row in the same kernel with the t1 line adjoints in LDS, transpose of the t1 sweep
//      (gather over five positions) and of C = (q^L + q^R)/2;
//   D  transpose of the normal reconstruction into the padded cell adjoint;
// B, C and D rebuild the coefficients of the WENO evaluations they transpose (frozen: the weights;
// exact: the Jacobian row) from those stored inputs, or from the field for the normal evaluations, with
// the recompute's own routine on the same values, so the coefficients are bitwise the recompute's;
// then the transpose of the ghost-cell fill folds ghost adjoints into interior cells.
#pragma once

#include <stddef.h>

#include "gks_body.h"
#include "gks_internal.h"

namespace gks {

struct AdjFaceArgs {
    const double* q[4];     // field in LOCAL variable order (padded)
    const double* mu0[4];   // seed of L (interior, local order), stage 1 only
    const double* mu1[4];   // seed of L_t
    double* gpbar;          // [80][nface]
    double* t1v;            // [16][nt1pos]: t1 line values q^L_m, q^R_m, index (v * 2 + side) * 2 + m
    double* fv;             // [8][nnpos]: normal face values q^L, q^R, index v * 2 + side
    double* fabar;          // [12][nnpos]
    double* acc[4];         // padded cell adjoint accumulator (LOCAL order)
    int n_n, n_t1, n_t2;
    int chunk, tiles_t1, tiles_t2;
    long long st_n, st_t1, st_t2;
    long long ist_n, ist_t1, ist_t2;
    long long pad0;
    long long nface, nt1pos, nnpos;
    // inverse spacings (device, the forward's arrays; 1/h on a uniform axis): normal face spacings
    // [n_n + 1], normal widths [n_n], t1 widths [n_t1], t2 widths [n_t2]
    const double* ihf;
    const double* ihc;
    const double* ih1;
    const double* ih2;
    double eps;
    FluxConst<double> fc;
    int exact;              // 1: the WENO weights are differentiated (Jacobian rows), 0: frozen
};

size_t adjoint_workspace_bytes(int nx, int ny, int nz, int n_act);

struct AdjBuffers {
    double* lam[4];      // padded: adjoint of Q^{n+1} (then of Q^n)
    double* lam_pre[4];  // padded: adjoint of Q^{n+1,pre}
    double* lam_star[4]; // padded: adjoint of Q*
    double* acc[4];      // padded: transpose results
    double* qwork[4];    // padded: Q^n recomputed
    double* qpre[4];     // padded: Q^{n+1,pre}
    double* mu0[4];      // interior seeds
    double* mu1[4];
    double* gpbar;
    double* t1v;
    double* fv;
    double* fabar;
    double* pt;          // per-point scratch of the ALM adjoint: [16][n_act]
};

void adjoint_carve(char* base, int nx, int ny, int nz, int n_act, AdjBuffers* b, size_t* total);

hipError_t launch_adj_direction(const AdjFaceArgs& a, int stage, hipStream_t s);
// transpose of the axis-by-axis ghost fill (z, y, x); inflow sides are linearised at the padded field q
// (global variable order) the fill was applied to
hipError_t launch_adj_fold(double* f[4], const GridDesc& g, const int bc[6], const double* const q[4],
                           const double u_in[3], double c, double rho_ref, hipStream_t s);
// y = a x + b z over n elements (z may be null)
hipError_t launch_axpby(double* y, const double* x, double a, const double* z, double b, long long n, hipStream_t s);
// interior extraction / scatter between padded and interior layouts: dst_int = a * src_pad (+ b * src2_pad)
hipError_t launch_pad_to_int(double* dst, const double* src, double a, const double* src2, double b,
                             const GridDesc& g, hipStream_t s);
hipError_t launch_zero(double* y, long long n, hipStream_t s);

// immersed-body adjoint (a body at rest): lam (padded, adjoint of the field after the forcing) becomes
// the adjoint of the field before it, in place
hipError_t launch_ibm_adjoint(double* lam[4], const IbmArgs& a, hipStream_t s);

// actuator-line adjoint
struct AlmAdjArgs {
    AlmArgs fwd;             // forward arguments (positions and per-point data of this step)
    const double* lam_m[3];  // padded momentum adjoint (of the field after the projection)
    double* lam_pre[4];      // padded adjoint being formed (of the field before the projection)
    const double* qpre[4];   // padded field before the projection (FP64)
    double* grad_s;          // n_act, accumulated
    double* pt;              // scratch [16][n_act]
    double w0, w1, inv_n;    // objective weights and 1/(window steps)
};
hipError_t launch_alm_adjoint(const AlmAdjArgs& a, hipStream_t s);

}  // namespace gks
