// gks_internal.h -- structures shared by the host library and the kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gks_device.h"

namespace gks {

constexpr int NG = 3;                    // ghost layers per side
constexpr int TILE1 = 16, TILE2 = 16;    // tangential faces per workgroup (t1 x t2)
constexpr int EXT1 = TILE1 + 4, EXT2 = TILE2 + 4;
constexpr int FACE_THREADS = 512;        // 8 wave64 per workgroup

// Tile of the high-order face kernel per precision. FP32: 16 x 16 faces, 512 threads (two waves per
// SIMD, up to 256 registers each). FP64: 16 x 8 faces, 256 threads: one workgroup per CU (its LDS), one
// wave per SIMD, so that a wave can use the 512 registers of the unified VGPR/AGPR file its doubled live
// state needs instead of spilling to scratch. Both map one thread per tile column (20 x 20 and 20 x 12)
// and one thread per face and Gauss line.
template <typename real>
struct FaceTile {
    static constexpr int T2 = 16, THREADS = 512;
};
template <>
struct FaceTile<double> {
    static constexpr int T2 = 8, THREADS = 256;
};

// Arguments of the per-direction face kernel. Arrays are in the face's LOCAL variable order
// (rho', m_normal, m_t1, m_t2); the caller permutes the global pointers.
template <typename real>
struct FaceArgs {
    const real* q[4];        // reconstructed field (padded layout)
    // residual contributions, four variables per cell in the global order (rho', rho U, rho V, rho W):
    real* r0;                // y pass: L (stage 1), interior layout [cell][4]
    real* r1;                // y pass: L_t, same layout
    real* rx0;               // x pass: L in the blocked layout [z][y/16][x][y%16][4]
    real* rx1;               // x pass: L_t, same layout
    int rx_nx, rx_nyb;       // nx and ceil(ny / 16) of the blocked layout
    real* out_a[4];          // epilogue: stage 1 -> Q*, stage 2 -> Q^{n+1} (padded)
    real* out_b[4];          // epilogue: stage 1 -> S (padded)
    const real* s_in[4];     // epilogue: stage 2 reads S (padded)
    const real* q_c[4];      // epilogue: stage 1 reads Q^n at the cell (padded)
    // FP32 compensated state, interior layout [cell][4] in the global order: the low-order parts of the
    // stage input of the epilogue (Q^n in stage 1, S in stage 2) and of its outputs (Q* and S; Q^{n+1});
    // null in FP64
    const real* lo_in;
    real* lo_a;
    real* lo_b;
    int n_n, n_t1, n_t2;     // interior cells along normal, t1, t2
    int chunk, tiles_t1, tiles_t2;
    // work split of the order-5 face kernel over its n_wg logical workgroups: seg_len == 0, workgroup b
    // marches chunk b / (tiles) of tile b % (tiles); seg_len > 0, it marches cells
    // [b seg_len, (b + 1) seg_len) of the tile-major (tile, cell) order, one segment per tile it meets
    int seg_len, n_wg;
    long long st_n, st_t1, st_t2;     // padded strides
    long long ist_n, ist_t1, ist_t2;  // interior strides
    long long pad0;                   // padded offset of interior cell (0,0,0)
    real inv_hn, inv_h1, inv_h2;
    // inverse spacings (device) of a stretched mesh (stretched != 0): normal face spacings [n_n + 1],
    // normal widths [n_n], t1 widths [n_t1], t2 widths [n_t2]; on a uniform axis every entry is 1/h
    int stretched;
    const real* ihf;
    const real* ihc;
    const real* ih1;
    const real* ih2;
    real eps;
    FluxConst<real> fc;
    real g_global[3];                 // constant body force (x, y, z) for the stage-2 epilogue
    const double* dt_ptr;             // device dt of the current step
    int mode;  // 3: x pass (write the blocked x arrays), 0: y pass (write the main arrays),
               // 4: z pass (add both, S2O4 stage update)
};

// Index of cell (x, y, z) in the blocked layout [z][y/16][x][y%16]: the x pass stores 16 consecutive y
// per row (its lanes run along y), the z pass reads a 16 x 16 (x, y) tile as one contiguous block.
__host__ __device__ inline long long rx_block_index(int x, int y, int z, int nx, int nyb) {
    return (((long long)z * nyb + (y >> 4)) * nx + x) * 16 + (y & 15);
}

// Device-resident scalars of a context (lives in the workspace).
constexpr int UMAX_BLOCKS = 2048;  // partial maxima of |U|^2 per step (one per umax workgroup)

struct DevState {
    double t, dt, t_next;
    long long step;
    double thrust, torque, power, cp, ct;
    double ibm_force[3];
    unsigned long long ibm_res_bits;
    double win_p, win_t;
    long long win_n;
    double mass, mom[3];
    unsigned long long umax_diag_bits;
    int nonfinite;
    int ibm_iters_used;
    int ibm_outside;  // a moving body's point support left the interior (sticky until new points)
};

struct GridDesc {
    int n[3];                 // interior cells x, y, z
    long long st[3];          // padded strides x, y, z
    long long pad0;           // padded offset of interior cell (0,0,0)
    long long n_padded;       // elements per padded field
    double h[3];              // mean cell size lx/nx, ... (the cell size of a uniform axis)
    double x0[3];
    const double* wrel[3];    // device, n[a]: cell width / h[a] of a stretched axis, null when uniform
};

template <typename real>
struct Field4 {
    real* v[4];
};

// host launchers (gks_stage.hip)
template <typename real>
hipError_t launch_face(const FaceArgs<real>& a, int stage, hipStream_t s);
template <typename real>
int face_chunk(int n_n, int tiles, int slots);
// order-5 face launches: the work split (FaceArgs seg_len, n_wg) for chunks of `chunk` cells
void face_plan(int n_n, int tiles, int slots, int chunk, int* seg_len, int* n_wg);
template <typename real>
int face_slots();
// second-order variant (gks_stage2.hip)
template <typename real>
hipError_t launch_face2(const FaceArgs<real>& a, int stage, hipStream_t s);
template <typename real>
int face2_slots();

// host launchers (gks_aux.hip)
template <typename real>
hipError_t launch_ghost(Field4<real> f, const GridDesc& g, int axis, int bc_lo, int bc_hi, const double u_in[3],
                        double c, double rho_ref, hipStream_t s);
template <typename real>
hipError_t launch_umax(Field4<real> f, const GridDesc& g, double rho_ref, double* part, hipStream_t s);
int umax_blocks(const GridDesc& g);
hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t s);
template <typename real>
hipError_t launch_transpose_xy(Field4<real> in, Field4<real> out, const GridDesc& g, hipStream_t s);
template <typename real>
hipError_t launch_ghost_transpose(Field4<real> q, Field4<real> qt, const GridDesc& gd, const int bc[6],
                                  const double u_in[3], double c, double rho_ref, hipStream_t s);
hipError_t launch_dt(DevState* st, const double* part, int nparts, double cfl, double hmin, double c,
                     double dt_fixed, hipStream_t s);
hipError_t launch_finish(DevState* st, int has_rotor, double* hist, hipStream_t s);
hipError_t launch_window_reset(DevState* st, hipStream_t s);
template <typename real>
hipError_t launch_diag(Field4<real> f, const real* lo, const GridDesc& g, double rho_ref, double* partials, int nblk,
                       DevState* st,
                       hipStream_t s);
int diag_blocks(const GridDesc& g);
hipError_t launch_copy_field(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace gks
