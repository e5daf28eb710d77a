// gks_stage.hip -- the S2O4 stage kernels: reconstruction, gas-kinetic flux, flux divergence and the
// stage combination, one launch per face direction (Section 2, Eqs. (semi), (finite), (x_example),
// (flux); the two-stage fourth-order combinations).
//
// One workgroup owns a tile of faces in the tangential plane (FP32: 16 x 16 faces, 512 threads = 8 wave64;
// FP64: 16 x 8 faces, 256 threads) and marches along the face normal through a chunk of faces (or
// through an equal share of the tile-major (tile, cell) order, one march per tile the share meets, when
// the tiles do not divide the resident workgroup slots: see face_plan):
//   * column phase: each of the 20 x 20 (FP64 20 x 12) tangential columns (tile + 2-cell halo per side) keeps a
//     5-cell window of the field in registers; per cell it evaluates the WENO-JS values at both of its
//     faces with one set of smoothness indicators, the normal derivative D (cubic through four cells)
//     and C = (q^L + q^R)/2 for all four variables -> LDS;
//   * t1 phase: WENO-JS at the two Gauss points of q^L, q^R, quartic Gauss values of D and C and the
//     quartic Gauss derivative of C along t1, the 4 x 320 (FP64 4 x 192) (variable, position) items spread
//     over all threads -> LDS;
//   * t2 phase: the same along t2 for each Gauss line, giving per Gauss point q^L, q^R, dQ/dn, dQ/dt1,
//     dQ/dt2 in registers (one thread per face and Gauss line);
//   * flux phase: closed-form flux per Gauss point, quadrature over the face, divergence against the
//     previous face of the column, and the accumulation (or the S2O4 epilogue in the last direction).
// No face flux is written to memory. FP32 runs the phases as a software pipeline over two LDS buffers
// (the face step of f, the t1 phase of f + 1 and the column phase of f + 2 between two barriers; 155 KB of
// the 160 KB per CU); FP64 runs them in turn with two barriers per face step (93 KB).
#include <algorithm>

#include "gks_internal.h"

namespace gks {

template <typename T>
__device__ __forceinline__ T pick(bool c, T x, T y) {
    return c ? x : y;
}

template <typename real>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

// The pair of variables (2m, 2m + 1) of cell i in an array that holds four variables per cell.
template <typename real>
__device__ __forceinline__ typename Vec2<real>::type ld2(const real* p, long long i, int m) {
    return *reinterpret_cast<const typename Vec2<real>::type*>(p + 4 * i + 2 * m);
}
template <typename real>
__device__ __forceinline__ void st2(real* p, long long i, int m, typename Vec2<real>::type v) {
    *reinterpret_cast<typename Vec2<real>::type*>(p + 4 * i + 2 * m) = v;
}

// Local index (the pass's variable order: density, normal momentum, t1, t2 momenta) of each global
// variable (density, x, y, z momenta) for the x (MODE 3), y (MODE 0) and z (MODE 4) passes.
template <int MODE>
struct LocalOrder;
template <>
struct LocalOrder<3> {
    static constexpr int v[4] = {0, 1, 2, 3};
};
template <>
struct LocalOrder<0> {
    static constexpr int v[4] = {0, 2, 1, 3};
};
template <>
struct LocalOrder<4> {
    static constexpr int v[4] = {0, 2, 3, 1};
};

// The value of the partner lane (lane ^ 1; all lanes are active where it is used). FP32, bound by VALU
// issue, moves it through the LDS crossbar (ds_bpermute), off the VALU; FP64, bound by latency at one
// wave per SIMD, takes it with a DPP quad permutation [1, 0, 3, 2] on the VALU, without the LDS round trip
// (with the crossbar the compiler waited for each value in turn).
__device__ __forceinline__ float pair_swap(float x) { return __shfl_xor(x, 1); }
__device__ __forceinline__ double pair_swap(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffu), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Error-free sum (Knuth): s + e == a + b exactly, s = fl(a + b).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// MODE (the direction's role): 3 = x pass, writes its residual to the blocked arrays; 0 = y pass,
// writes the main residual arrays; 4 = z pass, adds both and applies the S2O4 stage update.
// STR: the mesh is stretched and the spacings come from the per-axis arrays; otherwise the uniform
// inverse spacings are kernel arguments (no memory access for them inside the march).
template <typename real, int STAGE, int MODE, bool STR>
__global__ void __launch_bounds__(FaceTile<real>::THREADS) face_kernel(const FaceArgs<real> a) {
    static_assert(MODE == 0 || MODE == 3 || MODE == 4, "face pass mode");
    // tile of this precision: TILE1 x T2 faces, EXT1 x X2 columns, NTH threads
    constexpr int T2 = FaceTile<real>::T2, X2 = T2 + 4, NTH = FaceTile<real>::THREADS;
    static_assert(EXT1 * X2 <= NTH && 2 * TILE1 * T2 == NTH, "one thread per column and per face line");
    constexpr bool NEED_F0 = (STAGE == 1);
    // the z pass loads its epilogue operands at the top of the step, so that their latency overlaps the
    // step's arithmetic; FP32 also updates the compensated state (high part in the field, low part in
    // lo_in / lo_a / lo_b)
    constexpr bool EPI_PREFETCH = true;
    constexpr bool COMPENSATED = sizeof(real) == 4;
    using real2 = typename Vec2<real>::type;
    constexpr int LOC[4] = {LocalOrder<MODE>::v[0], LocalOrder<MODE>::v[1], LocalOrder<MODE>::v[2],
                            LocalOrder<MODE>::v[3]};
    // LDS: per variable, the column values [q^L, q^R, D, C][t2 row][t1 column] and the t1-phase results
    // [q^L_m, q^R_m, D_m, (dC/dt1)_m, C_m][t2 row][t1 position][Gauss line m]. A wave of the t1 phase takes
    // one row of all four variables, 16 consecutive positions each; the variable blocks are padded to
    // start 16 words apart modulo 64 (FP32; 32 in FP64, whose elements take two banks), so its reads
    // meet no bank twice, and the t1-phase results of the four variables start 32 words apart modulo 64
    // (FP32), the least the wave's 64-bit stores can share banks.
    // PAIR_PREV: the FP32 stage-1 z pass, which sits at the register limit, keeps only its lane's two
    // variables of the previous face's fluxes (the other passes keep all four: fewer selects per step).
    constexpr bool PAIR_PREV = (MODE == 4 && STAGE == 1 && sizeof(real) == 4);
    struct NrmV {
        real a[4][X2][EXT1];
        real pad[16];
    };
    struct T1V {
        real a[5][X2][TILE1][2];
        real pad[sizeof(real) == 4 ? 32 : 2];
    };
    // DB (FP32): two LDS buffers, so that the phases of consecutive faces overlap (FP64 has no room)
    constexpr bool DB = sizeof(real) == 4;
    constexpr int NB = DB ? 2 : 1;
    __shared__ NrmV s_nrm[NB][4];
    __shared__ T1V s_t1[NB][4];

    const int tid = threadIdx.x;
    // consecutive logical workgroups run on the same XCD (the hardware deals workgroups round-robin to
    // the 8 XCDs; the grid is padded to a multiple of 8), so neighbouring tiles share that XCD's L2 for
    // their halo columns
    const int b = (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8);
    if (b >= a.n_wg) return;
    // this workgroup's cells as a range [lin, lin_end) of the tile-major (tile, cell) order
    const int tiles = a.tiles_t1 * a.tiles_t2;
    long long lin, lin_end;
    if (a.seg_len > 0) {
        lin = (long long)b * a.seg_len;
        lin_end = min(lin + a.seg_len, (long long)tiles * a.n_n);
    } else {
        const int c0 = (b / tiles) * a.chunk;
        lin = (long long)(b % tiles) * a.n_n + c0;
        lin_end = lin + min(a.chunk, a.n_n - c0);
    }
    // one march per tile the range meets (the shift cm, the window and the face fluxes restart)
    while (lin < lin_end) {
    const int tile = (int)(lin / a.n_n);
    const int f0 = (int)(lin - (long long)tile * a.n_n);
    const int f1 = (int)min((long long)a.n_n, f0 + (lin_end - lin));  // residuals of cells [f0, f1); faces f0..f1
    lin += f1 - f0;
    const int tile1 = tile % a.tiles_t1, tile2 = tile / a.tiles_t1;
    const int j0 = tile1 * TILE1, k0 = tile2 * T2;
    const real eps = a.eps;

    // column role
    const bool col = tid < EXT1 * X2;
    const int c1 = tid % EXT1, c2 = tid / EXT1;
    const int jc = j0 - 2 + c1, kc = k0 - 2 + c2;
    const bool col_ld = col && (jc < a.n_t1 + NG) && (kc < a.n_t2 + NG);
    const long long cbase = a.pad0 + (long long)jc * a.st_t1 + (long long)kc * a.st_t2;
    // the in-loop prefetch of the column cells is done by every thread, columns outside the padded domain
    // and threads without a column reading a clamped column (its values are never used): a load on every
    // path leaves the compiler no merge of a loaded and a kept value, which would make it wait for the
    // load within the same step, and for the step's stores at the next one
    const long long cbase_ld = a.pad0 + (long long)min(jc, a.n_t1 + NG - 1) * a.st_t1 +
                               (long long)min(kc, a.n_t2 + NG - 1) * a.st_t2;
    // face role: face (fj, fk) of the tile, Gauss line m (partner lane tid ^ 1 holds the other line)
    const int m = tid & 1;
    const int fj = (tid >> 1) % TILE1, fk = (tid >> 1) / TILE1;
    const bool face_ok = (j0 + fj < a.n_t1) && (k0 + fk < a.n_t2);

    // FP32: inside the kernel the normal momentum is carried as its deviation from a workgroup constant
    // cm (the midrange of its values in the first window of the tile), so that the O(1) part of the
    // mass flux cancels exactly between the two faces of a cell and FP32 rounding acts on the deviation
    // only. The WENO and linear stencils commute with the shift (their weights sum to one and the
    // smoothness indicators use differences); the derivatives are unchanged.
    constexpr bool SHIFT = sizeof(real) == 4;
    real cm = real(0);
    real ring[4][5];
    real carry[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        carry[v] = real(0);
#pragma unroll
        for (int r = 0; r < 5; ++r) ring[v][r] = real(0);
    }
    // warm-up: window of cells f0-3 .. f0+1, then the right-face value of cell f0-1 (q^L of face f0)
    if (col_ld) {
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            const long long idx = cbase + (long long)(f0 - 3 + r) * a.st_n;
#pragma unroll
            for (int v = 0; v < 4; ++v) ring[v][r] = a.q[v][idx];
        }
    }
    if constexpr (SHIFT) {
        __shared__ float s_range[2][NTH / 64];
        float lo = col_ld ? float(ring[1][0]) : 3.0e38f, up = col_ld ? float(ring[1][0]) : -3.0e38f;
#pragma unroll
        for (int r = 1; r < 5; ++r) {
            lo = col_ld ? fminf(lo, float(ring[1][r])) : lo;
            up = col_ld ? fmaxf(up, float(ring[1][r])) : up;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo = fminf(lo, __shfl_xor(lo, o));
            up = fmaxf(up, __shfl_xor(up, o));
        }
        if ((tid & 63) == 0) {
            s_range[0][tid >> 6] = lo;
            s_range[1][tid >> 6] = up;
        }
        __syncthreads();
        lo = s_range[0][0];
        up = s_range[1][0];
#pragma unroll
        for (int w = 1; w < NTH / 64; ++w) {
            lo = fminf(lo, s_range[0][w]);
            up = fmaxf(up, s_range[1][w]);
        }
        cm = lo <= up ? real(0.5f * (lo + up)) : real(0);
#pragma unroll
        for (int r = 0; r < 5; ++r) ring[1][r] -= cm;
    }
    if (col_ld) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            real right, left;
            weno_faces<real>(ring[v][0], ring[v][1], ring[v][2], ring[v][3], ring[v][4], eps, right, left);
            carry[v] = right;
        }
    }
    // software pipelining: the cell entering the window at the next step is loaded one step ahead
    real nxt[4] = {real(0), real(0), real(0), real(0)};
    if (col_ld) {
        const long long idx = cbase + (long long)(f0 + 2) * a.st_n;
#pragma unroll
        for (int v = 0; v < 4; ++v) nxt[v] = a.q[v][idx];
    }
    const real dt = real(*a.dt_ptr);
    // the previous face's fluxes: all four variables, or (PAIR_PREV) only this lane's two
    real fprev0[4] = {0, 0, 0, 0}, fprev1[4] = {0, 0, 0, 0};
    real2 pprev0 = {0, 0}, pprev1 = {0, 0};

    const bool hi = m != 0;
    // tangential inverse widths, loaded once (a vector load inside the march would make the wait for
    // it also wait for the column prefetch): t2 of this thread's face line; t1 of its t1-phase items,
    // whose t1 position is tid % TILE1 for every item
    const real ih2 = STR ? a.ih2[min(k0 + fk, a.n_t2 - 1)] : a.inv_h2;
    const real ih1 = STR ? a.ih1[min(j0 + tid % TILE1, a.n_t1 - 1)] : a.inv_h1;
    // epilogue operands (z pass) of cell f - 1
    struct Epi {
        real2 r0, r1, x0, x1, lo;
        real q[2];
    };
    auto epi_load = [&](int f, Epi& ep) {
        if constexpr (EPI_PREFETCH && MODE == 4) {
            // loaded on every path (for the same reason as the column prefetch): at f = f0, one face past
            // the march and for faces outside the domain a clamped cell is read and its values are not used
            const int cell = min(max(f - 1, 0), a.n_n - 1), je = min(j0 + fj, a.n_t1 - 1), ke = min(k0 + fk, a.n_t2 - 1);
            const long long ridx = (long long)cell * a.ist_n + (long long)je * a.ist_t1 + (long long)ke * a.ist_t2;
            const long long pidx = a.pad0 + (long long)cell * a.st_n + (long long)je * a.st_t1 + (long long)ke * a.st_t2;
            const long long xidx = rx_block_index(je, ke, cell, a.rx_nx, a.rx_nyb);
            ep.r1 = ld2(a.r1, ridx, m);
            ep.x1 = ld2(a.rx1, xidx, m);
            if (COMPENSATED) ep.lo = ld2(a.lo_in, ridx, m);
            if (NEED_F0) {
                ep.r0 = ld2(a.r0, ridx, m);
                ep.x0 = ld2(a.rx0, xidx, m);
            }
#pragma unroll
            for (int vv = 0; vv < 2; ++vv) {
                const real* const src = NEED_F0 ? pick(hi, a.q_c[LOC[2 + vv]], a.q_c[LOC[vv]])
                                                : pick(hi, a.s_in[LOC[2 + vv]], a.s_in[LOC[vv]]);
                ep.q[vv] = src[pidx];
            }
        }
    };
    // column phase of face f into LDS buffer buf
    auto column_step = [&](int f, int buf) {
        const real ihf_f = STR ? a.ihf[f] : a.inv_hn;  // inverse spacing at face f (normal derivative)
        // ---- column phase (all variables): window cells f-2 .. f+2, prefetch cell f+3
        if (col) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
#pragma unroll
                for (int r = 0; r < 4; ++r) ring[v][r] = ring[v][r + 1];
                // the shift is applied here, a step after the load, so that the prefetch stays in flight
                ring[v][4] = (SHIFT && v == 1) ? nxt[v] - cm : nxt[v];
            }
        }
        {
            const long long idx = cbase_ld + (long long)min(f + 3, a.n_n + 2) * a.st_n;
#pragma unroll
            for (int v = 0; v < 4; ++v) nxt[v] = a.q[v][idx];
        }
        if (col) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                real right, left;
                weno_faces<real>(ring[v][0], ring[v][1], ring[v][2], ring[v][3], ring[v][4], eps, right, left);
                const real qL = carry[v];
                const real D = (ring[v][0] - real(15) * ring[v][1] + real(15) * ring[v][2] - ring[v][3]) *
                               (real(1.0 / 12.0) * ihf_f);
                s_nrm[buf][v].a[0][c2][c1] = qL;
                s_nrm[buf][v].a[1][c2][c1] = left;
                s_nrm[buf][v].a[2][c2][c1] = D;
                s_nrm[buf][v].a[3][c2][c1] = real(0.5) * (qL + left);
                carry[v] = right;
            }
        }
    };
    // t1 phase of LDS buffer buf
    auto t1_step = [&](int buf) {
        // ---- t1 phase: the 4 x 16 x X2 items (variable v, t2 row tk, t1 position tj) spread over all
        // threads in row-wave order: a thread keeps tj = tid % 16 and v = tid / 16 % 4 and takes the rows
        // tid / 64 + k NTH / 64, so its LDS addresses move by a fixed step (no index arithmetic in the
        // march)
        static_assert(TILE1 == 16 && NTH % 64 == 0, "t1 items: 16 positions x 4 variables per wave");
        {
            constexpr int RSTEP = NTH / 64, NK = (X2 + RSTEP - 1) / RSTEP;
            const int tj = tid & 15, v = (tid >> 4) & 3;
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) {
                const int tk = (tid >> 6) + kk * RSTEP;
                if (X2 % RSTEP == 0 || tk < X2) {
                    real x[4][5];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int r = 0; r < 5; ++r) x[q][r] = s_nrm[buf][v].a[q][tk][tj + r];
                    real vm, vp;
                    weno_gauss<real>(x[0][0], x[0][1], x[0][2], x[0][3], x[0][4], eps, vm, vp);
                    s_t1[buf][v].a[0][tk][tj][0] = vm;
                    s_t1[buf][v].a[0][tk][tj][1] = vp;
                    weno_gauss<real>(x[1][0], x[1][1], x[1][2], x[1][3], x[1][4], eps, vm, vp);
                    s_t1[buf][v].a[1][tk][tj][0] = vm;
                    s_t1[buf][v].a[1][tk][tj][1] = vp;
                    quartic_gauss_value<real>(x[2][0], x[2][1], x[2][2], x[2][3], x[2][4], vm, vp);
                    s_t1[buf][v].a[2][tk][tj][0] = vm;
                    s_t1[buf][v].a[2][tk][tj][1] = vp;
                    quartic_gauss_deriv<real>(x[3][0], x[3][1], x[3][2], x[3][3], x[3][4], vm, vp);
                    s_t1[buf][v].a[3][tk][tj][0] = vm * ih1;
                    s_t1[buf][v].a[3][tk][tj][1] = vp * ih1;
                    quartic_gauss_value<real>(x[3][0], x[3][1], x[3][2], x[3][3], x[3][4], vm, vp);
                    s_t1[buf][v].a[4][tk][tj][0] = vm;
                    s_t1[buf][v].a[4][tk][tj][1] = vp;
                }
            }
        }
    };
    // t2 phase, flux and residual (or stage update) of face f from LDS buffer buf
    auto face_step = [&](int f, int buf, const Epi& ep) {
        // ---- t2 phase: per thread one face and one Gauss line, all variables
        real gp[4][2][5];  // [variable][Gauss n][q^L, q^R, d/dn, d/dt1, d/dt2]
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            real y[5][5];
#pragma unroll
            for (int q = 0; q < 5; ++q)
#pragma unroll
                for (int r = 0; r < 5; ++r) y[q][r] = s_t1[buf][v].a[q][fk + r][fj][m];
            real vm, vp;
            weno_gauss<real>(y[0][0], y[0][1], y[0][2], y[0][3], y[0][4], eps, vm, vp);
            gp[v][0][0] = vm;
            gp[v][1][0] = vp;
            weno_gauss<real>(y[1][0], y[1][1], y[1][2], y[1][3], y[1][4], eps, vm, vp);
            gp[v][0][1] = vm;
            gp[v][1][1] = vp;
            quartic_gauss_value<real>(y[2][0], y[2][1], y[2][2], y[2][3], y[2][4], vm, vp);
            gp[v][0][2] = vm;
            gp[v][1][2] = vp;
            quartic_gauss_value<real>(y[3][0], y[3][1], y[3][2], y[3][3], y[3][4], vm, vp);
            gp[v][0][3] = vm;
            gp[v][1][3] = vp;
            quartic_gauss_deriv<real>(y[4][0], y[4][1], y[4][2], y[4][3], y[4][4], vm, vp);
            gp[v][0][4] = vm * ih2;
            gp[v][1][4] = vp * ih2;
        }

        // ---- flux at this thread's two Gauss points, quadrature weight 1/4 each
        real fa0[4] = {0, 0, 0, 0}, fa1[4] = {0, 0, 0, 0};
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            real qL[4], qR[4], g[3][4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                qL[v] = gp[v][n][0];
                qR[v] = gp[v][n][1];
                g[0][v] = gp[v][n][2];
                g[1][v] = gp[v][n][3];
                g[2][v] = gp[v][n][4];
            }
            gp_flux<real, NEED_F0, SHIFT>(qL, qR, g, a.fc, real(0.25), fa0, fa1, cm);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            fa1[v] += pair_swap(fa1[v]);
            if (NEED_F0) fa0[v] += pair_swap(fa0[v]);
        }
        // this lane's two variables of the face fluxes: global variables 2m and 2m + 1, local indices
        // LOC[2m], LOC[2m + 1], picked by value with a per-lane select between compile-time indices
        // (indexing a register array with the lane-dependent index would move it to scratch)
        auto lane_pair = [&](const real (&x)[4]) -> real2 {
            real2 r;
            r.x = pick(hi, x[LOC[2]], x[LOC[0]]);
            r.y = pick(hi, x[LOC[3]], x[LOC[1]]);
            return r;
        };
        const real2 fcur1 = lane_pair(fa1);
        const real2 fcur0 = NEED_F0 ? lane_pair(fa0) : real2{0, 0};
        if (f > f0 && face_ok) {
            const int cell = f - 1;
            const long long ridx = (long long)cell * a.ist_n + (long long)(j0 + fj) * a.ist_t1 +
                                   (long long)(k0 + fk) * a.ist_t2;
            const long long pidx = a.pad0 + (long long)cell * a.st_n + (long long)(j0 + fj) * a.st_t1 +
                                   (long long)(k0 + fk) * a.st_t2;
            // lane m owns the global variables 2m and 2m + 1 (local indices LOC[2m], LOC[2m + 1]); the
            // residual and low-order arrays hold the four variables of a cell together, so the lane moves
            // them as one pair. Per-variable pointers and values are picked by value with a per-lane select
            // between compile-time indices: indexing the argument or register arrays with the
            // lane-dependent index would fetch pointers from memory and move the arrays to scratch.
            real2 d1, d0;
            const real ihc = STR ? a.ihc[cell] : a.inv_hn;
            const real2 prev1 = PAIR_PREV ? pprev1 : lane_pair(fprev1);
            d1.x = -(fcur1.x - prev1.x) * ihc;
            d1.y = -(fcur1.y - prev1.y) * ihc;
            if (NEED_F0) {
                const real2 prev0 = PAIR_PREV ? pprev0 : lane_pair(fprev0);
                d0.x = -(fcur0.x - prev0.x) * ihc;
                d0.y = -(fcur0.y - prev0.y) * ihc;
            } else {
                d0.x = d0.y = real(0);
            }
            if constexpr (MODE == 3) {
                const long long xidx = rx_block_index(cell, j0 + fj, k0 + fk, a.rx_nx, a.rx_nyb);
                st2(a.rx1, xidx, m, d1);
                if (NEED_F0) st2(a.rx0, xidx, m, d0);
            } else if constexpr (MODE == 0) {
                st2(a.r1, ridx, m, d1);
                if (NEED_F0) st2(a.r0, ridx, m, d0);
            } else {
                real2 r1v, x1v, r0v = {0, 0}, x0v = {0, 0};
                if constexpr (EPI_PREFETCH) {
                    r1v = ep.r1;
                    x1v = ep.x1;
                    r0v = ep.r0;
                    x0v = ep.x0;
                } else {
                    const long long xidx = rx_block_index(j0 + fj, k0 + fk, cell, a.rx_nx, a.rx_nyb);
                    r1v = ld2(a.r1, ridx, m);
                    x1v = ld2(a.rx1, xidx, m);
                    if (NEED_F0) {
                        r0v = ld2(a.r0, ridx, m);
                        x0v = ld2(a.rx0, xidx, m);
                    }
                }
                const real L1[2] = {r1v.x + (d1.x + x1v.x), r1v.y + (d1.y + x1v.y)};
                const real L0[2] = {r0v.x + (d0.x + x0v.x), r0v.y + (d0.y + x0v.y)};
                if constexpr (COMPENSATED) {
                    // FP32: the state is carried as hi + lo; each update is an error-free sum of the
                    // stored high part and (low part + increment)
                    const real lo[2] = {ep.lo.x, ep.lo.y};
                    real2 la = {0, 0}, lb = {0, 0};
#pragma unroll
                    for (int vv = 0; vv < 2; ++vv) {
                        real* const outa = pick(hi, a.out_a[LOC[2 + vv]], a.out_a[LOC[vv]]);
                        float sh, sl;
                        if (NEED_F0) {
                            real* const outb = pick(hi, a.out_b[LOC[2 + vv]], a.out_b[LOC[vv]]);
                            two_sum(ep.q[vv], lo[vv] + (real(0.5) * dt * L0[vv] + real(0.125) * dt * dt * L1[vv]), sh, sl);
                            outa[pidx] = sh;
                            if (vv == 0) la.x = sl; else la.y = sl;
                            two_sum(ep.q[vv], lo[vv] + (dt * L0[vv] + (dt * dt * real(1.0 / 6.0)) * L1[vv]), sh, sl);
                            outb[pidx] = sh;
                            if (vv == 0) lb.x = sl; else lb.y = sl;
                        } else {
                            // body force G on the momenta (global variables 1..3)
                            const real gv = pick(hi, a.g_global[1 + vv], vv == 1 ? a.g_global[0] : real(0));
                            const real add = (dt * dt * real(1.0 / 3.0)) * L1[vv] + dt * gv;
                            two_sum(ep.q[vv], lo[vv] + add, sh, sl);
                            outa[pidx] = sh;
                            if (vv == 0) la.x = sl; else la.y = sl;
                        }
                    }
                    st2(a.lo_a, ridx, m, la);
                    if (NEED_F0) st2(a.lo_b, ridx, m, lb);
                } else {
                    // FP64: the plain stage update from the prefetched Q^n (stage 1) or S (stage 2)
#pragma unroll
                    for (int vv = 0; vv < 2; ++vv) {
                        real* const outa = pick(hi, a.out_a[LOC[2 + vv]], a.out_a[LOC[vv]]);
                        if (NEED_F0) {
                            const real Q = ep.q[vv];
                            real* const outb = pick(hi, a.out_b[LOC[2 + vv]], a.out_b[LOC[vv]]);
                            outa[pidx] = Q + real(0.5) * dt * L0[vv] + real(0.125) * dt * dt * L1[vv];
                            outb[pidx] = Q + dt * L0[vv] + (dt * dt * real(1.0 / 6.0)) * L1[vv];
                        } else {
                            const real gv = pick(hi, a.g_global[1 + vv], vv == 1 ? a.g_global[0] : real(0));
                            const real add = (dt * dt * real(1.0 / 3.0)) * L1[vv] + dt * gv;
                            outa[pidx] = ep.q[vv] + add;
                        }
                    }
                }
            }
        }
        if constexpr (PAIR_PREV) {
            pprev1 = fcur1;
            if (NEED_F0) pprev0 = fcur0;
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                fprev1[v] = fa1[v];
                if (NEED_F0) fprev0[v] = fa0[v];
            }
        }
    };
    if constexpr (DB) {
        // software pipeline over two LDS buffers with one barrier per face: the face step of f reads
        // s_t1[buf], the t1 phase of f + 1 reads s_nrm[buf ^ 1] and writes s_t1[buf ^ 1], the column
        // phase of f + 2 writes s_nrm[buf]; each buffer was last read or written before the previous
        // barrier. The epilogue operands of the next face step are loaded one step ahead. Waves whose
        // column phase is light (400 columns on 512 threads) go on to the next face's work.
        Epi ep = {};
        epi_load(f0, ep);
        column_step(f0, 0);
        __syncthreads();
        t1_step(0);
        column_step(f0 + 1, 1);
        __syncthreads();
        for (int f = f0; f <= f1; ++f) {
            const int buf = (f - f0) & 1;
            face_step(f, buf, ep);
            epi_load(f + 1, ep);
            if (f + 1 <= f1) t1_step(buf ^ 1);
            if (f + 2 <= f1) column_step(f + 2, buf);
            __syncthreads();
        }
    } else {
        for (int f = f0; f <= f1; ++f) {
            Epi ep = {};
            epi_load(f, ep);
            column_step(f, 0);
            __syncthreads();
            t1_step(0);
            __syncthreads();
            face_step(f, 0, ep);
        }
    }
    }  // segments
}

template <typename real>
int face_slots() {
    // workgroups of the face kernel that the device holds at once
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, face_kernel<real, 1, 4, false>, FaceTile<real>::THREADS,
                                                     0) != hipSuccess)
        return 0;
    return cus * per_cu;
}

template <typename real>
int face_chunk(int n_n, int tiles, int slots) {
    // Workgroups of one launch run in rounds of `slots`; a workgroup costs about (chunk + 2) face steps
    // (chunk + 1 faces, and the column phase primes five planes before the first one). Pick the chunk
    // that minimises rounds x (chunk + 2); ties go to the longer chunk.
    if (slots <= 0) slots = 512;
    int best_chunk = n_n;
    long long best = -1;
    for (int nc = 1; nc <= n_n; ++nc) {
        const int chunk = (n_n + nc - 1) / nc;
        const long long wgs = (long long)tiles * ((n_n + chunk - 1) / chunk);
        const long long cost = ((wgs + slots - 1) / slots) * (chunk + 2);
        if (best < 0 || cost < best) {
            best = cost;
            best_chunk = chunk;
        }
    }
    return best_chunk;
}

void face_plan(int n_n, int tiles, int slots, int chunk, int* seg_len, int* n_wg) {
    // Worst workgroup of each split, in face steps (a march over L cells costs about L + 2), times the
    // rounds of `slots` workgroups: aligned chunks of `chunk` cells, or equal runs of the tile-major
    // (tile, cell) order, whose workgroups fill the slots when the tiles do not divide them but pay a
    // second march where a run crosses into the next tile. The cheaper wins; ties go to the chunks.
    if (slots <= 0) slots = 512;
    const long long nch = (n_n + chunk - 1) / chunk;
    const long long wg_c = (long long)tiles * nch;
    long long best = ((wg_c + slots - 1) / slots) * (chunk + 2);
    *seg_len = 0;
    *n_wg = (int)wg_c;
    const long long total = (long long)tiles * n_n;
    for (long long rounds = 1; rounds <= 8; ++rounds) {
        const long long len = (total + rounds * slots - 1) / (rounds * slots);
        const long long wgs = (total + len - 1) / len;
        long long worst = 0;
        for (long long w = 0; w < wgs; ++w) {
            const long long c0 = w * len, c1 = std::min(c0 + len, total);
            const long long segs = (c1 - 1) / n_n - c0 / n_n + 1;
            worst = std::max(worst, (c1 - c0) + 2 * segs);
        }
        const long long cost = ((wgs + slots - 1) / slots) * worst;
        if (cost < best && wgs <= 0x7ffffff8LL) {
            best = cost;
            *seg_len = (int)len;
            *n_wg = (int)wgs;
        }
        if (len == 1) break;
    }
}

template <typename real>
hipError_t launch_face(const FaceArgs<real>& a, int stage, hipStream_t s) {
    const long long blocks = ((long long)a.n_wg + 7) / 8 * 8;
    if (a.n_wg <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(FaceTile<real>::THREADS);
#define GKS_FACE_LAUNCH(ST, MD)                                                                     \
    do {                                                                                            \
        if (a.stretched) hipLaunchKernelGGL((face_kernel<real, ST, MD, true>), grid, block, 0, s, a);  \
        else hipLaunchKernelGGL((face_kernel<real, ST, MD, false>), grid, block, 0, s, a);             \
    } while (0)
    if (stage == 1) {
        if (a.mode == 0) GKS_FACE_LAUNCH(1, 0);
        else if (a.mode == 3) GKS_FACE_LAUNCH(1, 3);
        else if (a.mode == 4) GKS_FACE_LAUNCH(1, 4);
        else return hipErrorInvalidValue;
    } else {
        if (a.mode == 0) GKS_FACE_LAUNCH(2, 0);
        else if (a.mode == 3) GKS_FACE_LAUNCH(2, 3);
        else if (a.mode == 4) GKS_FACE_LAUNCH(2, 4);
        else return hipErrorInvalidValue;
    }
#undef GKS_FACE_LAUNCH
    return hipGetLastError();
}

template hipError_t launch_face<float>(const FaceArgs<float>&, int, hipStream_t);
template hipError_t launch_face<double>(const FaceArgs<double>&, int, hipStream_t);
template int face_chunk<float>(int, int, int);
template int face_chunk<double>(int, int, int);
template int face_slots<float>();
template int face_slots<double>();

}  // namespace gks
