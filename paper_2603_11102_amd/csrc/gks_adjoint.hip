// gks_adjoint.hip -- discrete adjoint of the S2O4 step (FP64) with the actuator-line body force, for
// the gradient of a rotor objective with respect to per-point force scalings.
//
// Forward operator per face direction (Section 2): normal WENO/derivative reconstruction ->
// t1 Gauss-point sweep -> t2 Gauss-point sweep -> gas-kinetic flux at the 2x2 Gauss points ->
// face quadrature and divergence. Its transpose is applied pass by pass in gather form (each output
// is one thread summing a fixed list of terms), with the WENO nonlinear weights frozen at their
// forward values; every other operation is linearised exactly. No atomics are used, so gradients are
// bitwise reproducible.
#include <algorithm>
#include <type_traits>

#include "gks_adjoint.h"

namespace gks {

namespace {

__device__ __forceinline__ long long face_ix(const AdjFaceArgs& a, int f, int j, int k) {
    return ((long long)f * a.n_t2 + k) * a.n_t1 + j;
}
__device__ __forceinline__ long long t1_ix(const AdjFaceArgs& a, int f, int j, int kx) {
    return ((long long)f * (a.n_t2 + 4) + (kx + 2)) * a.n_t1 + j;
}
__device__ __forceinline__ long long n_ix(const AdjFaceArgs& a, int f, int jx, int kx) {
    return ((long long)f * (a.n_t2 + 4) + (kx + 2)) * (a.n_t1 + 4) + (jx + 2);
}

// Coefficients of one WENO evaluation on `side` (stencil q, nonlinear weights w, value v): the frozen
// weights w0 and w2 (w1 = 1 - w0 - w2 is rebuilt where they are used) or (EXACT) the Jacobian row.
template <bool EXACT>
__device__ __forceinline__ void weno_coefs(int side, const double q[5], double eps, const double w[3], double v,
                                           double* out) {
    if constexpr (EXACT) {
        weno_jacobian(side, q, eps, w, v, out);
    } else {
        out[0] = w[0];
        out[1] = w[2];
    }
}

// Coefficient of stencil cell r in a WENO evaluation on `side` from its coefficients: the frozen weights
// expanded over the sub-stencils, or (EXACT) the Jacobian entry.
template <bool EXACT>
__device__ __forceinline__ double wcoef(int side, const double* c, int r) {
    if constexpr (EXACT) {
        return c[r];
    } else {
        const double w[3] = {c[0], 1.0 - c[0] - c[1], c[1]};
        return weno_eff(side, w, r);
    }
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// pass A: recompute the face pipeline of one direction (the forward's 16 x 8 face tiles of 256 threads,
// one wave per SIMD so that the FP64 state fits the unified register file), store the inputs of the
// tangential WENO evaluations (normal face values, t1 line values) and, per face and Gauss point, the
// adjoints of the Gauss-point inputs from the reverse of the flux (seeds Fbar(f) = (mu(f) - mu(f-1)) / h)
// ------------------------------------------------------------------------------------------------
template <int STAGE>
__global__ void __launch_bounds__(FaceTile<double>::THREADS) adj_face_kernel(const AdjFaceArgs a) {
    constexpr bool NEED_F0 = (STAGE == 1);
    constexpr int T2 = FaceTile<double>::T2, X2 = T2 + 4, NTH = FaceTile<double>::THREADS;
    static_assert(EXT1 * X2 <= NTH && 2 * TILE1 * T2 == NTH && TILE1 * X2 <= NTH, "thread roles");
    __shared__ double s_nrm[4][X2][EXT1];
    __shared__ double s_t1[5][X2][TILE1][2];
    // Gauss-point states of each thread's face line: [(variable * 2 + Gauss point) * 5 + quantity][thread]
    __shared__ double s_gp[40][NTH];

    const int tid = threadIdx.x;
    // consecutive logical workgroups on the same XCD (grid padded to a multiple of 8), as in the forward
    int b = (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8);
    if (b >= a.tiles_t1 * a.tiles_t2 * ((a.n_n + a.chunk - 1) / a.chunk)) return;
    const int tile1 = b % a.tiles_t1;
    b /= a.tiles_t1;
    const int tile2 = b % a.tiles_t2;
    b /= a.tiles_t2;
    const int f0 = b * a.chunk;
    const int f1 = min(f0 + a.chunk, a.n_n);
    const int j0 = tile1 * TILE1, k0 = tile2 * T2;
    const double eps = a.eps;

    const bool col = tid < EXT1 * X2;
    const int c1 = tid % EXT1, c2 = tid / EXT1;
    const int jc = j0 - 2 + c1, kc = k0 - 2 + c2;
    const bool col_ld = col && (jc < a.n_t1 + NG) && (kc < a.n_t2 + NG);
    const bool col_st = col && (jc < a.n_t1 + 2) && (kc < a.n_t2 + 2);
    const long long cbase = a.pad0 + (long long)jc * a.st_t1 + (long long)kc * a.st_t2;
    const bool t1r = tid < TILE1 * X2;
    const int tj = tid % TILE1, tk = tid / TILE1;
    const bool t1_st = t1r && (j0 + tj < a.n_t1) && (k0 - 2 + tk < a.n_t2 + 2);
    const int m = tid & 1;
    const int fj = (tid >> 1) % TILE1, fk = (tid >> 1) / TILE1;
    const bool face_ok = (j0 + fj < a.n_t1) && (k0 + fk < a.n_t2);

    double ring[4][5];
    double carry[4];
    for (int v = 0; v < 4; ++v) {
        carry[v] = 0.0;
        for (int r = 0; r < 5; ++r) ring[v][r] = 0.0;
    }
    if (col_ld) {
        for (int r = 0; r < 5; ++r) {
            const long long idx = cbase + (long long)(f0 - 3 + r) * a.st_n;
            for (int v = 0; v < 4; ++v) ring[v][r] = a.q[v][idx];
        }
        for (int v = 0; v < 4; ++v) {
            double right, left, wr[3], wl[3];
            weno_faces_w<double>(ring[v][0], ring[v][1], ring[v][2], ring[v][3], ring[v][4], eps, right, left, wr, wl);
            carry[v] = right;
        }
    }

    // the next cell of the column is loaded one step ahead, by every thread (columns outside the padded
    // domain and threads without a column read a clamped column whose values only reach faces outside
    // the domain): a load on every path needs no merge that would wait for it within the step
    const long long cbase_ld = a.pad0 + (long long)min(jc, a.n_t1 + NG - 1) * a.st_t1 +
                               (long long)min(kc, a.n_t2 + NG - 1) * a.st_t2;
    double nxt[4];
    for (int v = 0; v < 4; ++v) nxt[v] = a.q[v][cbase_ld + (long long)min(f0 + 2, a.n_n + 2) * a.st_n];
    // inverse spacings: t1 width of this thread's tangential-line cell, t2 width of its face cell, and
    // (per face, fetched one face ahead) the normal face spacing and the widths of the two cells
    // sharing the face (clamped at the ends, where the terms they scale vanish)
    const double ih1 = a.ih1[min(j0 + tj, a.n_t1 - 1)], ih2 = a.ih2[min(k0 + fk, a.n_t2 - 1)];
    double ihf_nxt = a.ihf[f0], ihc_nxt = a.ihc[min(f0, a.n_n - 1)], ihc_lo = a.ihc[max(f0 - 1, 0)];
    for (int f = f0; f <= f1; ++f) {
        for (int v = 0; v < 4; ++v) {
            for (int r = 0; r < 4; ++r) ring[v][r] = ring[v][r + 1];
            ring[v][4] = nxt[v];
        }
        const double ihf = ihf_nxt, ihc_hi = ihc_nxt;
        ihf_nxt = a.ihf[min(f + 1, a.n_n)];
        ihc_nxt = a.ihc[min(f + 1, a.n_n - 1)];
        {
            const long long idx = cbase_ld + (long long)min(f + 3, a.n_n + 2) * a.st_n;
            for (int v = 0; v < 4; ++v) nxt[v] = a.q[v][idx];
        }
        // column phase of one variable; v is a compile-time constant so that ring stays in registers
        auto column = [&](auto vc) {
            constexpr int v = decltype(vc)::value;
            if (col) {
                double right, left, wr[3], wl[3];
                weno_faces_w<double>(ring[v][0], ring[v][1], ring[v][2], ring[v][3], ring[v][4], eps, right, left,
                                     wr, wl);
                const double qL = carry[v];
                const double D = (ring[v][0] - 15.0 * ring[v][1] + 15.0 * ring[v][2] - ring[v][3]) * (ihf / 12.0);
                s_nrm[0][c2][c1] = qL;
                s_nrm[1][c2][c1] = left;
                s_nrm[2][c2][c1] = D;
                s_nrm[3][c2][c1] = 0.5 * (qL + left);
                carry[v] = right;
                if (col_st) {
                    // the inputs of the t1 WENO evaluations (pass C rebuilds their coefficients)
                    const long long p = n_ix(a, f, jc, kc);
                    a.fv[(v * 2 + 0) * a.nnpos + p] = qL;
                    a.fv[(v * 2 + 1) * a.nnpos + p] = left;
                }
            }
        };

        auto put = [&](int v, int n, int q, double val) { s_gp[(v * 2 + n) * 5 + q][tid] = val; };
        column(std::integral_constant<int, 0>{});
        __syncthreads();
        for (int v = 0; v < 4; ++v) {
            if (t1r) {
                double x[4][5];
                for (int q = 0; q < 4; ++q)
                    for (int r = 0; r < 5; ++r) x[q][r] = s_nrm[q][tk][tj + r];
                double vm, vp, wm[3], wp[3];
                const long long p = t1_st ? t1_ix(a, f, j0 + tj, k0 - 2 + tk) : 0;
                for (int side = 0; side < 2; ++side) {
                    weno_gauss_w<double>(x[side][0], x[side][1], x[side][2], x[side][3], x[side][4], eps, vm, vp, wm, wp);
                    s_t1[side][tk][tj][0] = vm;
                    s_t1[side][tk][tj][1] = vp;
                    if (t1_st) {
                        // the inputs of the t2 WENO evaluations (pass B rebuilds their coefficients)
                        a.t1v[((v * 2 + side) * 2 + 0) * a.nt1pos + p] = vm;
                        a.t1v[((v * 2 + side) * 2 + 1) * a.nt1pos + p] = vp;
                    }
                }
                quartic_gauss_value<double>(x[2][0], x[2][1], x[2][2], x[2][3], x[2][4], vm, vp);
                s_t1[2][tk][tj][0] = vm;
                s_t1[2][tk][tj][1] = vp;
                quartic_gauss_deriv<double>(x[3][0], x[3][1], x[3][2], x[3][3], x[3][4], vm, vp);
                s_t1[3][tk][tj][0] = vm * ih1;
                s_t1[3][tk][tj][1] = vp * ih1;
                quartic_gauss_value<double>(x[3][0], x[3][1], x[3][2], x[3][3], x[3][4], vm, vp);
                s_t1[4][tk][tj][0] = vm;
                s_t1[4][tk][tj][1] = vp;
            }
            __syncthreads();
            {
                double y[5][5];
                for (int q = 0; q < 5; ++q)
                    for (int r = 0; r < 5; ++r) y[q][r] = s_t1[q][fk + r][fj][m];
                double vm, vp, wm[3], wp[3];
                for (int side = 0; side < 2; ++side) {
                    weno_gauss_w<double>(y[side][0], y[side][1], y[side][2], y[side][3], y[side][4], eps, vm, vp, wm, wp);
                    put(v, 0, side, vm);
                    put(v, 1, side, vp);
                }
                quartic_gauss_value<double>(y[2][0], y[2][1], y[2][2], y[2][3], y[2][4], vm, vp);
                put(v, 0, 2, vm);
                put(v, 1, 2, vp);
                quartic_gauss_value<double>(y[3][0], y[3][1], y[3][2], y[3][3], y[3][4], vm, vp);
                put(v, 0, 3, vm);
                put(v, 1, 3, vp);
                quartic_gauss_deriv<double>(y[4][0], y[4][1], y[4][2], y[4][3], y[4][4], vm, vp);
                put(v, 0, 4, vm * ih2);
                put(v, 1, 4, vp * ih2);
            }
            switch (v) {
                case 0: column(std::integral_constant<int, 1>{}); break;
                case 1: column(std::integral_constant<int, 2>{}); break;
                case 2: column(std::integral_constant<int, 3>{}); break;
                default: break;
            }
            __syncthreads();
        }

        // reverse of the flux at this thread's two Gauss points: the adjoints of their inputs go to the
        // gpbar slots of this face
        if (face_ok) {
            const long long fi = face_ix(a, f, j0 + fj, k0 + fk);
            const long long jk = (long long)(j0 + fj) * a.ist_t1 + (long long)(k0 + fk) * a.ist_t2;
            double b0[4], b1[4];
            for (int v = 0; v < 4; ++v) {
                const double hi1 = f < a.n_n ? a.mu1[v][(long long)f * a.ist_n + jk] : 0.0;
                const double lo1 = f >= 1 ? a.mu1[v][(long long)(f - 1) * a.ist_n + jk] : 0.0;
                // Fbar(f) = mu(f) / w_f - mu(f-1) / w_{f-1} (cell widths w)
                b1[v] = hi1 * ihc_hi - lo1 * ihc_lo;
                if (NEED_F0) {
                    const double hi0 = f < a.n_n ? a.mu0[v][(long long)f * a.ist_n + jk] : 0.0;
                    const double lo0 = f >= 1 ? a.mu0[v][(long long)(f - 1) * a.ist_n + jk] : 0.0;
                    b0[v] = hi0 * ihc_hi - lo0 * ihc_lo;
                } else {
                    b0[v] = 0.0;
                }
            }
            for (int n = 0; n < 2; ++n) {
                double qL[4], qR[4], g[3][4], qLb[4] = {0, 0, 0, 0}, qRb[4] = {0, 0, 0, 0};
                double gb[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
                for (int v = 0; v < 4; ++v) {
                    const int q0 = (v * 2 + n) * 5;
                    qL[v] = s_gp[q0][tid];
                    qR[v] = s_gp[q0 + 1][tid];
                    g[0][v] = s_gp[q0 + 2][tid];
                    g[1][v] = s_gp[q0 + 3][tid];
                    g[2][v] = s_gp[q0 + 4][tid];
                }
                gp_flux_adj<NEED_F0>(qL, qR, g, a.fc, 0.25, b0, b1, qLb, qRb, gb);
                for (int v = 0; v < 4; ++v) {
                    const long long base = (long long)(((v * 2 + m) * 2 + n) * 5) * a.nface + fi;
                    a.gpbar[base] = qLb[v];
                    a.gpbar[base + a.nface] = qRb[v];
                    a.gpbar[base + 2 * a.nface] = gb[0][v];
                    a.gpbar[base + 3 * a.nface] = gb[1][v];
                    a.gpbar[base + 4 * a.nface] = gb[2][v];
                }
            }
        }
        ihc_lo = ihc_hi;
    }
}

// ------------------------------------------------------------------------------------------------
// passes B and C fused: the transpose of the t2 sweep produces one row (fixed t2 position) of t1 line
// adjoints at a time into LDS, and the transpose of the t1 sweep and of C = (q^L + q^R)/2 consumes it
// there, so the t1 line adjoints never reach HBM
// ------------------------------------------------------------------------------------------------
constexpr int BC_ROWS = 64;  // t2 rows (outputs kx) per workgroup

// Work split of the fused pass along t1 for n_t1 cells: outputs jx per segment, t1 positions per
// segment at most (the threads are two per position: Gauss lines m = 0, 1), segments per row.
struct BcSplit {
    int seg, npt, nseg;
};
inline BcSplit bc_split(int n_t1) {
    BcSplit b;
    // at most 128 positions (LDS of the exact mode: 33 KB)
    if (n_t1 <= 128) {  // one segment: all outputs -2 .. n_t1 + 1 from all positions 0 .. n_t1 - 1
        b.seg = n_t1 + 4;
        b.npt = (n_t1 + 31) / 32 * 32;
    } else {  // segments of 124 outputs read 128 positions
        b.seg = 124;
        b.npt = 128;
    }
    b.nseg = (n_t1 + 4 + b.seg - 1) / b.seg;
    return b;
}

template <bool EXACT>
__global__ void __launch_bounds__(256) adj_t21_kernel(const AdjFaceArgs a, int seg_len, int npt) {
    constexpr int NW = EXACT ? 5 : 2;
    // one workgroup per (row chunk of BC_ROWS t2 positions incl. halo, t1 segment, variable, face) of
    // 2 npt threads. Thread (jl, m), jl = tid % npt, m = tid / npt, runs the t2 transpose of t1 position
    // j = jlo + jl, Gauss line m: it walks the faces of the chunk in ascending t2 order, each face adding
    // its terms to the five rows kx = k-2 .. k+2 it reaches (a ring), the face's two t2 WENO
    // coefficients rebuilt from the t1 line values of its stencil (a second ring). When row kx = k-2 is
    // complete it goes to LDS, and the workgroup transposes the t1 sweep of that row: the coefficients
    // of every position's t1 WENO evaluations are rebuilt from the normal face values of its stencil,
    // and every output jx gathers its five positions (ascending t1, Gauss line m inner). Sums are in
    // the same fixed orders as the separate passes.
    extern __shared__ double lds[];
    double* const s_tb = lds;                        // [10][npt]: t1 line adjoints [m * 5 + q][position]
    double* const s_w = s_tb + 10 * npt;             // [4 NW][npt]: coefficients [(side * 2 + m) * NW + kk]
    double* const s_f = s_w + 4 * NW * npt;          // [2][npt + 4]: normal face values q^L, q^R
    double* const s_h1 = s_f + 2 * (npt + 4);        // [npt]: inverse t1 widths of the positions
    const int tid = threadIdx.x;
    const int nrc = (a.n_t2 + 4 + BC_ROWS - 1) / BC_ROWS;
    const int nseg = (a.n_t1 + 4 + seg_len - 1) / seg_len;
    long long r_ = blockIdx.x;
    const int rc = (int)(r_ % nrc);
    r_ /= nrc;
    const int seg = (int)(r_ % nseg);
    r_ /= nseg;
    const int v = (int)(r_ % 4);
    const int f = (int)(r_ / 4);
    const int kx_lo = -2 + rc * BC_ROWS, kx_hi = min(kx_lo + BC_ROWS, a.n_t2 + 2);
    const int seg0 = -2 + seg * seg_len, seg1 = min(seg0 + seg_len, a.n_t1 + 2);  // outputs jx
    const int jlo = max(0, seg0 - 2), jhi = min(a.n_t1, seg1 + 2);                 // positions j
    const int npos = jhi - jlo;
    const int jl = tid % npt, m = tid / npt;
    const bool tb = jl < npos;
    const int j = jlo + jl;
    const int vm = v * 2 + m;
    if (tid < npos) s_h1[tid] = a.ih1[jlo + tid];  // read after the first row's barrier
    auto t1val = [&](int side, int kx) -> double {
        return (tb && kx >= -2 && kx < a.n_t2 + 2) ? a.t1v[((v * 2 + side) * 2 + m) * a.nt1pos + t1_ix(a, f, j, kx)]
                                                   : 0.0;
    };
    // the adjoints of face k's Gauss-point inputs, [Gauss point n][quantity]
    auto gp_in = [&](int k, double g[2][5]) {
        const bool ok = tb && k >= 0 && k < a.n_t2;
        const long long fi = ok ? face_ix(a, f, j, k) : 0;
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int q = 0; q < 5; ++q) g[n][q] = ok ? a.gpbar[(long long)((vm * 2 + n) * 5 + q) * a.nface + fi] : 0.0;
    };
    // software pipelining: the next face's inputs and the t1 line value two positions ahead are loaded
    // one step before they are used
    double y[2][5], ynext[2], gnext[2][5];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        y[side][0] = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) y[side][r + 1] = t1val(side, kx_lo - 4 + r);
        ynext[side] = t1val(side, kx_lo);
    }
    gp_in(kx_lo - 2, gnext);
    // inverse t2 width of face k's cell, fetched one face ahead (clamped outside the cells, where unused)
    double ih2_nxt = a.ih2[min(max(kx_lo - 2, 0), a.n_t2 - 1)];
    double acc[5][5];
#pragma unroll
    for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[r][q] = 0.0;
    for (int k = kx_lo - 2; k < kx_hi + 2; ++k) {
        // ---- t2 transpose: face k of this thread's position
        double gcur[2][5];
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int q = 0; q < 5; ++q) gcur[n][q] = gnext[n][q];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
#pragma unroll
            for (int r = 0; r < 4; ++r) y[side][r] = y[side][r + 1];
            y[side][4] = ynext[side];
            ynext[side] = t1val(side, k + 3);
        }
        gp_in(k + 1, gnext);
        const double ih2 = ih2_nxt;
        ih2_nxt = a.ih2[min(max(k + 1, 0), a.n_t2 - 1)];
        if (tb && k >= 0 && k < a.n_t2) {
            double cw[2][2][NW];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                double gm, gp, wm[3], wp[3];
                weno_gauss_w<double>(y[side][0], y[side][1], y[side][2], y[side][3], y[side][4], a.eps, gm, gp, wm, wp);
                weno_coefs<EXACT>(2, y[side], a.eps, wm, gm, cw[side][0]);
                weno_coefs<EXACT>(3, y[side], a.eps, wp, gp, cw[side][1]);
            }
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                const int side = n == 0 ? 2 : 3;
                const int sg = n == 0 ? -1 : 1;
                const double* const gv = gcur[n];
#pragma unroll
                for (int r = 0; r < 5; ++r) {
                    const double cv = quartic_coef(0, sg, r), cd = quartic_coef(1, sg, r) * ih2;
                    acc[r][0] += wcoef<EXACT>(side, cw[0][n], r) * gv[0];
                    acc[r][1] += wcoef<EXACT>(side, cw[1][n], r) * gv[1];
                    acc[r][2] += cv * gv[2];
                    acc[r][3] += cv * gv[3];
                    acc[r][4] += cd * gv[4];
                }
            }
        }
        const int kx = k - 2;  // row kx has all its faces now
        if (kx >= kx_lo && kx < kx_hi) {
            // ---- t1 transpose of row kx
            if (tb)
#pragma unroll
                for (int q = 0; q < 5; ++q) s_tb[(m * 5 + q) * npt + jl] = acc[0][q];
            for (int l = tid; l < npos + 4; l += 2 * npt) {
                const int jx = jlo - 2 + l;
                const bool in = jx >= -2 && jx < a.n_t1 + 2;
                const long long p = in ? n_ix(a, f, jx, kx) : 0;
                s_f[l] = in ? a.fv[(v * 2 + 0) * a.nnpos + p] : 0.0;
                s_f[(npt + 4) + l] = in ? a.fv[(v * 2 + 1) * a.nnpos + p] : 0.0;
            }
            __syncthreads();
            {
                // coefficients of position jl (side = the thread's m slot): stencil at t1 cells j-2 .. j+2
                const int side = m;
                if (tb) {
                    double x[5];
#pragma unroll
                    for (int r = 0; r < 5; ++r) x[r] = s_f[side * (npt + 4) + jl + r];
                    double gm, gp, wm[3], wp[3], cm[NW], cp[NW];
                    weno_gauss_w<double>(x[0], x[1], x[2], x[3], x[4], a.eps, gm, gp, wm, wp);
                    weno_coefs<EXACT>(2, x, a.eps, wm, gm, cm);
                    weno_coefs<EXACT>(3, x, a.eps, wp, gp, cp);
#pragma unroll
                    for (int kk = 0; kk < NW; ++kk) {
                        s_w[((side * 2 + 0) * NW + kk) * npt + jl] = cm[kk];
                        s_w[((side * 2 + 1) * NW + kk) * npt + jl] = cp[kk];
                    }
                }
            }
            __syncthreads();
            for (int o = tid; o < seg1 - seg0; o += 2 * npt) {
                const int jx = seg0 + o;
                double bar[3] = {0.0, 0.0, 0.0}, Cb = 0.0;
                // positions jx - 2 .. jx + 2 in ascending order (stencil slot r = jx - jj + 2 descending)
#pragma unroll
                for (int r = 4; r >= 0; --r) {
                    const int jj = jx - r + 2;
                    if (jj < 0 || jj >= a.n_t1) continue;
                    const int l = jj - jlo;
#pragma unroll
                    for (int mm = 0; mm < 2; ++mm) {
                        const int side = mm == 0 ? 2 : 3;
                        const int sg = mm == 0 ? -1 : 1;
                        const double cv = quartic_coef(0, sg, r), cd = quartic_coef(1, sg, r) * s_h1[l];
                        double wL[NW], wR[NW];
#pragma unroll
                        for (int kk = 0; kk < NW; ++kk) {
                            wL[kk] = s_w[((0 * 2 + mm) * NW + kk) * npt + l];
                            wR[kk] = s_w[((1 * 2 + mm) * NW + kk) * npt + l];
                        }
                        bar[0] += wcoef<EXACT>(side, wL, r) * s_tb[(mm * 5 + 0) * npt + l];
                        bar[1] += wcoef<EXACT>(side, wR, r) * s_tb[(mm * 5 + 1) * npt + l];
                        bar[2] += cv * s_tb[(mm * 5 + 2) * npt + l];
                        Cb += cd * s_tb[(mm * 5 + 3) * npt + l];
                        Cb += cv * s_tb[(mm * 5 + 4) * npt + l];
                    }
                }
                const long long p = n_ix(a, f, jx, kx);
                a.fabar[(long long)(v * 3 + 0) * a.nnpos + p] = bar[0] + 0.5 * Cb;
                a.fabar[(long long)(v * 3 + 1) * a.nnpos + p] = bar[1] + 0.5 * Cb;
                a.fabar[(long long)(v * 3 + 2) * a.nnpos + p] = bar[2];
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int q = 0; q < 5; ++q) acc[r][q] = acc[r + 1][q];
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[4][q] = 0.0;
    }
}

// ------------------------------------------------------------------------------------------------
// pass D: transpose of the normal reconstruction -> padded cell adjoint (accumulated)
// ------------------------------------------------------------------------------------------------
constexpr int N_CHUNK = 32;  // consecutive cells along the normal per thread in pass D

template <bool EXACT>
__global__ void __launch_bounds__(256) adj_normal_kernel(const AdjFaceArgs a) {
    constexpr int NW = EXACT ? 5 : 2;
    // one thread per (tangential position incl. halo, variable, chunk of N_CHUNK cells along the
    // normal); the t1 position is the fastest index. The thread walks its cells in order with the six
    // faces f = i-2 .. i+3 that reach cell i in registers (slot s holds face i-2+s), loading each face
    // once, and sums per cell the q^L terms, then the q^R terms, then the D terms, each in ascending f.
    // The coefficients of the normal WENO evaluations are rebuilt from the field as the recompute's
    // column march formed them: the evaluation on cell c (stencil c-2 .. c+2) gives q^R of face c and
    // q^L of face c+1, so a five-cell window and the carried q^L coefficients suffice.
    const int ncell = a.n_n + 6;  // padded cells i = -3 .. n_n + 2
    const int nchunk = (ncell + N_CHUNK - 1) / N_CHUNK;
    const long long total = (long long)nchunk * 4 * (a.n_t2 + 4) * (a.n_t1 + 4);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int jx = (int)(t % (a.n_t1 + 4)) - 2;
    long long r_ = t / (a.n_t1 + 4);
    const int v = (int)(r_ % 4);
    r_ /= 4;
    const int kx = (int)(r_ % (a.n_t2 + 4)) - 2;
    const int c = (int)(r_ / (a.n_t2 + 4));
    const int i_lo = -3 + c * N_CHUNK, i_hi = min(i_lo + N_CHUNK, a.n_n + 3);
    const long long colq = a.pad0 + (long long)jx * a.st_t1 + (long long)kx * a.st_t2;
    auto cell = [&](int i) -> double { return (i >= -3 && i < a.n_n + 3) ? a.q[v][colq + (long long)i * a.st_n] : 0.0; };
    double wl[6][NW], wr[6][NW], fb[6][3];
    bool ok[6];
    // the next face to enter the window, the field cells fn-2 .. fn+2 and the q^L coefficients of face fn
    int fn = i_lo - 2;
    double win[5], carryL[NW];
    {
        double s5[5];
#pragma unroll
        for (int r = 0; r < 5; ++r) s5[r] = cell(fn - 3 + r);
        double right, left, w_r[3], w_l[3];
        weno_faces_w<double>(s5[0], s5[1], s5[2], s5[3], s5[4], a.eps, right, left, w_r, w_l);
        weno_coefs<EXACT>(0, s5, a.eps, w_r, right, carryL);
#pragma unroll
        for (int r = 0; r < 4; ++r) win[r] = s5[r + 1];
        win[4] = cell(fn + 2);
    }
    auto enter = [&](int s) {
        ok[s] = fn >= 0 && fn <= a.n_n;
        double right, left, w_r[3], w_l[3];
        weno_faces_w<double>(win[0], win[1], win[2], win[3], win[4], a.eps, right, left, w_r, w_l);
#pragma unroll
        for (int kk = 0; kk < NW; ++kk) wl[s][kk] = carryL[kk];
        weno_coefs<EXACT>(1, win, a.eps, w_l, left, wr[s]);
        weno_coefs<EXACT>(0, win, a.eps, w_r, right, carryL);
        const long long p = ok[s] ? n_ix(a, fn, jx, kx) : 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) fb[s][q] = ok[s] ? a.fabar[(long long)(v * 3 + q) * a.nnpos + p] : 0.0;
        fb[s][2] *= a.ihf[min(max(fn, 0), a.n_n)];  // D's 1/h at face fn
#pragma unroll
        for (int r = 0; r < 4; ++r) win[r] = win[r + 1];
        win[4] = cell(fn + 3);
        ++fn;
    };
#pragma unroll
    for (int s = 0; s < 6; ++s) enter(s);
    const double cD[4] = {1.0 / 12.0, -15.0 / 12.0, 15.0 / 12.0, -1.0 / 12.0};
    for (int i = i_lo; i < i_hi; ++i) {
        double bar = 0.0;
        // q^L(f) = sum_r W^L_f[r] Q(f-3+r): faces i-1 .. i+3 (slots 1..5), r = 5 - s
#pragma unroll
        for (int s = 1; s <= 5; ++s)
            if (ok[s]) bar += wcoef<EXACT>(0, wl[s], 5 - s) * fb[s][0];
        // q^R(f) = sum_r W^R_f[r] Q(f-2+r): faces i-2 .. i+2 (slots 0..4), r = 4 - s
#pragma unroll
        for (int s = 0; s <= 4; ++s)
            if (ok[s]) bar += wcoef<EXACT>(1, wr[s], 4 - s) * fb[s][1];
        // D(f) = (Q(f-2) - 15 Q(f-1) + 15 Q(f) - Q(f+1)) / (12 h_f): faces i-1 .. i+2 (slots 1..4), the
        // 1/h_f already in fb
#pragma unroll
        for (int s = 1; s <= 4; ++s)
            if (ok[s]) bar += cD[4 - s] * fb[s][2];
        const long long q = a.pad0 + (long long)i * a.st_n + (long long)jx * a.st_t1 + (long long)kx * a.st_t2;
        a.acc[v][q] += bar;
        // slide the window: face i + 4 enters
        if (i + 1 < i_hi) {
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                ok[s] = ok[s + 1];
#pragma unroll
                for (int kk = 0; kk < NW; ++kk) {
                    wl[s][kk] = wl[s + 1][kk];
                    wr[s][kk] = wr[s + 1][kk];
                }
#pragma unroll
                for (int qq = 0; qq < 3; ++qq) fb[s][qq] = fb[s + 1][qq];
            }
            enter(5);
        }
    }
}

template <bool EXACT>
hipError_t launch_adj_passes(const AdjFaceArgs& a, int stage, hipStream_t s) {
    const int nchunks = (a.n_n + a.chunk - 1) / a.chunk;
    const long long blocks = ((long long)a.tiles_t1 * a.tiles_t2 * nchunks + 7) / 8 * 8;
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 fgrid((unsigned)blocks), fblock(FaceTile<double>::THREADS);
    if (stage == 1) hipLaunchKernelGGL((adj_face_kernel<1>), fgrid, fblock, 0, s, a);
    else hipLaunchKernelGGL((adj_face_kernel<2>), fgrid, fblock, 0, s, a);
    const BcSplit bc = bc_split(a.n_t1);
    const long long nBC = (long long)(a.n_n + 1) * 4 * bc.nseg * ((a.n_t2 + 4 + BC_ROWS - 1) / BC_ROWS);
    const size_t lds = ((size_t)(11 + 4 * (EXACT ? 5 : 2)) * bc.npt + 2 * (size_t)(bc.npt + 4)) * sizeof(double);
    if (nBC > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((adj_t21_kernel<EXACT>), dim3((unsigned)nBC), dim3(2 * bc.npt), lds, s, a, bc.seg, bc.npt);
    const long long nD = (long long)((a.n_n + 6 + N_CHUNK - 1) / N_CHUNK) * 4 * (a.n_t1 + 4) * (a.n_t2 + 4);
    hipLaunchKernelGGL((adj_normal_kernel<EXACT>), dim3((unsigned)((nD + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_direction(const AdjFaceArgs& a, int stage, hipStream_t s) {
    return a.exact ? launch_adj_passes<true>(a, stage, s) : launch_adj_passes<false>(a, stage, s);
}

// ------------------------------------------------------------------------------------------------
// transpose of the ghost fill: axes in reverse order (z, y, x); each thread folds the six ghost cells
// of one line in a fixed order
// ------------------------------------------------------------------------------------------------
struct FoldArgs {
    int axis, n, np1, np2;
    long long st_a, st_1, st_2;
    int bc_lo, bc_hi;
    // inflow sides: the prescribed velocity, the sound speed, rho_ref and the padded field the ghost fill
    // was applied to (global variable order), at which the fill is linearised
    double u_in[3], c, rho_ref;
    Field4<const double> q;
};

__global__ void adj_fold_kernel(Field4<double> f, FoldArgs g) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)g.np1 * g.np2) return;
    const int p1 = (int)(t % g.np1), p2 = (int)(t / g.np1);
    const long long base = (long long)p1 * g.st_1 + (long long)p2 * g.st_2;
    for (int side = 0; side < 2; ++side) {
        const int kind = side == 0 ? g.bc_lo : g.bc_hi;
        for (int layer = 0; layer < 3; ++layer) {
            const int gi = side == 0 ? (2 - layer) : (g.n + 3 + layer);
            int src_i;
            if (kind == 0) src_i = side == 0 ? (g.n - 1 - layer) : layer;
            else if (kind == 1 || kind == 2) src_i = side == 0 ? layer : (g.n - 1 - layer);
            else src_i = side == 0 ? 0 : g.n - 1;
            const long long dst = base + (long long)gi * g.st_a;
            const long long src = base + (long long)(src_i + 3) * g.st_a;
            if (kind == 3) {  // inflow
                // ghost = (rho_g - rho_ref, rho_g u_in) with rho_g = rho_i e^x, x = s (u_in,n - m_n / rho_i) / C
                // (s = +1 on the low side, -1 on the high side): only rho' and m_n of the source enter,
                // d rho_g / d rho' = e^x (1 + s u_n / C), d rho_g / d m_n = -s e^x / C
                const double sgn = side == 0 ? 1.0 : -1.0;
                const double rho_i = g.rho_ref + g.q.v[0][src];
                const double un = g.q.v[1 + g.axis][src] / rho_i;
                const double ex = exp(sgn * (g.u_in[g.axis] - un) / g.c);
                const double br = f.v[0][dst] + g.u_in[0] * f.v[1][dst] + g.u_in[1] * f.v[2][dst] + g.u_in[2] * f.v[3][dst];
                f.v[0][src] += ex * (1.0 + sgn * un / g.c) * br;
                f.v[1 + g.axis][src] += -sgn * ex / g.c * br;
                for (int v = 0; v < 4; ++v) f.v[v][dst] = 0.0;
                continue;
            }
            for (int v = 0; v < 4; ++v) {
                double sg = 1.0;
                if (kind == 1 && v > 0) sg = -1.0;
                if (kind == 2 && v == 1 + g.axis) sg = -1.0;
                f.v[v][src] += sg * f.v[v][dst];
                f.v[v][dst] = 0.0;
            }
        }
    }
}

hipError_t launch_adj_fold(double* fp[4], const GridDesc& gd, const int bc[6], const double* const q[4],
                           const double u_in[3], double c, double rho_ref, hipStream_t s) {
    Field4<double> f;
    for (int v = 0; v < 4; ++v) f.v[v] = fp[v];
    for (int axis = 2; axis >= 0; --axis) {
        FoldArgs g;
        g.axis = axis;
        g.n = gd.n[axis];
        const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
        g.np1 = gd.n[a1] + 6;
        g.np2 = gd.n[a2] + 6;
        g.st_a = gd.st[axis];
        g.st_1 = gd.st[a1];
        g.st_2 = gd.st[a2];
        g.bc_lo = bc[2 * axis];
        g.bc_hi = bc[2 * axis + 1];
        for (int j = 0; j < 3; ++j) g.u_in[j] = u_in[j];
        g.c = c;
        g.rho_ref = rho_ref;
        for (int v = 0; v < 4; ++v) g.q.v[v] = q[v];
        const long long total = (long long)g.np1 * g.np2;
        hipLaunchKernelGGL(adj_fold_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, f, g);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// elementwise helpers
// ------------------------------------------------------------------------------------------------
__global__ void axpby_kernel(double* y, const double* x, double a, const double* z, double b, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = a * x[i] + (z ? b * z[i] : 0.0);
}

hipError_t launch_axpby(double* y, const double* x, double a, const double* z, double b, long long n, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, x, a, z, b, n);
    return hipGetLastError();
}

__global__ void pad_to_int_kernel(double* dst, const double* src, double a, const double* src2, double b, GridDesc g) {
    const long long n = (long long)g.n[0] * g.n[1] * g.n[2];
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int i = (int)(c % g.n[0]);
    const long long r = c / g.n[0];
    const int j = (int)(r % g.n[1]);
    const int k = (int)(r / g.n[1]);
    const long long p = g.pad0 + i * g.st[0] + j * g.st[1] + (long long)k * g.st[2];
    dst[c] = a * src[p] + (src2 ? b * src2[p] : 0.0);
}

hipError_t launch_pad_to_int(double* dst, const double* src, double a, const double* src2, double b,
                             const GridDesc& g, hipStream_t s) {
    const long long n = (long long)g.n[0] * g.n[1] * g.n[2];
    hipLaunchKernelGGL(pad_to_int_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, a, src2, b, g);
    return hipGetLastError();
}

__global__ void zero_kernel(double* y, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = 0.0;
}

hipError_t launch_zero(double* y, long long n, hipStream_t s) {
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// immersed-body adjoint (body at rest). Per forced cell the S direct-forcing iterations are affine in
// (rho, m): m^{s+1} = m^s + r (rho v-bar - m^s), r = V-bar / |Omega|, with V-bar and v-bar fixed by the
// body. Their transpose, taken through the iterations in reverse order, scales the momentum adjoint by
// (1 - r) per iteration and adds r v-bar . lambda_m to the density adjoint (the density is not forced).
// Every forced cell appears once in the body's cell list, so the cells are independent.
// ------------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) ibm_adj_kernel(Field4<double> lam, IbmArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncell) return;
    const long long q = a.g.pad0 + (long long)a.cell[3 * c] * a.g.st[0] + (long long)a.cell[3 * c + 1] * a.g.st[1] +
                        (long long)a.cell[3 * c + 2] * a.g.st[2];
    const double r = a.vbar[c] / (a.g.h[0] * a.g.h[1] * a.g.h[2]);
    const double vv[3] = {a.vbar_vel[3 * c], a.vbar_vel[3 * c + 1], a.vbar_vel[3 * c + 2]};
    double lm[3] = {lam.v[1][q], lam.v[2][q], lam.v[3][q]};
    double lr = lam.v[0][q];
    for (int s = 0; s < a.iters; ++s) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lr += r * vv[d] * lm[d];
            lm[d] *= 1.0 - r;
        }
    }
    lam.v[0][q] = lr;
#pragma unroll
    for (int d = 0; d < 3; ++d) lam.v[1 + d][q] = lm[d];
}

hipError_t launch_ibm_adjoint(double* lam[4], const IbmArgs& a, hipStream_t s) {
    if (a.moving || a.ncell_dev) return hipErrorInvalidValue;
    if (a.ncell <= 0 || a.iters <= 0) return hipSuccess;
    Field4<double> f;
    for (int v = 0; v < 4; ++v) f.v[v] = lam[v];
    hipLaunchKernelGGL(ibm_adj_kernel, dim3((unsigned)((a.ncell + 255) / 256)), dim3(256), 0, s, f, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// actuator-line adjoint
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ long long pidx_g(const GridDesc& g, int i, int j, int k) {
    return g.pad0 + (long long)i * g.st[0] + (long long)j * g.st[1] + (long long)k * g.st[2];
}

// per point: fvbar = dt sum_cells G(x - X_p) lambda_m(x) over the projection sphere; one workgroup per
// point, its threads striding over the cells of the sphere's bounding box, then a fixed-order tree sum
__global__ void __launch_bounds__(256) alm_adj_gather_kernel(AlmAdjArgs A) {
    const AlmArgs& a = A.fwd;
    const int p = blockIdx.x;  // uniform over the workgroup
    if (p >= a.n_act) return;
    const double X[3] = {a.X[3 * p], a.X[3 * p + 1], a.X[3 * p + 2]};
    const double cut = 9.0 * a.eps * a.eps, ie2 = 1.0 / (a.eps * a.eps);
    const double norm = 1.0 / (a.eps * a.eps * a.eps * M_PI * sqrt(M_PI));
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = (int)ceil((X[d] - 3.0 * a.eps - a.g.x0[d]) / a.g.h[d] - 0.5);
        hi[d] = (int)floor((X[d] + 3.0 * a.eps - a.g.x0[d]) / a.g.h[d] - 0.5);
        lo[d] = max(lo[d], a.box_lo[d]);
        hi[d] = min(hi[d], a.box_lo[d] + a.box_n[d] - 1);
    }
    const int nx = hi[0] - lo[0] + 1, ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
    const int ncell = (nx > 0 && ny > 0 && nz > 0) ? nx * ny * nz : 0;
    double acc[3] = {0, 0, 0};
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
        const int i = lo[0] + c % nx, r = c / nx;
        const int j = lo[1] + r % ny, k = lo[2] + r / ny;
        const double dx = a.g.x0[0] + (i + 0.5) * a.g.h[0] - X[0];
        const double dy = a.g.x0[1] + (j + 0.5) * a.g.h[1] - X[1];
        const double dz = a.g.x0[2] + (k + 0.5) * a.g.h[2] - X[2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 <= cut) {
            const double gw = norm * exp(-r2 * ie2);
            const long long q = pidx_g(a.g, i, j, k);
            for (int d = 0; d < 3; ++d) acc[d] += gw * A.lam_m[d][q];
        }
    }
    __shared__ double red[3][256];
    for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = acc[d];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double dt = a.st->dt;
        for (int d = 0; d < 3; ++d) A.pt[d * a.n_act + p] = dt * red[d][0];
    }
}

// per point: reverse of the blade-element forces; gradient in s and the adjoint of the sampled U
__global__ void alm_adj_points_kernel(AlmAdjArgs A) {
    const AlmArgs& a = A.fwd;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_act) return;
    const int bl = p / a.npb, ip = p % a.npb;
    const double t = a.st->t_next;
    const double th = a.theta0 + a.omega * t + 2.0 * M_PI * (double)bl / (double)a.nb;
    const double et1 = -sin(th), et2 = cos(th);
    const double rr = a.r[ip], chord = a.chord[ip], twist = a.twist[ip], width = a.width[ip];
    const double om = a.omega;
    const double U0 = a.out_u[3 * p], U1 = a.out_u[3 * p + 1], U2 = a.out_u[3 * p + 2];
    const double ux0 = U0, ut0 = U1 * et1 + U2 * et2;
    // forward recompute
    double ux = ux0, ut = ut0, fac = 1.0, g = 1.0, al0 = 0.0, U2_0 = 0.0;
    const double kc = chord / (4.0 * sqrt(M_PI) * a.eps);
    if (a.corr) {
        const double x0 = om * rr - ut0;
        U2_0 = ux0 * ux0 + x0 * x0;
        al0 = atan2(ux0, x0) - twist;
        const double cd0 = a.cd0 + a.cd2 * al0 * al0;
        g = 1.0 - cd0 * kc;
        fac = 1.0 / g;
        ux = ux0 * fac;
        ut = ut0 * fac;
    }
    const double xx = om * rr - ut;
    const double phi = atan2(ux, xx);
    const double alpha = phi - twist;
    const double wr = ut - om * rr;
    const double U2r = ux * ux + wr * wr;
    const bool inside = (alpha > -a.alpha_clip) && (alpha < a.alpha_clip);
    const double alc = fmin(fmax(alpha, -a.alpha_clip), a.alpha_clip);
    const double cl = a.cl_slope * alc, cd = a.cd0 + a.cd2 * alpha * alpha;
    const double q = 0.5 * a.rho_ref * chord * width * U2r;
    const double L = q * cl, D = q * cd;
    const double cph = cos(phi), sph = sin(phi);
    const double X0 = L * cph + D * sph, Y0 = L * sph - D * cph;
    double fa = 1.0, ftn = 1.0, dfa = 0.0, dft = 0.0;
    if (a.tip) {
        fa = tip_factor(a.g1_axi, a.nb, a.radius, rr, phi, &dfa);
        ftn = tip_factor(a.g1_tan, a.nb, a.radius, rr, phi, &dft);
    }
    const double fx0 = fa * X0, ft0 = ftn * Y0;
    const double sp = a.scale ? a.scale[p] : 1.0;
    // reverse
    const double fv0 = A.pt[p], fv1 = A.pt[a.n_act + p], fv2 = A.pt[2 * a.n_act + p];
    const double fxb = -fv0 + A.w1 * A.inv_n;
    const double ftb = -(fv1 * et1 + fv2 * et2) + A.w0 * A.inv_n * om * rr;
    A.grad_s[p] += fxb * fx0 + ftb * ft0;
    const double fx0b = sp * fxb, ft0b = sp * ftb;
    const double X0b = fx0b * fa, Y0b = ft0b * ftn;
    const double Lb = X0b * cph + Y0b * sph;
    const double Db = X0b * sph - Y0b * cph;
    double phib = -X0b * Y0 + Y0b * X0 + fx0b * X0 * dfa + ft0b * Y0 * dft;
    const double qb = Lb * cl + Db * cd;
    const double clb = Lb * q, cdb = Db * q;
    const double alb = clb * a.cl_slope * (inside ? 1.0 : 0.0) + cdb * 2.0 * a.cd2 * alpha;
    phib += alb;
    const double U2b = qb * 0.5 * a.rho_ref * chord * width;
    double uxb = U2b * 2.0 * ux + phib * xx / U2r;
    double utb = U2b * 2.0 * wr + phib * ux / U2r;
    if (a.corr) {
        const double facb = uxb * ux0 + utb * ut0;
        uxb *= fac;
        utb *= fac;
        const double gb = -facb / (g * g);
        const double cd0b = -gb * kc;
        const double al0b = cd0b * 2.0 * a.cd2 * al0;
        const double x0 = om * rr - ut0;
        uxb += al0b * x0 / U2_0;
        utb += al0b * ux0 / U2_0;
    }
    A.pt[3 * a.n_act + p] = uxb;
    A.pt[4 * a.n_act + p] = utb * et1;
    A.pt[5 * a.n_act + p] = utb * et2;
}

// adjoint of the velocity sampling (trilinear, or the mean of trilinear samples along the direction of
// motion) in gather form: one thread per cell of the sampling box adds, for the points in ascending
// order and their samples in ascending order, the terms of every sample whose eight trilinear cells
// hold it (the order of a serial sweep over points, samples and corners)
__global__ void __launch_bounds__(256) alm_adj_scatter_kernel(AlmAdjArgs A) {
    const AlmArgs& a = A.fwd;
    const long long ncell = (long long)a.samp_n[0] * a.samp_n[1] * a.samp_n[2];
    const long long tcell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tcell >= ncell) return;
    const int ci = a.samp_lo[0] + (int)(tcell % a.samp_n[0]);
    const int cj = a.samp_lo[1] + (int)((tcell / a.samp_n[0]) % a.samp_n[1]);
    const int ck = a.samp_lo[2] + (int)(tcell / ((long long)a.samp_n[0] * a.samp_n[1]));
    const long long q = pidx_g(a.g, ci, cj, ck);
    const double rho = a.rho_ref + A.qpre[0][q];
    const double Uc[3] = {A.qpre[1][q] / rho, A.qpre[2][q] / rho, A.qpre[3][q] / rho};
    double lam[4] = {A.lam_pre[0][q], A.lam_pre[1][q], A.lam_pre[2][q], A.lam_pre[3][q]};
    bool touched = false;
    const int ns = a.line_n > 1 ? a.line_n : 1;
    const double t = a.st->t_next;
    for (int p = 0; p < a.n_act; ++p) {
        double Ub[3] = {A.pt[3 * a.n_act + p], A.pt[4 * a.n_act + p], A.pt[5 * a.n_act + p]};
        if (ns > 1)
            for (int c = 0; c < 3; ++c) Ub[c] /= (double)ns;
        const int bl = p / a.npb;
        const double th = a.theta0 + a.omega * t + 2.0 * M_PI * (double)bl / (double)a.nb;
        const double et1 = -sin(th), et2 = cos(th);
        for (int k = 0; k < ns; ++k) {
            const double sk = ns > 1 ? line_offset(a, k) : 0.0;
            const double Xs[3] = {a.X[3 * p], a.X[3 * p + 1] + sk * et1, a.X[3 * p + 2] + sk * et2};
            int i0[3];
            double w1[3];
            for (int d = 0; d < 3; ++d) {
                const double fc = (Xs[d] - a.g.x0[d]) / a.g.h[d] - 0.5;
                const double fl = floor(fc);
                i0[d] = (int)fl;
                w1[d] = fc - fl;
            }
            const int dx = ci - i0[0], dy = cj - i0[1], dz = ck - i0[2];
            if (dx < 0 || dx > 1 || dy < 0 || dy > 1 || dz < 0 || dz > 1) continue;
            const double w = (dx ? w1[0] : 1.0 - w1[0]) * (dy ? w1[1] : 1.0 - w1[1]) * (dz ? w1[2] : 1.0 - w1[2]);
            double dot = 0.0;
            for (int c = 0; c < 3; ++c) {
                lam[1 + c] += w * Ub[c] / rho;
                dot += Ub[c] * Uc[c];
            }
            lam[0] += -w * dot / rho;
            touched = true;
        }
    }
    if (touched)
        for (int v = 0; v < 4; ++v) A.lam_pre[v][q] = lam[v];
}

hipError_t launch_alm_adjoint(const AlmAdjArgs& A, hipStream_t s) {
    const int n = A.fwd.n_act;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(alm_adj_gather_kernel, dim3(n), dim3(256), 0, s, A);
    hipLaunchKernelGGL(alm_adj_points_kernel, dim3((n + 63) / 64), dim3(64), 0, s, A);
    const long long ncell = (long long)A.fwd.samp_n[0] * A.fwd.samp_n[1] * A.fwd.samp_n[2];
    hipLaunchKernelGGL(alm_adj_scatter_kernel, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, A);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// workspace
// ------------------------------------------------------------------------------------------------
void adjoint_carve(char* base, int nx, int ny, int nz, int n_act, AdjBuffers* b, size_t* total) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~size_t(255);
        return p;
    };
    const size_t np = (size_t)(nx + 6) * (ny + 6) * (nz + 6);
    const size_t N = (size_t)nx * ny * nz;
    double** pads[6] = {b->lam, b->lam_pre, b->lam_star, b->acc, b->qwork, b->qpre};
    for (int a = 0; a < 6; ++a)
        for (int v = 0; v < 4; ++v) pads[a][v] = reinterpret_cast<double*>(take(np * 8));
    for (int v = 0; v < 4; ++v) b->mu0[v] = reinterpret_cast<double*>(take(N * 8));
    for (int v = 0; v < 4; ++v) b->mu1[v] = reinterpret_cast<double*>(take(N * 8));
    const int n[3] = {nx, ny, nz};
    const int ax[3][3] = {{0, 1, 2}, {1, 0, 2}, {2, 0, 1}};
    size_t nface = 0, nt1 = 0, nn = 0;
    for (int d = 0; d < 3; ++d) {
        const size_t a0 = n[ax[d][0]] + 1, a1 = n[ax[d][1]], a2 = n[ax[d][2]];
        nface = std::max(nface, a0 * a1 * a2);
        nt1 = std::max(nt1, a0 * a1 * (a2 + 4));
        nn = std::max(nn, a0 * (a1 + 4) * (a2 + 4));
    }
    b->gpbar = reinterpret_cast<double*>(take(80 * nface * 8));
    b->t1v = reinterpret_cast<double*>(take(16 * nt1 * 8));
    b->fv = reinterpret_cast<double*>(take(8 * nn * 8));
    b->fabar = reinterpret_cast<double*>(take(12 * nn * 8));
    b->pt = reinterpret_cast<double*>(take(16 * (size_t)std::max(n_act, 1) * 8));
    *total = off;
}

size_t adjoint_workspace_bytes(int nx, int ny, int nz, int n_act) {
    AdjBuffers b;
    size_t t = 0;
    adjoint_carve(nullptr, nx, ny, nz, n_act, &b, &t);
    return t;
}

}  // namespace gks
