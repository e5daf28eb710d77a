// gks_stage2.hip -- face pass of the second-order GKS variant (the comparison scheme of the paper's
// accuracy study, Section 4.3.3; its construction is defined by reference only): the gas-kinetic flux
// and the S2O4 stages of the high-order scheme, with van Leer-limited linear face states, central-
// difference gradients of the equilibrium state and one flux evaluation at the face centre.
//
// Layout of one workgroup (384 threads): a 16 x 16 tile of faces marching along the normal. Threads
// 0..323 own the 18 x 18 columns of the tile and its one-cell tangential halo: they keep the cells
// f-2 .. f+1 of their column in registers (next cell prefetched one step ahead) and publish the face
// states, the normal derivative and the face average C to LDS. Threads 0..255 own one face each: they
// read their column's states and the four neighbouring face averages, evaluate the flux and the
// divergence against the previous face of the column, and run the same epilogue roles as the
// high-order face pass (x: blocked residual, y: main residual, z: S2O4 stage update). Two LDS buffers of
// face states let the face phase of one face and the column phase of the next run between one pair of
// barriers (one barrier per face).
#include "gks_internal.h"

namespace gks {

namespace {

constexpr int T2O_THREADS = 384;
constexpr int T2O_EXT = TILE1 + 2;  // 18 columns per tangential direction

template <typename real>
__device__ __forceinline__ real van_leer(real dm, real dp) {
    const real prod = dm * dp;
    return prod > real(0) ? real(2) * prod / (dm + dp) : real(0);
}

template <int MODE>
struct LocalOrder2;
template <>
struct LocalOrder2<3> {
    static constexpr int v[4] = {0, 1, 2, 3};
};
template <>
struct LocalOrder2<0> {
    static constexpr int v[4] = {0, 2, 1, 3};
};
template <>
struct LocalOrder2<4> {
    static constexpr int v[4] = {0, 2, 3, 1};
};

template <typename real>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double4;
};

// the four variables of cell i in an array that holds them together
template <typename real>
__device__ __forceinline__ void ld4(const real* p, long long i, real out[4]) {
    const typename Vec4<real>::type v = *reinterpret_cast<const typename Vec4<real>::type*>(p + 4 * i);
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
}
template <typename real>
__device__ __forceinline__ void st4(real* p, long long i, const real in[4]) {
    typename Vec4<real>::type v;
    v.x = in[0];
    v.y = in[1];
    v.z = in[2];
    v.w = in[3];
    *reinterpret_cast<typename Vec4<real>::type*>(p + 4 * i) = v;
}

__device__ __forceinline__ void two_sum2(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

}  // namespace

template <typename real, int STAGE, int MODE, bool STR>
__global__ void __launch_bounds__(T2O_THREADS) face2_kernel(const FaceArgs<real> a) {
    static_assert(MODE == 0 || MODE == 3 || MODE == 4, "face pass mode");
    constexpr bool NEED_F0 = (STAGE == 1);
    constexpr bool COMP = sizeof(real) == 4;  // FP32: compensated state in the z-pass stage update
    constexpr int LOC[4] = {LocalOrder2<MODE>::v[0], LocalOrder2<MODE>::v[1], LocalOrder2<MODE>::v[2],
                            LocalOrder2<MODE>::v[3]};
    __shared__ real s_face[2][4][4][T2O_EXT][T2O_EXT];  // [buffer][variable][q^L, q^R, D, C][t2][t1]

    const int tid = threadIdx.x;
    // consecutive logical workgroups run on the same XCD (the hardware deals workgroups round-robin to
    // the 8 XCDs; the grid is padded to a multiple of 8), so neighbouring tiles share that XCD's L2 for
    // their halo columns
    int b = (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8);
    if (b >= a.tiles_t1 * a.tiles_t2 * ((a.n_n + a.chunk - 1) / a.chunk)) return;
    const int tile1 = b % a.tiles_t1;
    b /= a.tiles_t1;
    const int tile2 = b % a.tiles_t2;
    b /= a.tiles_t2;
    const int f0 = b * a.chunk;
    const int f1 = min(f0 + a.chunk, a.n_n);  // residuals of cells [f0, f1); faces f0..f1
    const int j0 = tile1 * TILE1, k0 = tile2 * TILE2;

    // column role: column (c1, c2) of the 18 x 18 grid, cells (j0 - 1 + c1, k0 - 1 + c2)
    const bool col = tid < T2O_EXT * T2O_EXT;
    const int c1 = tid % T2O_EXT, c2 = tid / T2O_EXT;
    const int jc = j0 - 1 + c1, kc = k0 - 1 + c2;
    const bool col_ld = col && (jc <= a.n_t1) && (kc <= a.n_t2);
    const long long cbase = a.pad0 + (long long)jc * a.st_t1 + (long long)kc * a.st_t2;
    // the in-loop column prefetch is done by every thread (threads without a column read a clamped one
    // whose values are not used): a load on every path keeps the compiler from waiting for it, and for
    // the step's stores, before the next step
    const long long cbase_ld = a.pad0 + (long long)min(jc, a.n_t1 + NG - 1) * a.st_t1 +
                               (long long)min(kc, a.n_t2 + NG - 1) * a.st_t2;
    // face role
    const bool face = tid < TILE1 * TILE2;
    const int fj = tid % TILE1, fk = tid / TILE1;
    const bool face_ok = face && (j0 + fj < a.n_t1) && (k0 + fk < a.n_t2);

    // FP32: the normal momentum is carried as its deviation from a workgroup constant (the midrange of
    // its values in the tile's first window) and the mass flux is formed in deviation form, as in the
    // high-order pass; the limiter and the differences commute with the shift
    constexpr bool SHIFT = sizeof(real) == 4;
    real cm = real(0);
    real ring[4][4];  // cells f-2, f-1, f, f+1
    real nxt[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        nxt[v] = real(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) ring[v][r] = real(0);
    }
    if (col_ld) {
#pragma unroll
        for (int r = 1; r < 4; ++r) {  // cells f0-2 .. f0; the step shifts in f0+1
            const long long idx = cbase + (long long)(f0 - 3 + r) * a.st_n;
#pragma unroll
            for (int v = 0; v < 4; ++v) ring[v][r] = a.q[v][idx];
        }
        const long long idx = cbase + (long long)(f0 + 1) * a.st_n;
#pragma unroll
        for (int v = 0; v < 4; ++v) nxt[v] = a.q[v][idx];
    }
    if constexpr (SHIFT) {
        __shared__ float s_range[2][T2O_THREADS / 64];
        float lo = col_ld ? float(ring[1][1]) : 3.0e38f, up = col_ld ? float(ring[1][1]) : -3.0e38f;
#pragma unroll
        for (int r = 2; r < 4; ++r) {
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
        for (int w = 1; w < T2O_THREADS / 64; ++w) {
            lo = fminf(lo, s_range[0][w]);
            up = fmaxf(up, s_range[1][w]);
        }
        cm = lo <= up ? real(0.5f * (lo + up)) : real(0);
#pragma unroll
        for (int r = 1; r < 4; ++r) ring[1][r] -= cm;
    }
    const real dt = real(*a.dt_ptr);
    real fprev0[4] = {0, 0, 0, 0}, fprev1[4] = {0, 0, 0, 0};
    // tangential inverse widths of this thread's face line
    const real ih1 = STR ? a.ih1[min(j0 + fj, a.n_t1 - 1)] : a.inv_h1;
    const real ih2 = STR ? a.ih2[min(k0 + fk, a.n_t2 - 1)] : a.inv_h2;

    // column phase of face f into LDS buffer buf
    auto column_step = [&](int f, int buf) {
        const real ihf_f = STR ? a.ihf[f] : a.inv_hn;  // inverse spacing at face f (normal derivative)
        // ---- column phase: window cells f-2 .. f+1 (prefetch f+2)
        if (col) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
#pragma unroll
                for (int r = 0; r < 3; ++r) ring[v][r] = ring[v][r + 1];
                // the shift is applied here, a step after the load, so that the prefetch stays in flight
                ring[v][3] = (SHIFT && v == 1) ? nxt[v] - cm : nxt[v];
            }
        }
        {
            const long long idx = cbase_ld + (long long)min(f + 2, a.n_n + 2) * a.st_n;
#pragma unroll
            for (int v = 0; v < 4; ++v) nxt[v] = a.q[v][idx];
        }
        if (col) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const real qm2 = ring[v][0], qm1 = ring[v][1], q0 = ring[v][2], qp1 = ring[v][3];
                s_face[buf][v][0][c2][c1] = qm1 + real(0.5) * van_leer(qm1 - qm2, q0 - qm1);
                s_face[buf][v][1][c2][c1] = q0 - real(0.5) * van_leer(q0 - qm1, qp1 - q0);
                s_face[buf][v][2][c2][c1] = (q0 - qm1) * ihf_f;
                s_face[buf][v][3][c2][c1] = real(0.5) * (qm1 + q0);
            }
        }
    };
    // two LDS buffers, one barrier per face: the face phase of f reads buffer f mod 2 while the column
    // phase of f + 1 fills the other
    column_step(f0, 0);
    __syncthreads();
    for (int f = f0; f <= f1; ++f) {
        const int buf = (f - f0) & 1;
        // ---- face phase: flux at the face centre (weight 1)
        real fa0[4] = {0, 0, 0, 0}, fa1[4] = {0, 0, 0, 0};
        if (face) {
            const int cj = fj + 1, ck = fk + 1;
            real qL[4], qR[4], g[3][4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                qL[v] = s_face[buf][v][0][ck][cj];
                qR[v] = s_face[buf][v][1][ck][cj];
                g[0][v] = s_face[buf][v][2][ck][cj];
                g[1][v] = (s_face[buf][v][3][ck][cj + 1] - s_face[buf][v][3][ck][cj - 1]) * (real(0.5) * ih1);
                g[2][v] = (s_face[buf][v][3][ck + 1][cj] - s_face[buf][v][3][ck - 1][cj]) * (real(0.5) * ih2);
            }
            gp_flux<real, NEED_F0, SHIFT>(qL, qR, g, a.fc, real(1), fa0, fa1, cm);
        }
        if (f + 1 <= f1) column_step(f + 1, buf ^ 1);
        if (f > f0 && face_ok) {
            const int cell = f - 1;
            const long long ridx = (long long)cell * a.ist_n + (long long)(j0 + fj) * a.ist_t1 +
                                   (long long)(k0 + fk) * a.ist_t2;
            const long long pidx = a.pad0 + (long long)cell * a.st_n + (long long)(j0 + fj) * a.st_t1 +
                                   (long long)(k0 + fk) * a.st_t2;
            real d1[4], d0[4];  // global variable order
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const real ihc = STR ? a.ihc[cell] : a.inv_hn;
                d1[g] = -(fa1[LOC[g]] - fprev1[LOC[g]]) * ihc;
                d0[g] = NEED_F0 ? -(fa0[LOC[g]] - fprev0[LOC[g]]) * ihc : real(0);
            }
            if constexpr (MODE == 3) {
                const long long xidx = rx_block_index(cell, j0 + fj, k0 + fk, a.rx_nx, a.rx_nyb);
                st4(a.rx1, xidx, d1);
                if (NEED_F0) st4(a.rx0, xidx, d0);
            } else if constexpr (MODE == 0) {
                st4(a.r1, ridx, d1);
                if (NEED_F0) st4(a.r0, ridx, d0);
            } else {
                const long long xidx = rx_block_index(j0 + fj, k0 + fk, cell, a.rx_nx, a.rx_nyb);
                real r1v[4], x1v[4], r0v[4] = {0, 0, 0, 0}, x0v[4] = {0, 0, 0, 0}, lov[4] = {0, 0, 0, 0};
                real loa[4], lob[4];
                ld4(a.r1, ridx, r1v);
                ld4(a.rx1, xidx, x1v);
                if (NEED_F0) {
                    ld4(a.r0, ridx, r0v);
                    ld4(a.rx0, xidx, x0v);
                }
                if (COMP) ld4(a.lo_in, ridx, lov);
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int lv = LOC[g];
                    const real L1 = r1v[g] + (d1[g] + x1v[g]);
                    const real L0 = NEED_F0 ? r0v[g] + (d0[g] + x0v[g]) : real(0);
                    if constexpr (COMP) {
                        const real lo = lov[g];
                        float sh, sl;
                        if (NEED_F0) {
                            const real Q = a.q_c[lv][pidx];
                            two_sum2(Q, lo + (real(0.5) * dt * L0 + real(0.125) * dt * dt * L1), sh, sl);
                            a.out_a[lv][pidx] = sh;
                            loa[g] = sl;
                            two_sum2(Q, lo + (dt * L0 + (dt * dt * real(1.0 / 6.0)) * L1), sh, sl);
                            a.out_b[lv][pidx] = sh;
                            lob[g] = sl;
                        } else {
                            const real add = (dt * dt * real(1.0 / 3.0)) * L1 + (g > 0 ? dt * a.g_global[g - 1] : real(0));
                            two_sum2(a.s_in[lv][pidx], lo + add, sh, sl);
                            a.out_a[lv][pidx] = sh;
                            loa[g] = sl;
                        }
                    } else {
                        if (NEED_F0) {
                            const real Q = a.q_c[lv][pidx];
                            a.out_a[lv][pidx] = Q + real(0.5) * dt * L0 + real(0.125) * dt * dt * L1;
                            a.out_b[lv][pidx] = Q + dt * L0 + (dt * dt * real(1.0 / 6.0)) * L1;
                        } else {
                            const real add = (dt * dt * real(1.0 / 3.0)) * L1 + (g > 0 ? dt * a.g_global[g - 1] : real(0));
                            a.out_a[lv][pidx] = a.s_in[lv][pidx] + add;
                        }
                    }
                }
                if constexpr (COMP) {
                    st4(a.lo_a, ridx, loa);
                    if (NEED_F0) st4(a.lo_b, ridx, lob);
                }
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            fprev1[v] = fa1[v];
            if (NEED_F0) fprev0[v] = fa0[v];
        }
        __syncthreads();
    }
}

template <typename real>
int face2_slots() {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, face2_kernel<real, 1, 4, false>, T2O_THREADS, 0) !=
        hipSuccess)
        return 0;
    return cus * per_cu;
}

template <typename real>
hipError_t launch_face2(const FaceArgs<real>& a, int stage, hipStream_t s) {
    const int nchunks = (a.n_n + a.chunk - 1) / a.chunk;
    const long long blocks = ((long long)a.tiles_t1 * a.tiles_t2 * nchunks + 7) / 8 * 8;
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(T2O_THREADS);
#define GKS_FACE2_LAUNCH(ST, MD)                                                                     \
    do {                                                                                             \
        if (a.stretched) hipLaunchKernelGGL((face2_kernel<real, ST, MD, true>), grid, block, 0, s, a);  \
        else hipLaunchKernelGGL((face2_kernel<real, ST, MD, false>), grid, block, 0, s, a);             \
    } while (0)
    if (stage == 1) {
        if (a.mode == 0) GKS_FACE2_LAUNCH(1, 0);
        else if (a.mode == 3) GKS_FACE2_LAUNCH(1, 3);
        else if (a.mode == 4) GKS_FACE2_LAUNCH(1, 4);
        else return hipErrorInvalidValue;
    } else {
        if (a.mode == 0) GKS_FACE2_LAUNCH(2, 0);
        else if (a.mode == 3) GKS_FACE2_LAUNCH(2, 3);
        else if (a.mode == 4) GKS_FACE2_LAUNCH(2, 4);
        else return hipErrorInvalidValue;
    }
#undef GKS_FACE2_LAUNCH
    return hipGetLastError();
}

template hipError_t launch_face2<float>(const FaceArgs<float>&, int, hipStream_t);
template hipError_t launch_face2<double>(const FaceArgs<double>&, int, hipStream_t);
template int face2_slots<float>();
template int face2_slots<double>();

}  // namespace gks
