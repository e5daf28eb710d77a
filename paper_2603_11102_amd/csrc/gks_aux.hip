// gks_aux.hip -- ghost cells, CFL time step, step bookkeeping and FP64 diagnostics.
//
// Boundary ghost cells (three layers) follow the boundary conditions named in Section 4:
// periodic; no-slip isothermal wall (mirror, rho even, all momenta odd); slip / symmetry wall
// (mirror, normal momentum odd); inflow with prescribed velocity and the density from the outgoing
// isothermal Riemann invariant U -+ C ln rho; zero-gradient outflow. Axes are filled x, then y, then z
// over the full padded extent of the other axes, so edges and corners are consistent.
// Time step: dt = CFL min(dx, dy, dz) / (|U|_max + C), C = sqrt(1/(2 lambda)) (Section 2).
#include "gks.h"
#include "gks_internal.h"

namespace gks {

struct GhostArgs {
    int axis, n, np1, np2;
    long long st_a, st_1, st_2;
    int bc_lo, bc_hi;
    double u_in[3];
    double c, rho_ref;
};

template <typename real>
__global__ void ghost_kernel(Field4<real> f, GhostArgs g) {
    const long long per_side = 3LL * g.np1 * g.np2;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * per_side) return;
    const int side = (int)(t / per_side);
    long long r = t % per_side;
    const int layer = (int)(r / ((long long)g.np1 * g.np2));
    r %= (long long)g.np1 * g.np2;
    const int p1 = (int)(r % g.np1), p2 = (int)(r / g.np1);
    const long long base = (long long)p1 * g.st_1 + (long long)p2 * g.st_2;
    // padded index along the axis: interior cell i sits at i + 3
    const int gi = side == 0 ? (2 - layer) : (g.n + 3 + layer);
    const int kind = side == 0 ? g.bc_lo : g.bc_hi;
    const long long dst = base + (long long)gi * g.st_a;
    int src_i;
    if (kind == 0) src_i = side == 0 ? (g.n - 1 - layer) : layer;                      // periodic
    else if (kind == 1 || kind == 2) src_i = side == 0 ? layer : (g.n - 1 - layer);    // mirror
    else src_i = side == 0 ? 0 : g.n - 1;                                              // adjacent cell
    const long long src = base + (long long)(src_i + 3) * g.st_a;
    if (kind == 0 || kind == 4) {
#pragma unroll
        for (int v = 0; v < 4; ++v) f.v[v][dst] = f.v[v][src];
    } else if (kind == 1) {
        f.v[0][dst] = f.v[0][src];
#pragma unroll
        for (int v = 1; v < 4; ++v) f.v[v][dst] = -f.v[v][src];
    } else if (kind == 2) {
#pragma unroll
        for (int v = 0; v < 4; ++v) f.v[v][dst] = (v == 1 + g.axis) ? -f.v[v][src] : f.v[v][src];
    } else {  // inflow
        const double rp = (double)f.v[0][src];
        const double rho_i = g.rho_ref + rp;
        const double un = (double)f.v[1 + g.axis][src] / rho_i;
        const double x = side == 0 ? (g.u_in[g.axis] - un) / g.c : (un - g.u_in[g.axis]) / g.c;
        const double rho_g = rho_i * exp(x);
        f.v[0][dst] = (real)(rp * exp(x) + g.rho_ref * expm1(x));
#pragma unroll
        for (int j = 0; j < 3; ++j) f.v[1 + j][dst] = (real)(rho_g * g.u_in[j]);
    }
}

template <typename real>
hipError_t launch_ghost(Field4<real> f, const GridDesc& gd, int axis, int bc_lo, int bc_hi, const double u_in[3],
                        double c, double rho_ref, hipStream_t s) {
    GhostArgs g;
    g.axis = axis;
    g.n = gd.n[axis];
    const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
    g.np1 = gd.n[a1] + 6;
    g.np2 = gd.n[a2] + 6;
    g.st_a = gd.st[axis];
    g.st_1 = gd.st[a1];
    g.st_2 = gd.st[a2];
    g.bc_lo = bc_lo;
    g.bc_hi = bc_hi;
    for (int j = 0; j < 3; ++j) g.u_in[j] = u_in[j];
    g.c = c;
    g.rho_ref = rho_ref;
    const long long total = 2LL * 3 * g.np1 * g.np2;
    const int bs = 256;
    hipLaunchKernelGGL((ghost_kernel<real>), dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, s, f, g);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// max |U|^2 over the interior cells (as a double; max is order independent, so the result is
// deterministic)
// ------------------------------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(256) umax_kernel(Field4<real> f, GridDesc g, double rho_ref, double* part) {
    // per-workgroup maximum of |U|^2 over the interior cells; dt_kernel reduces the partial maxima
    __shared__ double red[256];
    const unsigned n = (unsigned)g.n[0] * (unsigned)g.n[1] * (unsigned)g.n[2];
    const unsigned nx = (unsigned)g.n[0], ny = (unsigned)g.n[1];
    double mx = 0.0;
    for (unsigned c = blockIdx.x * 256u + threadIdx.x; c < n; c += gridDim.x * 256u) {
        const unsigned i = c % nx, r = c / nx;
        const unsigned j = r % ny, k = r / ny;
        const long long p = g.pad0 + i + (long long)j * g.st[1] + (long long)k * g.st[2];
        const double rho = rho_ref + (double)f.v[0][p];
        const double u = (double)f.v[1][p] / rho, v = (double)f.v[2][p] / rho, w = (double)f.v[3][p] / rho;
        const double s2 = u * u + v * v + w * w;
        mx = s2 > mx ? s2 : mx;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// One launch for the ghost cells of all three axes and the [x][z][y] copy of the padded field.
// A ghost cell takes the value the axis-by-axis fill (x, then y, then z, over the full padded extent
// of the other axes) leaves there: the interior source cell is found per axis, then the boundary
// transforms of the ghost axes are applied in the order x, y, z, with the same arithmetic and the same
// rounding to the field's precision after each transform.
struct GhostAll {
    int n[3];
    int bc_lo[3], bc_hi[3];
    double u_in[3];
    double c, rho_ref;
};

// interior source index along one axis and the transform to apply (-1: none, else side 0 / 1)
__device__ __forceinline__ int ghost_source(int i, int n, int lo, int hi, int& side) {
    if (i >= 0 && i < n) {
        side = -1;
        return i;
    }
    side = i < 0 ? 0 : 1;
    const int kind = side == 0 ? lo : hi;
    if (kind == GKS_BC_PERIODIC) return side == 0 ? n + i : i - n;
    if (kind == GKS_BC_NOSLIP_WALL || kind == GKS_BC_SLIP_WALL) return side == 0 ? -1 - i : 2 * n - 1 - i;
    return side == 0 ? 0 : n - 1;  // inflow, outflow: the adjacent interior cell
}

template <typename real>
__device__ __forceinline__ void ghost_transform(real v[4], int axis, int side, int kind, const GhostAll& G) {
    if (kind == GKS_BC_NOSLIP_WALL) {
        for (int j = 1; j < 4; ++j) v[j] = -v[j];
    } else if (kind == GKS_BC_SLIP_WALL) {
        v[1 + axis] = -v[1 + axis];
    } else if (kind == GKS_BC_INFLOW) {
        const double rp = (double)v[0];
        const double rho_i = G.rho_ref + rp;
        const double un = (double)v[1 + axis] / rho_i;
        const double x = side == 0 ? (G.u_in[axis] - un) / G.c : (un - G.u_in[axis]) / G.c;
        const double rho_g = rho_i * exp(x);
        v[0] = (real)(rp * exp(x) + G.rho_ref * expm1(x));
        for (int j = 0; j < 3; ++j) v[1 + j] = (real)(rho_g * G.u_in[j]);
    }
}

template <typename real>
__global__ void __launch_bounds__(256) ghost_transpose_kernel(Field4<real> q, Field4<real> qt, GhostAll G) {
    __shared__ real t[4][32][33];
    const int X = G.n[0] + 6, Y = G.n[1] + 6, Z = G.n[2] + 6;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // z is the fastest grid index: consecutive workgroups write neighbouring z rows of the [x][z][y]
    // copy (10 % faster than x-fastest tiles on the 192 x 96 x 96 channel)
    const int x0 = blockIdx.y * 32, y0 = blockIdx.z * 32, z = blockIdx.x;
    // every lane finds the cell its value comes from (itself inside the domain, the interior source of
    // a ghost cell) and all 16 loads are issued before any is used; cells outside the padded block read
    // cell 0 and are not used
    int sd[4][3];
    long long src[4], dst[4];
    bool in[4], gh[4];
    const int sk = ghost_source(z - 3, G.n[2], G.bc_lo[2], G.bc_hi[2], sd[0][2]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int x = x0 + tx, y = y0 + ty + 8 * i;
        in[i] = x < X && y < Y;
        sd[i][2] = sd[0][2];
        const int si = ghost_source(x - 3, G.n[0], G.bc_lo[0], G.bc_hi[0], sd[i][0]);
        const int sj = ghost_source(y - 3, G.n[1], G.bc_lo[1], G.bc_hi[1], sd[i][1]);
        gh[i] = in[i] && (sd[i][0] >= 0 || sd[i][1] >= 0 || sd[i][2] >= 0);
        dst[i] = ((long long)z * Y + y) * X + x;
        src[i] = in[i] ? ((long long)(sk + 3) * Y + (sj + 3)) * X + (si + 3) : 0;
    }
    real v[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int w = 0; w < 4; ++w) v[i][w] = q.v[w][src[i]];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (gh[i]) {
            for (int a = 0; a < 3; ++a)
                if (sd[i][a] >= 0) ghost_transform(v[i], a, sd[i][a], sd[i][a] == 0 ? G.bc_lo[a] : G.bc_hi[a], G);
#pragma unroll
            for (int w = 0; w < 4; ++w) q.v[w][dst[i]] = v[i][w];
        }
#pragma unroll
        for (int w = 0; w < 4; ++w) t[w][ty + 8 * i][tx] = v[i][w];
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int r = ty; r < 32; r += 8) {
            const int y = y0 + tx, x = x0 + r;
            if (x < X && y < Y) qt.v[w][((long long)x * Z + z) * Y + y] = t[w][tx][r];
        }
}

template <typename real>
hipError_t launch_ghost_transpose(Field4<real> q, Field4<real> qt, const GridDesc& gd, const int bc[6],
                                  const double u_in[3], double c, double rho_ref, hipStream_t s) {
    GhostAll G;
    for (int a = 0; a < 3; ++a) {
        G.n[a] = gd.n[a];
        G.bc_lo[a] = bc[2 * a];
        G.bc_hi[a] = bc[2 * a + 1];
        G.u_in[a] = u_in[a];
    }
    G.c = c;
    G.rho_ref = rho_ref;
    const int X = gd.n[0] + 6, Y = gd.n[1] + 6, Z = gd.n[2] + 6;
    hipLaunchKernelGGL((ghost_transpose_kernel<real>), dim3(Z, (X + 31) / 32, (Y + 31) / 32), dim3(256), 0, s, q,
                       qt, G);
    return hipGetLastError();
}

// Copy of a padded field in the layout [x][z][y] (y fastest), read by the x-direction face pass so that
// its column loads are contiguous along y. One 32 x 32 (x, y) tile of one z-plane per workgroup.
template <typename real>
__global__ void __launch_bounds__(256) transpose_xy_kernel(Field4<real> in, Field4<real> out, int X, int Y, int Z) {
    __shared__ real t[4][32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
    // all 16 loads of a thread are issued before the single barrier
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int r = ty; r < 32; r += 8) {
            const int x = x0 + tx, y = y0 + r;
            if (x < X && y < Y) t[v][r][tx] = in.v[v][((long long)z * Y + y) * X + x];
        }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int r = ty; r < 32; r += 8) {
            const int y = y0 + tx, x = x0 + r;
            if (x < X && y < Y) out.v[v][((long long)x * Z + z) * Y + y] = t[v][tx][r];
        }
}

template <typename real>
hipError_t launch_transpose_xy(Field4<real> in, Field4<real> out, const GridDesc& g, hipStream_t s) {
    const int X = g.n[0] + 6, Y = g.n[1] + 6, Z = g.n[2] + 6;
    hipLaunchKernelGGL((transpose_xy_kernel<real>), dim3((X + 31) / 32, (Y + 31) / 32, Z), dim3(256), 0, s, in, out,
                       X, Y, Z);
    return hipGetLastError();
}

int umax_blocks(const GridDesc& g) {
    const long long n = (long long)g.n[0] * g.n[1] * g.n[2];
    long long blocks = (n + 255) / 256;
    return (int)(blocks > UMAX_BLOCKS ? UMAX_BLOCKS : blocks);
}

template <typename real>
hipError_t launch_umax(Field4<real> f, const GridDesc& g, double rho_ref, double* part, hipStream_t s) {
    hipLaunchKernelGGL((umax_kernel<real>), dim3((unsigned)umax_blocks(g)), dim3(256), 0, s, f, g, rho_ref, part);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) dt_kernel(DevState* st, const double* part, int nparts, double cfl,
                                                 double hmin, double c, double dt_fixed) {
    __shared__ double red[256];
    double mx = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) mx = fmax(mx, part[i]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s2]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double dt;
    if (cfl > 0.0) {
        const double u = sqrt(red[0]);
        dt = cfl * hmin / (u + c);
    } else {
        dt = dt_fixed;
    }
    st->dt = dt;
    st->t_next = st->t + dt;
    st->ibm_res_bits = 0ULL;
}

hipError_t launch_dt(DevState* st, const double* part, int nparts, double cfl, double hmin, double c,
                     double dt_fixed, hipStream_t s) {
    hipLaunchKernelGGL(dt_kernel, dim3(1), dim3(256), 0, s, st, part, cfl > 0.0 ? nparts : 0, cfl, hmin, c,
                       dt_fixed);
    return hipGetLastError();
}

__global__ void finish_kernel(DevState* st, int has_rotor, double* hist) {
    if (threadIdx.x != 0) return;
    st->t = st->t_next;
    st->step += 1;
    if (has_rotor) {
        st->win_p += st->power;
        st->win_t += st->thrust;
    }
    st->win_n += 1;
    if (hist) {
        double h[10];
        h[0] = st->t;
        h[1] = st->dt;
        h[2] = st->thrust;
        h[3] = st->torque;
        h[4] = st->power;
        h[5] = st->cp;
        h[6] = st->ct;
        h[7] = st->ibm_force[0];
        h[8] = st->ibm_force[1];
        h[9] = st->ibm_force[2];
        for (int i = 0; i < 10; ++i) hist[i] = h[i];
    }
}

hipError_t launch_finish(DevState* st, int has_rotor, double* hist, hipStream_t s) {
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, st, has_rotor, hist);
    return hipGetLastError();
}

__global__ void window_reset_kernel(DevState* st) {
    if (threadIdx.x != 0) return;
    st->win_p = 0.0;
    st->win_t = 0.0;
    st->win_n = 0;
}

hipError_t launch_window_reset(DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(window_reset_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// FP64 conservation sums, max |U| and a non-finite flag; fixed-order block partials then one block
// ------------------------------------------------------------------------------------------------
int diag_blocks(const GridDesc& g) {
    const long long n = (long long)g.n[0] * g.n[1] * g.n[2];
    long long b = (n + 255) / 256;
    if (b > 1024) b = 1024;
    return (int)b;
}

template <typename real>
__global__ void __launch_bounds__(256) diag_kernel(Field4<real> f, const real* lo, GridDesc g, double rho_ref,
                                                   double* partials, DevState* st) {
    __shared__ double red[4][256];
    __shared__ double mxs[256];
    const long long n = (long long)g.n[0] * g.n[1] * g.n[2];
    double s[4] = {0, 0, 0, 0};
    double mx = 0.0;
    int bad = 0;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(c % g.n[0]);
        const long long r = c / g.n[0];
        const int j = (int)(r % g.n[1]);
        const int k = (int)(r / g.n[1]);
        const long long p = g.pad0 + i * g.st[0] + j * g.st[1] + (long long)k * g.st[2];
        double q[4];
        // stretched axes: each cell weighs its volume over the mean cell volume (exactly 1 when uniform)
        const double wgt = (g.wrel[0] ? g.wrel[0][i] : 1.0) * (g.wrel[1] ? g.wrel[1][j] : 1.0) *
                           (g.wrel[2] ? g.wrel[2][k] : 1.0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            // FP32: the state is the field plus its low-order part ([cell][4], interior cells)
            q[v] = lo ? (double)f.v[v][p] + (double)lo[4 * c + v] : (double)f.v[v][p];
            s[v] += q[v] * wgt;
            if (!isfinite(q[v])) bad = 1;
        }
        const double rho = rho_ref + q[0];
        const double s2 = (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / (rho * rho);
        mx = s2 > mx ? s2 : mx;
    }
    for (int v = 0; v < 4; ++v) red[v][threadIdx.x] = s[v];
    mxs[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            for (int v = 0; v < 4; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + w];
            mxs[threadIdx.x] = fmax(mxs[threadIdx.x], mxs[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int v = 0; v < 4; ++v) partials[4 * blockIdx.x + v] = red[v][0];
        atomicMax(&st->umax_diag_bits, (unsigned long long)__double_as_longlong(mxs[0]));
    }
    if (bad) atomicOr(&st->nonfinite, 1);
}

__global__ void __launch_bounds__(256) diag_final_kernel(const double* partials, int nblk, DevState* st, double vol) {
    __shared__ double red[4][256];
    double s[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int v = 0; v < 4; ++v) s[v] += partials[4 * b + v];
    for (int v = 0; v < 4; ++v) red[v][threadIdx.x] = s[v];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int v = 0; v < 4; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->mass = red[0][0] * vol;
        for (int v = 0; v < 3; ++v) st->mom[v] = red[1 + v][0] * vol;
    }
}

__global__ void diag_reset_kernel(DevState* st) {
    if (threadIdx.x == 0) {
        st->umax_diag_bits = 0ULL;
        st->nonfinite = 0;
    }
}

template <typename real>
hipError_t launch_diag(Field4<real> f, const real* lo, const GridDesc& g, double rho_ref, double* partials, int nblk,
                       DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(diag_reset_kernel, dim3(1), dim3(64), 0, s, st);
    hipLaunchKernelGGL((diag_kernel<real>), dim3(nblk), dim3(256), 0, s, f, lo, g, rho_ref, partials, st);
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, (const double*)partials, nblk, st,
                       g.h[0] * g.h[1] * g.h[2]);
    return hipGetLastError();
}

// zero-fill of device memory by a kernel (usable inside a captured graph, unlike a memset node)
__global__ void __launch_bounds__(256) zero_words_kernel(unsigned* p, long long n) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) p[i] = 0u;
}

hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t s) {
    const long long n = (long long)(bytes / 4);
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<unsigned*>(p), n);
    return hipGetLastError();
}

hipError_t launch_copy_field(const void* src, void* dst, size_t bytes, hipStream_t s) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

template hipError_t launch_ghost<float>(Field4<float>, const GridDesc&, int, int, int, const double*, double, double, hipStream_t);
template hipError_t launch_ghost<double>(Field4<double>, const GridDesc&, int, int, int, const double*, double, double, hipStream_t);
template hipError_t launch_ghost_transpose<float>(Field4<float>, Field4<float>, const GridDesc&, const int[6], const double[3], double, double, hipStream_t);
template hipError_t launch_ghost_transpose<double>(Field4<double>, Field4<double>, const GridDesc&, const int[6], const double[3], double, double, hipStream_t);
template hipError_t launch_transpose_xy<float>(Field4<float>, Field4<float>, const GridDesc&, hipStream_t);
template hipError_t launch_transpose_xy<double>(Field4<double>, Field4<double>, const GridDesc&, hipStream_t);
template hipError_t launch_umax<float>(Field4<float>, const GridDesc&, double, double*, hipStream_t);
template hipError_t launch_umax<double>(Field4<double>, const GridDesc&, double, double*, hipStream_t);
template hipError_t launch_diag<float>(Field4<float>, const float*, const GridDesc&, double, double*, int, DevState*,
                                      hipStream_t);
template hipError_t launch_diag<double>(Field4<double>, const double*, const GridDesc&, double, double*, int,
                                       DevState*, hipStream_t);

}  // namespace gks
