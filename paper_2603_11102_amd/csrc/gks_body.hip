// gks_body.hip -- external body forces applied after the S2O4 step (Section 3.3):
//   * actuator line model (Section 3.1): trilinear sampling of U at each actuator point, blade-element
//     forces (Eq. (axial-tangential)) with the optional free-stream correction, Gaussian projection
//     (Eq. (Gaussian)) truncated at 3 eps; rotor thrust / torque / power / C_P / C_T reduced in FP64
//     (Section 4.4.1);
//   * direct-forcing immersed boundary (Section 3.2): Peskin 4-point delta weights, static volumes
//     V-bar = sum_p W V_p with V_p = dx dS_p, per-cell forcing iterations (Eq. (ibm-1)), total force
//     (Eq. (force-ibm)) reduced in FP64, interpolation residual at the points.
// Every sum runs in a fixed order (one thread per output, gather form, tree reductions): results are
// bitwise reproducible and no floating-point atomics are used.
#include "gks_body.h"

namespace gks {

__device__ __forceinline__ double phi4d(double r) {
    r = fabs(r);
    if (r <= 1.0) return (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r)) * 0.125;
    if (r < 2.0) return (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) * 0.125;
    return 0.0;
}

__device__ __forceinline__ long long pidx(const GridDesc& g, int i, int j, int k) {
    return g.pad0 + (long long)i * g.st[0] + (long long)j * g.st[1] + (long long)k * g.st[2];
}

// ------------------------------------------------------------------------------------------------
// ALM: one workgroup, one thread per actuator point
// ------------------------------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(1024) alm_points_kernel(Field4<real> f, AlmArgs a) {
    __shared__ double red_t[1024];
    __shared__ double red_q[1024];
    const int p = threadIdx.x;
    double fx = 0.0, ft = 0.0, rr = 0.0;
    const double t = a.st->t_next;
    if (p < a.n_act) {
        const int bl = p / a.npb, ip = p % a.npb;
        const double th = a.theta0 + a.omega * t + 2.0 * M_PI * (double)bl / (double)a.nb;
        const double cth = cos(th), sth = sin(th);
        rr = a.r[ip];
        const double X[3] = {a.hub[0], a.hub[1] + rr * cth, a.hub[2] + rr * sth};
        const double et[3] = {0.0, -sth, cth};
        // velocity U = (rho U)/rho at the point: trilinear interpolation of the cell-centre values
        // (point sampling, Section 3.1), or the mean of such samples along the direction of motion
        // (line sampling of the NTNU rotor, Section 4.4)
        double U[3] = {0.0, 0.0, 0.0};
        const int ns = a.line_n > 1 ? a.line_n : 1;
        for (int k = 0; k < ns; ++k) {
            const double sk = ns > 1 ? line_offset(a, k) : 0.0;
            const double Xs[3] = {X[0], X[1] + sk * et[1], X[2] + sk * et[2]};
            int i0[3];
            double w1[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double fc = (Xs[d] - a.g.x0[d]) / a.g.h[d] - 0.5;
                const double fl = floor(fc);
                i0[d] = (int)fl;
                w1[d] = fc - fl;
            }
            double Us[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx) {
                        const double w = (dx ? w1[0] : 1.0 - w1[0]) * (dy ? w1[1] : 1.0 - w1[1]) *
                                         (dz ? w1[2] : 1.0 - w1[2]);
                        const long long q = pidx(a.g, i0[0] + dx, i0[1] + dy, i0[2] + dz);
                        const double rho = a.rho_ref + (double)f.v[0][q];
#pragma unroll
                        for (int c = 0; c < 3; ++c) Us[c] += w * ((double)f.v[1 + c][q] / rho);
                    }
#pragma unroll
            for (int c = 0; c < 3; ++c) U[c] += Us[c];
        }
        if (ns > 1)
#pragma unroll
            for (int c = 0; c < 3; ++c) U[c] /= (double)ns;
        double ux = U[0];
        double ut = U[1] * et[1] + U[2] * et[2];
        const double om = a.omega;
        const double chord = a.chord[ip], twist = a.twist[ip], width = a.width[ip];
        if (a.corr) {
            const double phi0 = atan2(ux, om * rr - ut);
            const double al0 = phi0 - twist;
            const double cd0 = a.cd0 + a.cd2 * al0 * al0;
            const double fac = 1.0 / (1.0 - cd0 * chord / (4.0 * sqrt(M_PI) * a.eps));
            ux *= fac;
            ut *= fac;
        }
        const double phi = atan2(ux, om * rr - ut);
        const double alpha = phi - twist;
        const double wr = ut - om * rr;
        const double urel2 = ux * ux + wr * wr;
        const double alc = fmin(fmax(alpha, -a.alpha_clip), a.alpha_clip);
        const double cl = a.cl_slope * alc;
        const double cd = a.cd0 + a.cd2 * alpha * alpha;
        const double q = 0.5 * a.rho_ref * chord * width * urel2;
        const double lift = q * cl, drag = q * cd;
        const double s = a.scale ? a.scale[p] : 1.0;
        const double cph = cos(phi), sph = sin(phi);
        fx = s * (lift * cph + drag * sph);
        ft = s * (lift * sph - drag * cph);
        if (a.tip) {
            fx *= tip_factor(a.g1_axi, a.nb, a.radius, rr, phi, nullptr);
            ft *= tip_factor(a.g1_tan, a.nb, a.radius, rr, phi, nullptr);
        }
        // force on the fluid: minus the blade force
        a.X[3 * p + 0] = X[0];
        a.X[3 * p + 1] = X[1];
        a.X[3 * p + 2] = X[2];
        a.fv[3 * p + 0] = -fx;
        a.fv[3 * p + 1] = -ft * et[1];
        a.fv[3 * p + 2] = -ft * et[2];
        a.out_alpha[p] = alpha;
        a.out_fx[p] = fx;
        a.out_ft[p] = ft;
        a.out_urel[p] = sqrt(urel2);
        a.out_phi[p] = phi;
        a.out_u[3 * p + 0] = U[0];
        a.out_u[3 * p + 1] = U[1];
        a.out_u[3 * p + 2] = U[2];
    }
    red_t[p] = fx;
    red_q[p] = rr * ft;
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if (p < w) {
            red_t[p] += red_t[p + w];
            red_q[p] += red_q[p + w];
        }
        __syncthreads();
    }
    if (p == 0) {
        const double T = red_t[0], Q = red_q[0];
        a.st->thrust = T;
        a.st->torque = Q;
        a.st->power = a.omega * Q;
        a.st->cp = a.omega * Q / (0.5 * a.rho_ref * a.area * a.u_inf * a.u_inf * a.u_inf);
        a.st->ct = T / (0.5 * a.rho_ref * a.area * a.u_inf * a.u_inf);
    }
}

// Gaussian projection of the point forces onto the cells of the rotor box; m += dt f (gather form)
template <typename real>
__global__ void __launch_bounds__(256) alm_spread_kernel(Field4<real> f, AlmArgs a) {
    extern __shared__ double sh[];
    double* sx = sh;                 // 3 n
    double* sf = sh + 3 * a.n_act;   // 3 n
    for (int i = threadIdx.x; i < 3 * a.n_act; i += blockDim.x) {
        sx[i] = a.X[i];
        sf[i] = a.fv[i];
    }
    __syncthreads();
    const long long nb = (long long)a.box_n[0] * a.box_n[1] * a.box_n[2];
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nb) return;
    const int i = a.box_lo[0] + (int)(c % a.box_n[0]);
    const long long r = c / a.box_n[0];
    const int j = a.box_lo[1] + (int)(r % a.box_n[1]);
    const int k = a.box_lo[2] + (int)(r / a.box_n[1]);
    const double xc = a.g.x0[0] + (i + 0.5) * a.g.h[0];
    const double yc = a.g.x0[1] + (j + 0.5) * a.g.h[1];
    const double zc = a.g.x0[2] + (k + 0.5) * a.g.h[2];
    const double ie2 = 1.0 / (a.eps * a.eps);
    const double cut = 9.0 * a.eps * a.eps;
    const double norm = 1.0 / (a.eps * a.eps * a.eps * M_PI * sqrt(M_PI));
    double acc[3] = {0.0, 0.0, 0.0};
    bool any = false;
    for (int p = 0; p < a.n_act; ++p) {
        const double dx = xc - sx[3 * p], dy = yc - sx[3 * p + 1], dz = zc - sx[3 * p + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 <= cut) {
            const double gw = norm * exp(-r2 * ie2);
            acc[0] += sf[3 * p] * gw;
            acc[1] += sf[3 * p + 1] * gw;
            acc[2] += sf[3 * p + 2] * gw;
            any = true;
        }
    }
    if (!any) return;
    const double dt = a.st->dt;
    const long long q = pidx(a.g, i, j, k);
#pragma unroll
    for (int d = 0; d < 3; ++d) f.v[1 + d][q] = (real)((double)f.v[1 + d][q] + dt * acc[d]);
}

template <typename real>
hipError_t launch_alm(Field4<real> f, const AlmArgs& a, hipStream_t s) {
    int bs = 64;
    while (bs < a.n_act) bs <<= 1;
    hipLaunchKernelGGL((alm_points_kernel<real>), dim3(1), dim3(bs), 0, s, f, a);
    const long long nb = (long long)a.box_n[0] * a.box_n[1] * a.box_n[2];
    const size_t shm = sizeof(double) * 6 * (size_t)a.n_act;
    hipLaunchKernelGGL((alm_spread_kernel<real>), dim3((unsigned)((nb + 255) / 256)), dim3(256), shm, s, f, a);
    return hipGetLastError();
}

hipError_t launch_alm_points_only(Field4<double> f, const AlmArgs& a, hipStream_t s) {
    int bs = 64;
    while (bs < a.n_act) bs <<= 1;
    hipLaunchKernelGGL((alm_points_kernel<double>), dim3(1), dim3(bs), 0, s, f, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// IBM
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ double ibm_weight(const GridDesc& g, const double* X, int i, int j, int k) {
    const double rx = (g.x0[0] + (i + 0.5) * g.h[0] - X[0]) / g.h[0];
    const double ry = (g.x0[1] + (j + 0.5) * g.h[1] - X[1]) / g.h[1];
    const double rz = (g.x0[2] + (k + 0.5) * g.h[2] - X[2]) / g.h[2];
    return phi4d(rx) * phi4d(ry) * phi4d(rz);
}

// V-bar_c = sum over the points whose support holds c of W V_p and the cell velocity
// v-bar_c = sum W V_p v_p / V-bar_c; one wavefront per cell: the lanes take the cell's points in
// strides of 64, then a butterfly sum (a fixed order, the same for every call)
__device__ __forceinline__ void vbar_cell(const IbmArgs& a, int c, int lane) {
    const int i = a.cell[3 * c], j = a.cell[3 * c + 1], k = a.cell[3 * c + 2];
    double v = 0.0, mv[3] = {0.0, 0.0, 0.0};
    for (int e = a.csr[c] + lane; e < a.csr[c + 1]; e += 64) {
        const int p = a.ent[e];
        const double wv = ibm_weight(a.g, a.xyz + 3 * p, i, j, k) * (a.g.h[0] * a.dS[p]);
        v += wv;
        if (a.vel)
            for (int d = 0; d < 3; ++d) mv[d] += wv * a.vel[3 * p + d];
    }
    for (int o = 32; o > 0; o >>= 1) {
        v += __shfl_xor(v, o, 64);
        for (int d = 0; d < 3; ++d) mv[d] += __shfl_xor(mv[d], o, 64);
    }
    if (lane == 0) {
        a.vbar[c] = v;
        for (int d = 0; d < 3; ++d) a.vbar_vel[3 * c + d] = (a.vel && v > 0.0) ? mv[d] / v : 0.0;
    }
}

__global__ void __launch_bounds__(256) ibm_vbar_kernel(IbmArgs a) {
    const int lane = threadIdx.x & 63;
    const int nc = a.ncell_dev ? *a.ncell_dev : a.ncell;
    for (int c = blockIdx.x * 4 + (threadIdx.x >> 6); c < nc; c += gridDim.x * 4)  // uniform over the wavefront
        vbar_cell(a, c, lane);
}

// per cell: S direct-forcing iterations towards v-bar; FP64 block partials of sum F
template <typename real>
__global__ void __launch_bounds__(256) ibm_cells_kernel(Field4<real> f, IbmArgs a) {
    __shared__ double red[3][256];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    double F[3] = {0.0, 0.0, 0.0};
    const bool stopped = a.moving && a.st->ibm_outside;  // a moving body left the interior: no forcing
    if (c < (a.ncell_dev ? *a.ncell_dev : a.ncell) && !stopped) {
        const int i = a.cell[3 * c], j = a.cell[3 * c + 1], k = a.cell[3 * c + 2];
        const long long q = pidx(a.g, i, j, k);
        const double dt = a.st->dt;
        const double rho = a.rho_ref + (double)f.v[0][q];
        const double vb = a.vbar[c];
        const double vv[3] = {a.vbar_vel[3 * c], a.vbar_vel[3 * c + 1], a.vbar_vel[3 * c + 2]};
        const double vol = a.g.h[0] * a.g.h[1] * a.g.h[2];
        double m[3] = {(double)f.v[1][q], (double)f.v[2][q], (double)f.v[3][q]};
        for (int s = 0; s < a.iters; ++s) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double U = m[d] / rho;
                const double Fs = rho * vb * (vv[d] - U) / dt;
                m[d] = m[d] + dt * Fs / vol;
                F[d] += Fs;
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) f.v[1 + d][q] = (real)m[d];
    }
    for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = F[d];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) a.partials[3 * blockIdx.x + d] = red[d][0];
}

__global__ void __launch_bounds__(256) ibm_final_kernel(IbmArgs a, int nblk) {
    __shared__ double red[3][256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int d = 0; d < 3; ++d) s[d] += a.partials[3 * b + d];
    for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = s[d];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int d = 0; d < 3; ++d) a.st->ibm_force[d] = -red[d][0];  // load on the body
        a.st->ibm_iters_used = a.iters;
    }
}

// residual: max_p |v_p - sum_c W_{c->p} U_c| after the last iteration (max: order independent)
template <typename real>
__global__ void __launch_bounds__(256) ibm_resid_kernel(Field4<real> f, IbmArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npts || (a.moving && a.st->ibm_outside)) return;
    const double* X = a.xyz + 3 * p;
    int i0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) i0[d] = (int)floor((X[d] - a.g.x0[d]) / a.g.h[d] - 0.5);
    double U[3] = {0.0, 0.0, 0.0};
    for (int dk = -1; dk <= 2; ++dk)
        for (int dj = -1; dj <= 2; ++dj)
            for (int di = -1; di <= 2; ++di) {
                const int i = i0[0] + di, j = i0[1] + dj, k = i0[2] + dk;
                const double w = ibm_weight(a.g, X, i, j, k);
                const long long q = pidx(a.g, i, j, k);
                const double rho = a.rho_ref + (double)f.v[0][q];
#pragma unroll
                for (int d = 0; d < 3; ++d) U[d] += w * ((double)f.v[1 + d][q] / rho);
            }
    if (a.vel)
        for (int d = 0; d < 3; ++d) U[d] -= a.vel[3 * p + d];
    const double r = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
    atomicMax(&a.st->ibm_res_bits, (unsigned long long)__double_as_longlong(r));
}

// ------------------------------------------------------------------------------------------------
// moving body: the positions of the step and its supports rebuilt on the device, in the order of
// the host binning (cells ascending, x fastest; points ascending within a cell): the (cell, point)
// pairs are sorted by cell with a stable radix sort, then the first pair of every cell is compacted
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ long long flat_cell(const GridDesc& g, int i, int j, int k) {
    return ((long long)k * g.n[1] + j) * g.n[0] + i;
}

// Rigid motion to t^{n+1}: X_p = X_p(t0) + V tau + (R - I) r with r = X_p(t0) - c0 and
// (R - I) r = sin(theta) k x r + (1 - cos theta) k x (k x r) (Rodrigues), v_p = V + omega x R r.
// Lowest support cell per axis, clamped into the body's run of cells when the support leaves it
// (then the flag stops the forcing; the clamp keeps every later index valid: the points were accepted
// by gks_set_ibm_points, so every run holds at least 4 cells).
__global__ void __launch_bounds__(256) ibm_move_kernel(IbmArgs a, IbmMoveArgs m) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npts) return;
    const double tau = a.st->t_next - m.t0;
    double r[3], d[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int x = 0; x < 3; ++x) r[x] = m.xyz0[3 * p + x] - m.c0[x];
    const double wn = sqrt(m.omega[0] * m.omega[0] + m.omega[1] * m.omega[1] + m.omega[2] * m.omega[2]);
    if (wn > 0.0) {
        const double k[3] = {m.omega[0] / wn, m.omega[1] / wn, m.omega[2] / wn};
        const double th = wn * tau;
        const double sn = sin(th), hs = sin(0.5 * th), vc = 2.0 * hs * hs;
        const double kr[3] = {k[1] * r[2] - k[2] * r[1], k[2] * r[0] - k[0] * r[2], k[0] * r[1] - k[1] * r[0]};
        const double kkr[3] = {k[1] * kr[2] - k[2] * kr[1], k[2] * kr[0] - k[0] * kr[2], k[0] * kr[1] - k[1] * kr[0]};
#pragma unroll
        for (int x = 0; x < 3; ++x) d[x] = sn * kr[x] + vc * kkr[x];
    }
    double X[3], rr[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        X[x] = m.xyz0[3 * p + x] + m.vel[x] * tau + d[x];
        rr[x] = r[x] + d[x];
    }
    const double v[3] = {m.vel[0] + m.omega[1] * rr[2] - m.omega[2] * rr[1],
                         m.vel[1] + m.omega[2] * rr[0] - m.omega[0] * rr[2],
                         m.vel[2] + m.omega[0] * rr[1] - m.omega[1] * rr[0]};
    bool out = false;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        // support cells b - 1 .. b + 2 inside the run [run_lo, run_hi] (within the interior)
        const double f = (X[x] - a.g.x0[x]) / a.g.h[x] - 0.5;
        const int lo = m.run_lo[x] + 1, hi = m.run_hi[x] - 2;
        int b;
        if (f >= (double)lo && f < (double)(hi + 1)) {
            b = (int)floor(f);
        } else {  // also NaN
            out = true;
            b = f >= (double)lo ? hi : lo;
        }
        m.xyz[3 * p + x] = X[x];
        m.pvel[3 * p + x] = v[x];
        m.base[3 * p + x] = b;
    }
    if (out) atomicOr(&a.st->ibm_outside, 1);
}

unsigned vbar_blocks(int ncell) { return (unsigned)std::min(4096, (ncell + 3) / 4); }

// (cell, point) pairs in point-major order: item e = 64 p + q is the q-th support cell of point p
__global__ void __launch_bounds__(256) ibm_pairs_kernel(IbmArgs a, IbmMoveArgs m) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 64LL * a.npts) return;
    const int p = (int)(e >> 6), q = (int)(e & 63);
    const int i = m.base[3 * p] + (q & 3) - 1, j = m.base[3 * p + 1] + ((q >> 2) & 3) - 1,
              k = m.base[3 * p + 2] + (q >> 4) - 1;
    m.key[0][e] = (unsigned)flat_cell(a.g, i, j, k);
    m.val[0][e] = p;
}

// exclusive scan of 256 values held one per thread (Hillis-Steele in LDS); returns the total
__device__ __forceinline__ int block_exclusive_scan_256(int v, int* sh, int* excl) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {
        const int u = threadIdx.x >= w ? sh[threadIdx.x - w] : 0;
        __syncthreads();
        sh[threadIdx.x] += u;
        __syncthreads();
    }
    *excl = sh[threadIdx.x] - v;
    const int total = sh[255];
    __syncthreads();
    return total;
}

// Stable least-significant-digit radix sort of the pairs by cell, 8 bits per pass; stability keeps
// the points of a cell in ascending order. A tile is RADIX_TILE consecutive items, 256 per round.
__global__ void __launch_bounds__(256) radix_hist_kernel(const unsigned* key, int n, int shift, int* hist, int ntiles) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const long long t0 = (long long)blockIdx.x * RADIX_TILE;
    for (int r = 0; r < RADIX_TILE / 256; ++r) {
        const long long e = t0 + r * 256 + threadIdx.x;
        if (e < n) atomicAdd(&h[(key[e] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];  // digit-major
}

// one workgroup per digit: exclusive scan in place of the digit's tile counts, digit total to dtot
__global__ void __launch_bounds__(256) radix_digit_scan_kernel(int* hist, int ntiles, int* dtot) {
    __shared__ int sh[256];
    int* h = hist + (long long)blockIdx.x * ntiles;
    const int per = (ntiles + 255) / 256;
    const int lo = threadIdx.x * per, hi = min(ntiles, lo + per);
    int t = 0;
    for (int x = lo; x < hi; ++x) t += h[x];
    int run;
    const int total = block_exclusive_scan_256(t, sh, &run);
    for (int x = lo; x < hi; ++x) {
        const int v = h[x];
        h[x] = run;
        run += v;
    }
    if (threadIdx.x == 0) dtot[blockIdx.x] = total;
}

// scatter with stable ranks: within a round a lane's rank among the earlier lanes of its wavefront
// with the same digit (ballot match), plus the counts of the earlier wavefronts, plus the running
// count of the tile's earlier rounds, plus the tile's offset within its digit and the digit's base
__global__ void __launch_bounds__(256) radix_scatter_kernel(const unsigned* key, const int* val, unsigned* key_out,
                                                            int* val_out, int n, int shift, const int* hist,
                                                            const int* dtot, int ntiles) {
    __shared__ int sh[256];
    __shared__ int run[256];
    __shared__ int wc[4][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int base;
    block_exclusive_scan_256(dtot[threadIdx.x], sh, &base);
    run[threadIdx.x] = base + hist[threadIdx.x * ntiles + blockIdx.x];
    const long long t0 = (long long)blockIdx.x * RADIX_TILE;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    for (int r = 0; r < RADIX_TILE / 256; ++r) {
        for (int x = 0; x < 4; ++x) wc[x][threadIdx.x] = 0;
        __syncthreads();
        const long long e = t0 + r * 256 + threadIdx.x;
        const bool ok = e < n;
        const unsigned kk = ok ? key[e] : 0u;
        const int d = (int)((kk >> shift) & 255);
        unsigned long long mask = __ballot(ok);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const unsigned long long bb = __ballot(bit);
            mask &= bit ? bb : ~bb;
        }
        const int rank = __popcll(mask & below);
        if (ok && rank == 0) wc[w][d] = __popcll(mask);
        __syncthreads();
        if (ok) {
            int off = run[d] + rank;
            for (int x = 0; x < w; ++x) off += wc[x][d];
            key_out[off] = kk;
            val_out[off] = val[e];
        }
        __syncthreads();
        run[threadIdx.x] += wc[0][threadIdx.x] + wc[1][threadIdx.x] + wc[2][threadIdx.x] + wc[3][threadIdx.x];
    }
}

__device__ __forceinline__ bool run_head(const unsigned* key, long long e, int n) {
    return e < n && (e == 0 || key[e] != key[e - 1]);
}

// first pairs of cells (run heads of the sorted keys) per tile
__global__ void __launch_bounds__(256) ibm_head_count_kernel(const unsigned* key, int n, int* tcnt) {
    __shared__ int sh[256];
    const long long t0 = (long long)blockIdx.x * RADIX_TILE;
    int c = 0;
    for (int r = 0; r < RADIX_TILE / 256; ++r) c += run_head(key, t0 + r * 256 + threadIdx.x, n);
    int excl;
    const int total = block_exclusive_scan_256(c, sh, &excl);
    if (threadIdx.x == 0) tcnt[blockIdx.x] = total;
}

// exclusive scan in place of the per-tile head counts (one workgroup, a contiguous run per thread);
// the number of cells to counts[0] and csr[cells] = n
__global__ void __launch_bounds__(256) ibm_head_scan_kernel(int* tcnt, int ntiles, int n, int* counts, int* csr) {
    __shared__ int sh[256];
    const int per = (ntiles + 255) / 256;
    const int lo = threadIdx.x * per, hi = min(ntiles, lo + per);
    int t = 0;
    for (int x = lo; x < hi; ++x) t += tcnt[x];
    int run;
    const int total = block_exclusive_scan_256(t, sh, &run);
    for (int x = lo; x < hi; ++x) {
        const int v = tcnt[x];
        tcnt[x] = run;
        run += v;
    }
    if (threadIdx.x == 0) {
        counts[0] = total;
        counts[1] = n;
        csr[total] = n;
    }
}

// cells in ascending order: (i, j, k) and the index of their first pair (csr)
__global__ void __launch_bounds__(256) ibm_head_compact_kernel(const unsigned* key, int n, const int* tcnt, GridDesc g,
                                                               int* cell, int* csr) {
    __shared__ int wc[4];
    __shared__ int run;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) run = tcnt[blockIdx.x];
    const long long t0 = (long long)blockIdx.x * RADIX_TILE;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    for (int r = 0; r < RADIX_TILE / 256; ++r) {
        const long long e = t0 + r * 256 + threadIdx.x;
        const bool hd = run_head(key, e, n);
        const unsigned long long b = __ballot(hd);
        if (lane == 0) wc[w] = __popcll(b);
        __syncthreads();
        if (hd) {
            int c = run + __popcll(b & below);
            for (int x = 0; x < w; ++x) c += wc[x];
            const long long x = key[e];
            cell[3 * c] = (int)(x % g.n[0]);
            cell[3 * c + 1] = (int)((x / g.n[0]) % g.n[1]);
            cell[3 * c + 2] = (int)(x / ((long long)g.n[0] * g.n[1]));
            csr[c] = (int)e;
        }
        __syncthreads();
        if (threadIdx.x == 0) run += wc[0] + wc[1] + wc[2] + wc[3];
    }
}

hipError_t launch_ibm_move(const IbmArgs& a, const IbmMoveArgs& m, hipStream_t s) {
    if (a.npts <= 0) return hipSuccess;
    const long long ncells = (long long)a.g.n[0] * a.g.n[1] * a.g.n[2];
    const int n = 64 * a.npts;
    const int ntiles = (n + RADIX_TILE - 1) / RADIX_TILE;
    hipLaunchKernelGGL(ibm_move_kernel, dim3((a.npts + 255) / 256), dim3(256), 0, s, a, m);
    hipLaunchKernelGGL(ibm_pairs_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, m);
    int bits = 1;
    while (bits < 32 && (1LL << bits) < ncells) ++bits;
    const int passes = (bits + 7) / 8;
    int src = 0;
    for (int ps = 0; ps < passes; ++ps, src ^= 1) {
        const bool last = ps == passes - 1;
        hipLaunchKernelGGL(radix_hist_kernel, dim3(ntiles), dim3(256), 0, s, m.key[src], n, 8 * ps, m.hist, ntiles);
        hipLaunchKernelGGL(radix_digit_scan_kernel, dim3(256), dim3(256), 0, s, m.hist, ntiles, m.dtot);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(ntiles), dim3(256), 0, s, m.key[src], m.val[src], m.key[src ^ 1],
                           last ? m.ent : m.val[src ^ 1], n, 8 * ps, m.hist, m.dtot, ntiles);
    }
    const unsigned* sorted = m.key[src];
    hipLaunchKernelGGL(ibm_head_count_kernel, dim3(ntiles), dim3(256), 0, s, sorted, n, m.tcnt);
    hipLaunchKernelGGL(ibm_head_scan_kernel, dim3(1), dim3(256), 0, s, m.tcnt, ntiles, n, m.counts, m.csr);
    hipLaunchKernelGGL(ibm_head_compact_kernel, dim3(ntiles), dim3(256), 0, s, sorted, n, m.tcnt, a.g, m.cell, m.csr);
    hipLaunchKernelGGL(ibm_vbar_kernel, dim3(vbar_blocks(n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ibm_vbar(const IbmArgs& a, hipStream_t s) {
    if (a.ncell <= 0) return hipSuccess;
    hipLaunchKernelGGL(ibm_vbar_kernel, dim3(vbar_blocks(a.ncell)), dim3(256), 0, s, a);
    return hipGetLastError();
}

int ibm_blocks(int ncell) { return (ncell + 255) / 256; }

template <typename real>
hipError_t launch_ibm(Field4<real> f, const IbmArgs& a, hipStream_t s) {
    if (a.ncell <= 0) return hipSuccess;
    const int nblk = ibm_blocks(a.ncell);
    hipLaunchKernelGGL((ibm_cells_kernel<real>), dim3(nblk), dim3(256), 0, s, f, a);
    hipLaunchKernelGGL(ibm_final_kernel, dim3(1), dim3(256), 0, s, a, nblk);
    hipLaunchKernelGGL((ibm_resid_kernel<real>), dim3((a.npts + 255) / 256), dim3(256), 0, s, f, a);
    return hipGetLastError();
}

template hipError_t launch_alm<float>(Field4<float>, const AlmArgs&, hipStream_t);
template hipError_t launch_alm<double>(Field4<double>, const AlmArgs&, hipStream_t);
template hipError_t launch_ibm<float>(Field4<float>, const IbmArgs&, hipStream_t);
template hipError_t launch_ibm<double>(Field4<double>, const IbmArgs&, hipStream_t);

}  // namespace gks
