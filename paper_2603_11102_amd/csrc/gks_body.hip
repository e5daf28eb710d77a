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
        // trilinear sampling of U = (rho U)/rho at cell centres
        int i0[3];
        double w1[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double fc = (X[d] - a.g.x0[d]) / a.g.h[d] - 0.5;
            const double fl = floor(fc);
            i0[d] = (int)fl;
            w1[d] = fc - fl;
        }
        double U[3] = {0.0, 0.0, 0.0};
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
                    for (int c = 0; c < 3; ++c) U[c] += w * ((double)f.v[1 + c][q] / rho);
                }
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

// static V-bar_c = sum over the points whose support holds c of W V_p, and the cell velocity
// v-bar_c = sum W V_p v_p / V-bar_c (fixed point order)
__global__ void __launch_bounds__(256) ibm_vbar_kernel(IbmArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (a.ncell_dev ? *a.ncell_dev : a.ncell)) return;
    const int i = a.cell[3 * c], j = a.cell[3 * c + 1], k = a.cell[3 * c + 2];
    double v = 0.0, mv[3] = {0.0, 0.0, 0.0};
    for (int e = a.csr[c]; e < a.csr[c + 1]; ++e) {
        const int p = a.ent[e];
        const double wv = ibm_weight(a.g, a.xyz + 3 * p, i, j, k) * (a.g.h[0] * a.dS[p]);
        v += wv;
        if (a.vel)
            for (int d = 0; d < 3; ++d) mv[d] += wv * a.vel[3 * p + d];
    }
    a.vbar[c] = v;
    for (int d = 0; d < 3; ++d) a.vbar_vel[3 * c + d] = (a.vel && v > 0.0) ? mv[d] / v : 0.0;
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
// the host binning (cells ascending, x fastest; points ascending within a cell)
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ long long flat_cell(const GridDesc& g, int i, int j, int k) {
    return ((long long)k * g.n[1] + j) * g.n[0] + i;
}

// Rigid motion to t^{n+1}: X_p = X_p(t0) + V tau + (R - I) r with r = X_p(t0) - c0 and
// (R - I) r = sin(theta) k x r + (1 - cos theta) k x (k x r) (Rodrigues), v_p = V + omega x R r.
// Lowest support cell per axis, clamped into the interior when the support leaves it (then the
// flag stops the forcing); one count per support cell.
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
    int b[3];
    bool out = false;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        const double f = (X[x] - a.g.x0[x]) / a.g.h[x] - 0.5;
        if (f >= 1.0 && f < (double)(a.g.n[x] - 2)) {
            b[x] = (int)floor(f);
        } else {  // also NaN
            out = true;
            b[x] = f >= 1.0 ? a.g.n[x] - 3 : 1;
        }
        m.xyz[3 * p + x] = X[x];
        m.pvel[3 * p + x] = v[x];
        m.base[3 * p + x] = b[x];
    }
    if (out) atomicOr(&a.st->ibm_outside, 1);
    for (int dk = -1; dk <= 2; ++dk)
        for (int dj = -1; dj <= 2; ++dj)
            for (int di = -1; di <= 2; ++di) atomicAdd(&m.dcnt[flat_cell(a.g, b[0] + di, b[1] + dj, b[2] + dk)], 1);
}

// block sums of (cells with a count, entries) over BIN_CELLS consecutive cells, 16 per thread
__global__ void __launch_bounds__(256) ibm_bincount_kernel(IbmMoveArgs m, long long ncells) {
    __shared__ int sc[256], se[256];
    const long long x0 = (long long)blockIdx.x * BIN_CELLS + 16 * threadIdx.x;
    int c = 0, e = 0;
    for (int q = 0; q < 16; ++q) {
        if (x0 + q < ncells) {
            const int v = m.dcnt[x0 + q];
            c += v > 0;
            e += v;
        }
    }
    sc[threadIdx.x] = c;
    se[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sc[threadIdx.x] += sc[threadIdx.x + w];
            se[threadIdx.x] += se[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        m.blk[2 * blockIdx.x] = sc[0];
        m.blk[2 * blockIdx.x + 1] = se[0];
    }
}

// exclusive scan of the block sums in place (one workgroup, a contiguous run of blocks per thread);
// totals to counts[0..1] and csr[cells] = entries
__global__ void __launch_bounds__(1024) ibm_binscan_kernel(IbmMoveArgs m) {
    __shared__ int sc[1024], se[1024];
    const int per = (m.nblk + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(m.nblk, lo + per);
    int c = 0, e = 0;
    for (int b = lo; b < hi; ++b) {
        c += m.blk[2 * b];
        e += m.blk[2 * b + 1];
    }
    sc[threadIdx.x] = c;
    se[threadIdx.x] = e;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {  // inclusive Hillis-Steele scan
        const int tc = threadIdx.x >= w ? sc[threadIdx.x - w] : 0;
        const int te = threadIdx.x >= w ? se[threadIdx.x - w] : 0;
        __syncthreads();
        sc[threadIdx.x] += tc;
        se[threadIdx.x] += te;
        __syncthreads();
    }
    c = sc[threadIdx.x] - c;
    e = se[threadIdx.x] - e;
    for (int b = lo; b < hi; ++b) {
        const int bc = m.blk[2 * b], be = m.blk[2 * b + 1];
        m.blk[2 * b] = c;
        m.blk[2 * b + 1] = e;
        c += bc;
        e += be;
    }
    if (threadIdx.x == 1023) {
        m.counts[0] = sc[1023];
        m.counts[1] = se[1023];
        m.csr[sc[1023]] = se[1023];
    }
}

// cells with a count, in ascending order: (i, j, k), csr start, and the start as the fill cursor
__global__ void __launch_bounds__(256) ibm_bincompact_kernel(IbmMoveArgs m, GridDesc g, long long ncells) {
    __shared__ int sc[256], se[256];
    const long long x0 = (long long)blockIdx.x * BIN_CELLS + 16 * threadIdx.x;
    int v[16];
    int c = 0, e = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        v[q] = x0 + q < ncells ? m.dcnt[x0 + q] : 0;
        c += v[q] > 0;
        e += v[q];
    }
    sc[threadIdx.x] = c;
    se[threadIdx.x] = e;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {
        const int tc = threadIdx.x >= w ? sc[threadIdx.x - w] : 0;
        const int te = threadIdx.x >= w ? se[threadIdx.x - w] : 0;
        __syncthreads();
        sc[threadIdx.x] += tc;
        se[threadIdx.x] += te;
        __syncthreads();
    }
    int ci = m.blk[2 * blockIdx.x] + sc[threadIdx.x] - c;
    int ei = m.blk[2 * blockIdx.x + 1] + se[threadIdx.x] - e;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        if (v[q] > 0) {
            const long long x = x0 + q;
            m.cell[3 * ci] = (int)(x % g.n[0]);
            m.cell[3 * ci + 1] = (int)((x / g.n[0]) % g.n[1]);
            m.cell[3 * ci + 2] = (int)(x / ((long long)g.n[0] * g.n[1]));
            m.csr[ci] = ei;
            m.dcnt[x] = ei;
            ++ci;
            ei += v[q];
        }
    }
}

// every (point, support cell) pair takes a slot of its cell
__global__ void __launch_bounds__(256) ibm_binfill_kernel(IbmArgs a, IbmMoveArgs m) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 64LL * a.npts) return;
    const int p = (int)(e >> 6), q = (int)(e & 63);
    const int i = m.base[3 * p] + (q & 3) - 1, j = m.base[3 * p + 1] + ((q >> 2) & 3) - 1,
              k = m.base[3 * p + 2] + (q >> 4) - 1;
    const int slot = atomicAdd(&m.dcnt[flat_cell(a.g, i, j, k)], 1);
    m.ent[slot] = p;
}

// points of a cell in ascending order (insertion sort); the cell's counter back to zero
__global__ void __launch_bounds__(256) ibm_binsort_kernel(IbmArgs a, IbmMoveArgs m) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m.counts[0]) return;
    const int lo = m.csr[c], hi = m.csr[c + 1];
    for (int x = lo + 1; x < hi; ++x) {
        const int key = m.ent[x];
        int y = x - 1;
        while (y >= lo && m.ent[y] > key) {
            m.ent[y + 1] = m.ent[y];
            --y;
        }
        m.ent[y + 1] = key;
    }
    m.dcnt[flat_cell(a.g, m.cell[3 * c], m.cell[3 * c + 1], m.cell[3 * c + 2])] = 0;
}

hipError_t launch_ibm_move(const IbmArgs& a, const IbmMoveArgs& m, hipStream_t s) {
    if (a.npts <= 0) return hipSuccess;
    const long long ncells = (long long)a.g.n[0] * a.g.n[1] * a.g.n[2];
    const unsigned pblocks = (unsigned)((a.npts + 255) / 256);
    const unsigned eblocks = (unsigned)((64LL * a.npts + 255) / 256);
    hipLaunchKernelGGL(ibm_move_kernel, dim3(pblocks), dim3(256), 0, s, a, m);
    hipLaunchKernelGGL(ibm_bincount_kernel, dim3(m.nblk), dim3(256), 0, s, m, ncells);
    hipLaunchKernelGGL(ibm_binscan_kernel, dim3(1), dim3(1024), 0, s, m);
    hipLaunchKernelGGL(ibm_bincompact_kernel, dim3(m.nblk), dim3(256), 0, s, m, a.g, ncells);
    hipLaunchKernelGGL(ibm_binfill_kernel, dim3(eblocks), dim3(256), 0, s, a, m);
    hipLaunchKernelGGL(ibm_binsort_kernel, dim3(eblocks), dim3(256), 0, s, a, m);
    hipLaunchKernelGGL(ibm_vbar_kernel, dim3(eblocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ibm_vbar(const IbmArgs& a, hipStream_t s) {
    if (a.ncell <= 0) return hipSuccess;
    hipLaunchKernelGGL(ibm_vbar_kernel, dim3((a.ncell + 255) / 256), dim3(256), 0, s, a);
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
