// gks_stats.hip -- running flow statistics of the cell velocity U = (rho U)/rho (Sections 4.1, 4.2,
// 4.3.2): time mean, RMS, Reynolds stresses and TKE = (<U'^2> + <V'^2> + <W'^2>) / (2 U_inf^2).
// One thread per cell updates the mean and the co-moments by Welford's recurrence in FP64
// (no cancellation between the second moment and the squared mean); results are deterministic.
#include "gks_stats.h"

namespace gks {

template <typename real>
__global__ void __launch_bounds__(256) stats_accum_kernel(Field4<real> f, StatsArgs s, double inv_n) {
    const long long n = (long long)s.g.n[0] * s.g.n[1] * s.g.n[2];
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int i = (int)(c % s.g.n[0]);
    const long long r = c / s.g.n[0];
    const int j = (int)(r % s.g.n[1]);
    const int k = (int)(r / s.g.n[1]);
    const long long p = s.g.pad0 + i * s.g.st[0] + j * s.g.st[1] + (long long)k * s.g.st[2];
    const double rho = s.rho_ref + (double)f.v[0][p];
    double u[3], d[3], d2[3];
    for (int a = 0; a < 3; ++a) {
        u[a] = (double)f.v[1 + a][p] / rho;
        const double m = s.buf[a * n + c];
        d[a] = u[a] - m;
        const double mn = m + d[a] * inv_n;
        d2[a] = u[a] - mn;
        s.buf[a * n + c] = mn;
    }
    // co-moments xx, yy, zz, xy, xz, yz
    s.buf[3 * n + c] += d[0] * d2[0];
    s.buf[4 * n + c] += d[1] * d2[1];
    s.buf[5 * n + c] += d[2] * d2[2];
    s.buf[6 * n + c] += d[0] * d2[1];
    s.buf[7 * n + c] += d[0] * d2[2];
    s.buf[8 * n + c] += d[1] * d2[2];
}

__global__ void __launch_bounds__(256) stats_final_kernel(StatsArgs s, double inv_n, double inv_u2, double* mean,
                                                          double* rms, double* stress, double* tke) {
    const long long n = (long long)s.g.n[0] * s.g.n[1] * s.g.n[2];
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    if (mean)
        for (int a = 0; a < 3; ++a) mean[a * n + c] = s.buf[a * n + c];
    const double vx = s.buf[3 * n + c] * inv_n, vy = s.buf[4 * n + c] * inv_n, vz = s.buf[5 * n + c] * inv_n;
    if (rms) {
        rms[c] = sqrt(vx);
        rms[n + c] = sqrt(vy);
        rms[2 * n + c] = sqrt(vz);
    }
    if (stress)
        for (int a = 0; a < 3; ++a) stress[a * n + c] = s.buf[(6 + a) * n + c] * inv_n;
    if (tke) tke[c] = 0.5 * (vx + vy + vz) * inv_u2;
}

__global__ void stats_zero_kernel(double* buf, long long m) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) buf[i] = 0.0;
}

template <typename real>
hipError_t launch_stats_accum(Field4<real> f, const StatsArgs& s, double inv_n, hipStream_t st) {
    const long long n = (long long)s.g.n[0] * s.g.n[1] * s.g.n[2];
    hipLaunchKernelGGL((stats_accum_kernel<real>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, f, s, inv_n);
    return hipGetLastError();
}

hipError_t launch_stats_final(const StatsArgs& s, double inv_n, double inv_u2, double* mean, double* rms,
                              double* stress, double* tke, hipStream_t st) {
    const long long n = (long long)s.g.n[0] * s.g.n[1] * s.g.n[2];
    hipLaunchKernelGGL(stats_final_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, inv_n, inv_u2,
                       mean, rms, stress, tke);
    return hipGetLastError();
}

hipError_t launch_stats_zero(const StatsArgs& s, hipStream_t st) {
    const long long m = 9LL * s.g.n[0] * s.g.n[1] * s.g.n[2];
    hipLaunchKernelGGL(stats_zero_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, s.buf, m);
    return hipGetLastError();
}

template hipError_t launch_stats_accum<float>(Field4<float>, const StatsArgs&, double, hipStream_t);
template hipError_t launch_stats_accum<double>(Field4<double>, const StatsArgs&, double, hipStream_t);

}  // namespace gks
