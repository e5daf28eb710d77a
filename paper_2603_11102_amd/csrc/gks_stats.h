// gks_stats.h -- running flow statistics (internal).
#pragma once

#include "gks_internal.h"

namespace gks {

struct StatsArgs {
    GridDesc g;
    double rho_ref;
    double* buf;  // 9 arrays of nx*ny*nz doubles: mean U, V, W; co-moments xx, yy, zz, xy, xz, yz
};

template <typename real>
hipError_t launch_stats_accum(Field4<real> f, const StatsArgs& s, double inv_n, hipStream_t st);
hipError_t launch_stats_final(const StatsArgs& s, double inv_n, double inv_u2, double* mean, double* rms,
                              double* stress, double* tke, hipStream_t st);
hipError_t launch_stats_zero(const StatsArgs& s, hipStream_t st);

}  // namespace gks
