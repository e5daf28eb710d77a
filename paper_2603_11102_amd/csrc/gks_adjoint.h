// gks_adjoint.h -- discrete adjoint of the S2O4 step (internal).
#pragma once

#include <stddef.h>

namespace gks {

size_t adjoint_workspace_bytes(int nx, int ny, int nz, int n_act);

}  // namespace gks
