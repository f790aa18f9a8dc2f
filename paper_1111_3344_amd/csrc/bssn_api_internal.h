// bssn_api_internal.h -- validation and error helpers shared by the C-ABI
// translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/bssn.h"
#include "bssn_internal.h"

namespace bssn {
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int check_grid(const bssn_grid* g, int order);
int check_params(const bssn_params* p);
Patch make_patch(const bssn_grid* g);
Gauge make_gauge(const bssn_params* p);
struct ConstraintArgs;
int constraint_args(const bssn_grid* grid, const bssn_params* params,
                    const double* u, double* H, double* M, double* G,
                    const double* centres, int ncent, double r_exc,
                    const double* norms, ConstraintArgs* A);
}  // namespace bssn
