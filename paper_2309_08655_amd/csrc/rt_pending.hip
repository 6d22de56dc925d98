// Entry points whose kernels are not built yet: they validate nothing and
// report RT_EUNSUPPORTED.
#include "rt_common.hpp"

using namespace rtd;

extern "C" int rt_flux_grad(const rt_star*, const rt_tol*, uint64_t, int64_t, const double*, int32_t, double, int32_t,
                            int32_t, int32_t, const double*, double*, double*, void*, size_t, void*) {
    return fail(RT_EUNSUPPORTED, "rt_flux_grad: not available in this build");
}
extern "C" size_t rt_flux_grad_workspace_size(int64_t, int32_t, int32_t, int32_t) { return 0; }
