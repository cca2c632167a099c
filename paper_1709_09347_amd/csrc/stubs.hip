#include "cbs_internal.hpp"
using namespace cbs;
extern "C" {
int32_t cbs_bicg(cbs_system*, double, int32_t, const double*, int32_t, const void*, const cbs_params*, void*, void*, int32_t*, double*, cbs_info*, void*) { set_error("not built"); return CBS_EINVAL; }
int32_t cbs_solve(cbs_system*, double, const cbs_params*, const void*, int32_t, double*, double*, void*, int32_t*, cbs_info*, void*) { set_error("not built"); return CBS_EINVAL; }
int32_t cbs_solve_batched(int32_t, cbs_system* const*, int32_t, const double*, const cbs_params*, const void* const*, int32_t, double*, int32_t*, cbs_info*, void*) { set_error("not built"); return CBS_EINVAL; }
int32_t cbs_grad_vloc(cbs_system*, int32_t, const int32_t*, void*, void*) { set_error("not built"); return CBS_EINVAL; }
}
