#include "cbs_internal.hpp"
using namespace cbs;
extern "C" {
int32_t cbs_solve_batched(int32_t, cbs_system* const*, int32_t, const double*, const cbs_params*, const void* const*, int32_t, double*, int32_t*, cbs_info*, void*) { set_error("not built"); return CBS_EINVAL; }
int32_t cbs_grad_vloc(cbs_system*, int32_t, const int32_t*, void*, void*) { set_error("not built"); return CBS_EINVAL; }
}
