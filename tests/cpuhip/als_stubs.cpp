// The CP-ALS dense kernels (FP64 matrix-core code) and the device planner
// are not part of the CPU build: these stand-ins fail loudly if reached.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "device_plan.hpp"
#include "kernels.hpp"

namespace {
[[noreturn]] void reached(const char* f) {
    std::fprintf(stderr, "not in the CPU build: %s\n", f);
    std::abort();
}
}  // namespace

namespace spt {
int gram_blocks(int64_t) { return 1; }  // workspace sizing only
void launch_gram_partial(int, const float*, int64_t, double*, hipStream_t) { reached("launch_gram_partial"); }
void launch_reduce_partials(const double*, int, int, double*, hipStream_t) { reached("launch_reduce_partials"); }
void launch_normal_inverse(int, int, int, const double*, double*, int32_t*, hipStream_t) {
    reached("launch_normal_inverse");
}
int solve_blocks(int64_t) { return 1; }
void launch_solve_rows(int, const float*, const double*, int64_t, float*, double*, double*, hipStream_t) {
    reached("launch_solve_rows");
}
void launch_als_finish(int, int, int, const double*, const double*, double*, double*, double, int, double*,
                       hipStream_t) {
    reached("launch_als_finish");
}
void launch_scale_cols(int, float*, int64_t, const double*, hipStream_t) { reached("launch_scale_cols"); }
void launch_zero_i32(int32_t*, int, hipStream_t) { reached("launch_zero_i32"); }
DevicePlanError build_plan_device(int, const int64_t*, int64_t, const int32_t*, const float*, const PlanOptions&,
                                  const RecordLayout&, int, hipStream_t, const DeviceAlloc&, DevicePlan*,
                                  std::string* msg) {
    *msg = "the device planner is not in the CPU build";
    return DevicePlanError::kHip;
}
}  // namespace spt
