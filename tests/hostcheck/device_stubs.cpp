// Stand-ins for the device-side launch functions, so the host layers of the
// library (the planner and the C ABI) link into a host-only test program
// built with AddressSanitizer and UndefinedBehaviorSanitizer.  The program
// never reaches a launch: without a GPU every load stops at its first device
// allocation.  A call that did get here aborts.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "device_plan.hpp"
#include "kernels.hpp"

namespace {
[[noreturn]] void reached(const char* f) {
    std::fprintf(stderr, "device stand-in %s was called\n", f);
    std::abort();
}
}  // namespace

namespace spt {
bool launch_ec(int, int, int, int, int, int, const EcArgs&, hipStream_t) { reached("launch_ec"); }
bool pick_ec_exists(int nmodes, int rank, int, int, int) {
    return nmodes >= 2 && nmodes <= 8 && (rank == 8 || rank == 16 || rank == 32 || rank == 64 || rank == 128);
}
int forward_blocks(int64_t) { reached("forward_blocks"); }
bool launch_forward(int, int, int, int, const ForwardArgs&, hipStream_t) { reached("launch_forward"); }
void launch_to_bf16(const float*, uint16_t*, int64_t, hipStream_t) { reached("launch_to_bf16"); }
void launch_fixup(int, const FixupArgs&, hipStream_t) { reached("launch_fixup"); }
void launch_remap(int, int64_t, const uint32_t*, uint32_t*, const int32_t* const*, int, hipStream_t) {
    reached("launch_remap");
}
int stage_chunk(int, int64_t) { reached("stage_chunk"); }
void launch_stage_tables(int, const int32_t*, int64_t, int32_t*, uint16_t*, int32_t*, uint16_t*, hipStream_t) {
    reached("launch_stage_tables");
}
void launch_remap_staged(int, int64_t, const uint32_t*, uint32_t*, const int32_t*, const uint16_t*, hipStream_t) {
    reached("launch_remap_staged");
}
int gram_blocks(int64_t) { reached("gram_blocks"); }
void launch_gram_partial(int, const float*, int64_t, double*, hipStream_t) { reached("launch_gram_partial"); }
void launch_reduce_partials(const double*, int, int, double*, hipStream_t) { reached("launch_reduce_partials"); }
void launch_normal_inverse(int, int, int, const double*, double*, int32_t*, hipStream_t) {
    reached("launch_normal_inverse");
}
int solve_blocks(int64_t) { reached("solve_blocks"); }
void launch_solve_rows(int, const float*, const double*, int64_t, float*, double*, double*, hipStream_t) {
    reached("launch_solve_rows");
}
void launch_als_finish(int, int, int, const double*, const double*, double*, double*, double, int, double*,
                       hipStream_t) {
    reached("launch_als_finish");
}
void launch_scale_cols(int, float*, int64_t, const double*, hipStream_t) { reached("launch_scale_cols"); }
void launch_copy_probe(const void*, void*, int64_t, hipStream_t) { reached("launch_copy_probe"); }
void launch_zero_i32(int32_t*, int, hipStream_t) { reached("launch_zero_i32"); }
hipError_t noalloc_scratch(void**) { reached("noalloc_scratch"); }
DevicePlanError build_plan_device(int, const int64_t*, int64_t, const int32_t*, const float*, const PlanOptions&,
                                  const RecordLayout&, int, hipStream_t, const DeviceAlloc&, DevicePlan*,
                                  std::string* msg) {
    *msg = "no device in the host-only build";
    return DevicePlanError::kHip;
}
}  // namespace spt
