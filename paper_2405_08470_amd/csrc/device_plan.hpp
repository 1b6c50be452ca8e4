// Preprocessing on the device: the per-nonzero work of the planner (row
// degrees, ranks of nonzeros within their rows, each mode's stream order,
// remap ids, next positions, record packing, ||X||^2) runs in HIP kernels
// built on a stable LSD radix sort; Alg. 1 itself (the least-loaded
// assignment of rows or pieces to partitions, Sec. 3.4) runs on the host
// from the degrees, with the host planner's own code.  Every integer result
// is identical to the host planner's; ||X||^2 differs only in the order of
// its FP64 summation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "plan.hpp"

namespace spt {

struct DevicePlan {
    int32_t kappa = 0;
    int64_t cap = 0;
    ModePlan mode[kMaxModes];                 // tables only: part, order, remap stay empty
    uint32_t* rec0 = nullptr;                 // stream in mode 0's order (copies == 0)
    int32_t* nxt[kMaxModes] = {};             // next positions (copies == 0)
    uint32_t* rec_mode[kMaxModes] = {};       // one stream per mode (copies == 1)
    std::vector<int32_t> order0;              // input nonzero at each mode-0 position
    double norm_sq = 0.0;
};

// Device memory that outlives the call (the streams and next positions),
// owned by the caller; returns nullptr on failure.
using DeviceAlloc = std::function<void*(size_t bytes)>;

enum class DevicePlanError { kNone, kInvalid, kRange, kOom, kHip };

// Plans and packs the tensor on the device (stream s; synchronous on return).
// idx/val are host arrays ([N][nnz] int32, [nnz] float).  Returns kNone, or
// an error with a message in *msg (the same message as the host validator
// for an index out of range).
DevicePlanError build_plan_device(int N, const int64_t* dims, int64_t nnz, const int32_t* idx,
                                  const float* val, const PlanOptions& opt,
                                  const RecordLayout& lay, int copies, hipStream_t s,
                                  const DeviceAlloc& persist, DevicePlan* out, std::string* msg);

}  // namespace spt
