// CPU stand-in for <hip/hip_runtime.h>: runs the library's HIP kernels on the
// host, for tests only.
//
// A launch runs its workgroups one after another; the threads of a workgroup
// are fibers (ucontext) of one OS thread, scheduled round-robin.  A thread
// yields at __syncthreads() (all threads of the workgroup must arrive) and at
// cross-lane operations (ds_bpermute, readlane, shfl_xor: all 64 lanes of
// the wave must arrive; the results are then formed from every lane's
// operand).  A thread that waits for lanes that never come is reported as a
// deadlock.  __shared__ variables are static locals (one workgroup runs at a
// time); dynamic LDS is a per-launch host buffer.  Device memory is host
// memory that ends at a PROT_NONE page, so a read or write past the end of
// an allocation faults at once.
#pragma once

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <functional>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define __shared__ static
#define HIP_DYNAMIC_SHARED(type, var) type* var = reinterpret_cast<type*>(cpuhip::dynamic_shared());
#define HIP_SYMBOL(x) (&(x))

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint3 {
    unsigned x, y, z;
};
struct alignas(16) uint4 {
    unsigned x, y, z, w;
};
struct alignas(16) float4 {
    float x, y, z, w;
};
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return uint4{a, b, c, d}; }
inline float4 make_float4(float a, float b, float c, float d) { return float4{a, b, c, d}; }

typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorInvalidDevice = 101,
    hipErrorLaunchFailure = 719
} hipError_t;
typedef struct cpuhip_stream* hipStream_t;
typedef struct cpuhip_event* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice,
                     hipMemcpyDefault };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount, hipDeviceAttributeMaxSharedMemoryPerBlock };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize };
struct hipFuncAttributes {
    size_t sharedSizeBytes;
    int maxThreadsPerBlock;
};
#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u

namespace cpuhip {
struct Thread {
    uint3 tid;
};
uint3 thread_idx();
uint3 block_idx();
dim3 block_dim();
dim3 grid_dim();
void* dynamic_shared();
void syncthreads();
int bpermute(int addr, int v);
int readlane(int v, int lane);
float shfl_xor(float v, int mask, int width);
void launch(const std::function<void()>& body, dim3 grid, dim3 block, size_t shmem);
}  // namespace cpuhip

#define threadIdx (cpuhip::thread_idx())
#define blockIdx (cpuhip::block_idx())
#define blockDim (cpuhip::block_dim())
#define gridDim (cpuhip::grid_dim())

inline void __syncthreads() { cpuhip::syncthreads(); }
inline unsigned __umulhi(unsigned a, unsigned b) { return (unsigned)(((uint64_t)a * b) >> 32); }
inline float __uint_as_float(unsigned u) {
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
inline unsigned __float_as_uint(float f) {
    unsigned u;
    std::memcpy(&u, &f, 4);
    return u;
}
inline int __builtin_amdgcn_ds_bpermute(int addr, int v) { return cpuhip::bpermute(addr, v); }
inline int __builtin_amdgcn_readlane(int v, int lane) { return cpuhip::readlane(v, lane); }
inline float __shfl_xor(float v, int mask, int width = 64) { return cpuhip::shfl_xor(v, mask, width); }
inline void __builtin_amdgcn_fence(int, const char*) {}
inline void __builtin_amdgcn_wave_barrier() {}

template <typename F, typename... A>
inline void hipLaunchKernelGGL(F kernel, dim3 grid, dim3 block, size_t shmem, hipStream_t, A... args) {
    cpuhip::launch([&]() { kernel(args...); }, grid, block, shmem);
}

hipError_t hipMalloc(void** p, size_t bytes);
template <typename T>
inline hipError_t hipMalloc(T** p, size_t bytes) {
    return hipMalloc(reinterpret_cast<void**>(p), bytes);
}
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags = 0);
template <typename T>
inline hipError_t hipHostMalloc(T** p, size_t bytes, unsigned flags = 0) {
    return hipHostMalloc(reinterpret_cast<void**>(p), bytes, flags);
}
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t);
hipError_t hipMemset(void* p, int v, size_t bytes);
hipError_t hipMemsetAsync(void* p, int v, size_t bytes, hipStream_t);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipDeviceSynchronize();
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetDevice(int* d);
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int dev);
hipError_t hipFuncGetAttributes(hipFuncAttributes* a, const void* f);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void* f, int block, size_t lds);
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute a, int v);
hipError_t hipGetSymbolAddress(void** p, const void* sym);
