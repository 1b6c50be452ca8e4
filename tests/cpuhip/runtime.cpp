// Runtime of the CPU stand-in for HIP (see hip/hip_runtime.h): fiber
// scheduling of workgroups, wave-level exchanges, guarded device memory.
#include <sys/mman.h>
#include <ucontext.h>
#include <unistd.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "hip/hip_runtime.h"

namespace cpuhip {
namespace {

[[noreturn]] void die(const char* what) {
    std::fprintf(stderr, "cpuhip: %s\n", what);
    std::fflush(stderr);
    std::abort();
}

enum Wait { kRun = 0, kBarrier, kPermute, kReadlane, kXor, kDone };

struct Fiber {
    ucontext_t ctx;
    void* stack = nullptr;
    uint3 tid{};
    int wave = 0, lane = 0;
    Wait wait = kRun;
    int a = 0, b = 0;   // operands of the pending exchange
    float f = 0.0f;
    int ri = 0;         // its result
    float rf = 0.0f;
};

constexpr size_t kStack = 256 * 1024;

struct Launch {
    const std::function<void()>* body = nullptr;
    dim3 grid, block;
    uint3 bid{};
    std::vector<Fiber> fib;
    Fiber* cur = nullptr;
    ucontext_t sched;
    std::vector<unsigned char> lds;
};

Launch g;

void trampoline() {
    (*g.body)();
    g.cur->wait = kDone;
    swapcontext(&g.cur->ctx, &g.sched);
    die("finished fiber resumed");
}

void yield_as(Wait w) {
    Fiber* self = g.cur;
    self->wait = w;
    swapcontext(&self->ctx, &g.sched);
}

// Releases the exchanges and barriers whose participants have all arrived;
// returns true if any fiber became runnable.
bool release() {
    const int n = (int)g.fib.size();
    bool any = false;
    // workgroup barrier: every fiber that has not finished waits there
    bool all_bar = true, some_bar = false;
    for (auto& f : g.fib) {
        if (f.wait == kDone) continue;
        if (f.wait != kBarrier) all_bar = false;
        else some_bar = true;
    }
    if (some_bar && all_bar) {
        for (auto& f : g.fib)
            if (f.wait == kBarrier) f.wait = kRun;
        for (auto& f : g.fib)
            if (f.wait == kDone) die("__syncthreads reached after some threads returned");
        return true;
    }
    const int nwaves = (n + 63) / 64;
    for (int w = 0; w < nwaves; ++w) {
        const int l0 = w * 64, l1 = std::min(n, l0 + 64);
        const Wait k = g.fib[l0].wait;
        if (k != kPermute && k != kReadlane && k != kXor) continue;
        bool ready = true;
        for (int i = l0; i < l1; ++i)
            if (g.fib[i].wait != k) ready = false;
        if (!ready) continue;
        const int width = l1 - l0;
        for (int i = l0; i < l1; ++i) {
            Fiber& f = g.fib[i];
            if (k == kPermute) {
                const int src = (f.a >> 2) & 63;
                if (src >= width) die("ds_bpermute from a lane outside the workgroup");
                f.ri = g.fib[l0 + src].b;
            } else if (k == kReadlane) {
                if (f.b != g.fib[l0].b) die("readlane with a lane index that differs across the wave");
                if (f.b < 0 || f.b >= width) die("readlane of a lane outside the workgroup");
                f.ri = g.fib[l0 + f.b].a;
            } else {
                const int src = (f.lane ^ f.a);
                if (src >= width || (src / f.b) != (f.lane / f.b)) die("shfl_xor outside its width");
                f.rf = g.fib[l0 + src].f;
            }
            f.wait = kRun;
        }
        any = true;
    }
    return any;
}

void run_block() {
    const int n = (int)g.fib.size();
    for (int i = 0; i < n; ++i) {
        Fiber& f = g.fib[i];
        getcontext(&f.ctx);
        f.ctx.uc_stack.ss_sp = f.stack;
        f.ctx.uc_stack.ss_size = kStack;
        f.ctx.uc_link = nullptr;
        makecontext(&f.ctx, trampoline, 0);
        f.wait = kRun;
    }
    for (;;) {
        bool ran = false, live = false;
        for (int i = 0; i < n; ++i) {
            Fiber& f = g.fib[i];
            if (f.wait == kDone) continue;
            live = true;
            if (f.wait != kRun) continue;
            g.cur = &f;
            swapcontext(&g.sched, &f.ctx);
            ran = true;
        }
        if (!live) return;
        if (!release() && !ran) {
            for (int i = 0; i < n; ++i)
                if (g.fib[i].wait != kDone && g.fib[i].wait != kRun)
                    std::fprintf(stderr, "  thread %d (wave %d lane %d) waits (kind %d)\n", i, g.fib[i].wave,
                                 g.fib[i].lane, (int)g.fib[i].wait);
            die("deadlock: threads wait for lanes or a barrier that never come");
        }
    }
}

// ---- guarded device memory
struct Region {
    void* base;
    size_t total;
};
std::mutex g_mem_mutex;
std::map<void*, Region> g_regions;
hipError_t g_last = hipSuccess;

}  // namespace

uint3 thread_idx() { return g.cur->tid; }
uint3 block_idx() { return g.bid; }
dim3 block_dim() { return g.block; }
dim3 grid_dim() { return g.grid; }
void* dynamic_shared() { return g.lds.data(); }
void syncthreads() { yield_as(kBarrier); }

int bpermute(int addr, int v) {
    g.cur->a = addr;
    g.cur->b = v;
    yield_as(kPermute);
    return g.cur->ri;
}

int readlane(int v, int lane) {
    g.cur->a = v;
    g.cur->b = lane;
    yield_as(kReadlane);
    return g.cur->ri;
}

float shfl_xor(float v, int mask, int width) {
    g.cur->a = mask;
    g.cur->b = width;
    g.cur->f = v;
    yield_as(kXor);
    return g.cur->rf;
}

void launch(const std::function<void()>& body, dim3 grid, dim3 block, size_t shmem) {
    const int n = (int)(block.x * block.y * block.z);
    if (n <= 0 || n > 1024) die("workgroup size outside 1..1024");
    if (shmem > 160 * 1024) die("dynamic LDS above 160 KB");
    g.body = &body;
    g.grid = grid;
    g.block = block;
    if ((int)g.fib.size() != n) {
        for (auto& f : g.fib) munmap(f.stack, kStack);
        g.fib.assign(n, Fiber{});
        for (int i = 0; i < n; ++i) {
            g.fib[i].stack = mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
            if (g.fib[i].stack == MAP_FAILED) die("fiber stack");
        }
    }
    for (int i = 0; i < n; ++i) {
        g.fib[i].tid = uint3{(unsigned)i % block.x, (unsigned)(i / block.x) % block.y, (unsigned)(i / (block.x * block.y))};
        g.fib[i].wave = i / 64;
        g.fib[i].lane = i % 64;
    }
    g.lds.assign(shmem + 16, 0xCD);  // not zero: kernels must fill what they read
    for (unsigned z = 0; z < grid.z; ++z)
        for (unsigned y = 0; y < grid.y; ++y)
            for (unsigned x = 0; x < grid.x; ++x) {
                g.bid = uint3{x, y, z};
                run_block();
            }
}

}  // namespace cpuhip

using cpuhip::g_last;

hipError_t hipMalloc(void** p, size_t bytes) {
    const size_t page = 4096;
    const size_t b16 = (std::max<size_t>(bytes, 1) + 15) / 16 * 16;
    const size_t body = (b16 + page - 1) / page * page;
    const size_t total = body + 2 * page;
    void* base = mmap(nullptr, total, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (base == MAP_FAILED) return g_last = hipErrorOutOfMemory;
    char* c = static_cast<char*>(base);
    mprotect(c, page, PROT_NONE);                  // before the region
    mprotect(c + page + body, page, PROT_NONE);    // right after the allocation
    void* ptr = c + page + body - b16;
    std::memset(ptr, 0xAB, b16);                    // not zero: nothing may read what it did not write
    std::lock_guard<std::mutex> lock(cpuhip::g_mem_mutex);
    cpuhip::g_regions[ptr] = cpuhip::Region{base, total};
    *p = ptr;
    return hipSuccess;
}

hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    std::lock_guard<std::mutex> lock(cpuhip::g_mem_mutex);
    auto it = cpuhip::g_regions.find(p);
    if (it == cpuhip::g_regions.end()) return g_last = hipErrorInvalidValue;
    munmap(it->second.base, it->second.total);
    cpuhip::g_regions.erase(it);
    return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
    *p = std::malloc(std::max<size_t>(bytes, 1));
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
    if (bytes) std::memmove(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind k, hipStream_t) {
    return hipMemcpy(dst, src, bytes, k);
}
hipError_t hipMemset(void* p, int v, size_t bytes) {
    if (bytes) std::memset(p, v, bytes);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int v, size_t bytes, hipStream_t) { return hipMemset(p, v, bytes); }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }

struct cpuhip_stream {
    int unused;
};
struct cpuhip_event {
    double t;
};
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = new cpuhip_stream{0};
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
    *e = new cpuhip_event{0.0};
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    e->t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    *ms = (float)(b->t - a->t);
    return hipSuccess;
}
hipError_t hipGetLastError() {
    hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "cpuhip error"; }
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
    // four CUs, so each wave of the elementwise kernel walks several partitions
    *v = a == hipDeviceAttributeMultiprocessorCount ? 4 : 160 * 1024;
    return hipSuccess;
}
hipError_t hipFuncGetAttributes(hipFuncAttributes* a, const void*) {
    a->sharedSizeBytes = 0;
    a->maxThreadsPerBlock = 1024;
    return hipSuccess;
}
// every kernel reports the same occupancy, so the library takes the forms
// it prefers at equal occupancy (builds with SPT_EC_FORM force one)
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) {
    *n = 16;
    return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int v) {
    return v <= 160 * 1024 ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
    *p = const_cast<void*>(sym);
    return hipSuccess;
}
