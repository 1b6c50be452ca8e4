// Preprocessing on the device (see device_plan.hpp).  Building block: a
// stable LSD radix sort of (uint32 key, int32 value) pairs, 8 bits per pass.
// A pass histograms the digits of each 4096-element tile, scans the
// (digit, tile) counts in digit-major order and scatters; inside a tile the
// rank of an element among equal digits comes from wave ballots (lanes with
// the same digit) plus per-wave counts in LDS, in element order, so equal
// keys keep their order.
//
// With the sort, each mode's stream is built the way the host planner
// builds it: sorting by the segment id (rank of the (partition, row) pair)
// of modes 1, 2, ..., N-1, 0 gives mode 0's stream; each further sort by
// mode d's segment id gives mode d's stream (Sec. 3.4-3.5 with the stream
// order read as (z_d, i_d, z_{d-1}, i_{d-1}, ..., e)).
#include "device_plan.hpp"

#include <algorithm>
#include <cstring>
#include <memory>
#include <thread>

namespace spt {

namespace {

constexpr int kT = 256;          // threads per block
constexpr int kI = 16;           // elements per thread
constexpr int kTile = kT * kI;   // elements per tile

int bit_len(int64_t v) {
    int b = 0;
    while (v > 0) {
        ++b;
        v >>= 1;
    }
    return b;
}

unsigned grid_for(int64_t n, int threads = kT, int64_t max_blocks = 65536) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, max_blocks));
}

// ------------------------------------------------------------------ scans

// Chunks of kTile entries: exclusive sum (MAX = false) or inclusive max
// (MAX = true) within the chunk, in place; the chunk's total (sum or max)
// to sums[chunk].
template <bool MAX>
__global__ __launch_bounds__(kT) void scan_chunk_kernel(uint32_t* __restrict__ d, int64_t n,
                                                        uint32_t* __restrict__ sums) {
    __shared__ uint32_t ts[kT];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)tid * kI;
    uint32_t v[kI];
    uint32_t tot = 0;
#pragma unroll
    for (int j = 0; j < kI; ++j) {
        const int64_t i = base + j;
        v[j] = i < n ? d[i] : 0u;
        tot = MAX ? max(tot, v[j]) : tot + v[j];
    }
    ts[tid] = tot;
    __syncthreads();
    for (int off = 1; off < kT; off <<= 1) {
        const uint32_t x = tid >= off ? ts[tid - off] : 0u;
        __syncthreads();
        if (tid >= off) ts[tid] = MAX ? max(ts[tid], x) : ts[tid] + x;
        __syncthreads();
    }
    uint32_t run = tid ? ts[tid - 1] : 0u;
#pragma unroll
    for (int j = 0; j < kI; ++j) {
        const int64_t i = base + j;
        if (MAX) {
            run = max(run, v[j]);
            if (i < n) d[i] = run;
        } else {
            if (i < n) d[i] = run;
            run += v[j];
        }
    }
    if (tid == kT - 1) sums[blockIdx.x] = ts[kT - 1];
}

// Adds the scanned chunk totals: exclusive sums for MAX = false; for MAX =
// true `offs` holds inclusive maxima, so chunk c takes offs[c - 1].
template <bool MAX>
__global__ void scan_add_kernel(uint32_t* __restrict__ d, int64_t n, const uint32_t* __restrict__ offs) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / kTile;
        if (MAX) {
            if (c > 0) d[i] = max(d[i], offs[c - 1]);
        } else {
            d[i] += offs[c];
        }
    }
}

// Per-level chunk-total buffers for scans of up to `cap` entries.
struct ScanScratch {
    std::vector<uint32_t*> level;
    std::vector<int64_t> size;
};

// --------------------------------------------------------------- radix sort

__global__ __launch_bounds__(kT) void rs_hist_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                     int shift, uint32_t* __restrict__ hist,
                                                     int64_t ntiles) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll 4
    for (int j = 0; j < kI; ++j) {
        const int64_t i = base + (int64_t)j * kT + tid;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

// offs[digit * ntiles + tile] = first output position of the tile's
// elements with that digit.
__global__ __launch_bounds__(kT) void rs_scatter_kernel(const uint32_t* __restrict__ kin,
                                                        const int32_t* __restrict__ vin,
                                                        uint32_t* __restrict__ kout,
                                                        int32_t* __restrict__ vout, int64_t n,
                                                        int shift, const uint32_t* __restrict__ offs,
                                                        int64_t ntiles) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t boff[256];
    __shared__ uint32_t wc[kT / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    run[tid] = 0;
    boff[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
    const uint64_t below_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int j = 0; j < kI; ++j) {
#pragma unroll
        for (int w = 0; w < kT / 64; ++w) wc[w][tid] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)j * kT + tid;
        const bool valid = i < n;
        const uint32_t k = valid ? kin[i] : 0u;
        const uint32_t dg = (k >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(m & below_mask);
        if (valid && below == 0) wc[wv][dg] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = boff[dg] + run[dg] + below;
            for (int w = 0; w < wv; ++w) pos += wc[w][dg];
            kout[pos] = k;
            vout[pos] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kT / 64; ++w) add += wc[w][tid];
        run[tid] += add;
    }
}

// ------------------------------------------------------------ plan kernels

__global__ void iota_kernel(int32_t* __restrict__ v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = (int32_t)i;
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ v, int64_t n, uint32_t x) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = x;
}

// out[p] = key[order[p]] (order == nullptr: out[p] = key[p])
__global__ void gather_key_kernel(uint32_t* __restrict__ out, const int32_t* __restrict__ key,
                                  const int32_t* __restrict__ order, int64_t n) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        out[p] = (uint32_t)key[order ? order[p] : p];
}

__global__ void copy_i32_kernel(int32_t* __restrict__ out, const int32_t* __restrict__ in, int64_t n) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        out[p] = in[p];
}

// ends[row] = one past the last position of the row in the row-sorted keys
__global__ void row_end_kernel(const uint32_t* __restrict__ K, int64_t n, uint32_t* __restrict__ ends) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        if (p == n - 1 || K[p + 1] != K[p]) ends[K[p]] = (uint32_t)(p + 1);
}

__device__ __forceinline__ int64_t piece_of_rank_dev(int64_t deg, int64_t k, int64_t rank) {
    const int64_t q = deg / k, rem = deg % k, big = rem * (q + 1);
    return rank < big ? rank / (q + 1) : rem + (rank - big) / q;
}

// Segment id of every nonzero from the row-sorted (K, E) of its mode: the
// nonzero's rank within its row (input order) gives its piece.
__global__ void seg_kernel(const uint32_t* __restrict__ K, const int32_t* __restrict__ E, int64_t n,
                           const uint32_t* __restrict__ ends, const int64_t* __restrict__ pbase,
                           const int32_t* __restrict__ pseg, int32_t* __restrict__ seg) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = K[p];
        const int64_t start = i ? ends[i - 1] : 0;
        const int64_t deg = (int64_t)ends[i] - start;
        const int64_t k = pbase[i + 1] - pbase[i];
        const int64_t j = k > 1 ? piece_of_rank_dev(deg, k, p - start) : 0;
        seg[E[p]] = pseg[pbase[i] + j];
    }
}

__global__ void scatter_pos_kernel(const int32_t* __restrict__ order, int64_t n, int32_t* __restrict__ pos) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        pos[order[p]] = (int32_t)p;
}

// nxt[b_d(e)] = b_{d+1}(e)
__global__ void nxt_kernel(const int32_t* __restrict__ bd, const int32_t* __restrict__ bn, int64_t n,
                           int32_t* __restrict__ nxt) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        nxt[bd[e]] = bn[e];
}

struct PackArgs {
    const int32_t* idx;  // [N][nnz]
    const float* val;
    int64_t nnz;
    int nmodes, words;
    int off[kMaxModes], bits[kMaxModes];
};

// out[p] = record of nonzero order[p]: index w at bits [off_w, off_w + bits_w)
// of the index words, the value in the last word.
__global__ void pack_kernel(const PackArgs a, const int32_t* __restrict__ order, uint32_t* __restrict__ out) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < a.nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = order[p];
        uint32_t w[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = 0;
        for (int m = 0; m < a.nmodes; ++m) {
            const uint64_t v = (uint32_t)a.idx[(int64_t)m * a.nnz + e];
            const int o = a.off[m], wi = o >> 5, sh = o & 31;
            w[wi] |= (uint32_t)(v << sh);
            if (sh + a.bits[m] > 32) w[wi + 1] |= (uint32_t)(v >> (32 - sh));
        }
        w[a.words - 1] = __float_as_uint(a.val[e]);
        if (a.words % 4 == 0) {
            uint4* dst = reinterpret_cast<uint4*>(out + p * a.words);
            for (int k = 0; k < a.words / 4; ++k)
                dst[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
        } else {
            for (int k = 0; k < a.words; ++k) out[p * a.words + k] = w[k];
        }
    }
}

struct Dims8 {
    int64_t d[kMaxModes];
};

// Smallest mode-major position w * nnz + e whose index is out of range.
__global__ void validate_kernel(const int32_t* __restrict__ idx, int64_t nnz, int nmodes, const Dims8 dims,
                                unsigned long long* __restrict__ bad) {
    const int64_t total = nnz * nmodes;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = idx[t];
        if (c < 0 || c >= dims.d[t / nnz]) atomicMin(bad, (unsigned long long)t);
    }
}

// Runs of equal coordinates in the coordinate-sorted order, in chunks of
// kRunChunk positions, one thread each: the values before the chunk's first
// run head (the continuation of a run from earlier chunks), the sum of the
// squared sums of runs that start and end inside the chunk, and the values
// from the chunk's last head on (a run that may continue).  Each run is
// summed in position order, which is input order (the sorts are stable).
constexpr int kRunChunk = 256;

__global__ void run_chunk_kernel(const int32_t* __restrict__ order, const int32_t* __restrict__ idx,
                                 const float* __restrict__ val, int nmodes, int64_t n,
                                 double* __restrict__ head_part, double* __restrict__ inner,
                                 double* __restrict__ tail, int32_t* __restrict__ has_head) {
    const int64_t nch = (n + kRunChunk - 1) / kRunChunk;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nch;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p0 = c * kRunChunk, p1 = min(n, p0 + kRunChunk);
        double cur = 0.0, head = 0.0, in = 0.0;
        bool seen = false;
        int64_t prev = p0 > 0 ? order[p0 - 1] : -1;
        for (int64_t p = p0; p < p1; ++p) {
            const int64_t e = order[p];
            bool start = prev < 0;
            for (int m = 0; m < nmodes && !start; ++m)
                start = idx[(int64_t)m * n + e] != idx[(int64_t)m * n + prev];
            if (start) {
                if (seen)
                    in += cur * cur;
                else
                    head = cur;
                cur = 0.0;
                seen = true;
            }
            cur += (double)val[e];
            prev = e;
        }
        head_part[c] = seen ? head : cur;
        inner[c] = in;
        tail[c] = seen ? cur : 0.0;
        has_head[c] = seen ? 1 : 0;
    }
}

// ------------------------------------------------------------ host helpers

struct Fail {
    DevicePlanError code;
    std::string msg;
};

struct Temps {
    std::vector<void*> ptrs;
    hipStream_t stream = nullptr;
    ~Temps() {
        // kernels of a failed call may still read these
        (void)hipStreamSynchronize(stream);
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    T* alloc(int64_t count) {
        void* p = nullptr;
        if (hipMalloc(&p, (size_t)std::max<int64_t>(1, count) * sizeof(T)) != hipSuccess)
            throw Fail{DevicePlanError::kOom, "device allocation failed in the device planner"};
        ptrs.push_back(p);
        return static_cast<T*>(p);
    }
};

struct JoinAll {
    std::vector<std::thread> th;
    void join() {
        for (auto& t : th)
            if (t.joinable()) t.join();
    }
    ~JoinAll() { join(); }
};

void check(hipError_t e, const char* what) {
    if (e != hipSuccess)
        throw Fail{DevicePlanError::kHip, std::string(what) + ": " + hipGetErrorString(e)};
}

template <typename K, typename... Args>
void launch(K kernel, unsigned grid, unsigned block, hipStream_t s, Args... args) {
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, args...);
    check(hipGetLastError(), "kernel launch");
}

ScanScratch make_scan_scratch(Temps& tmp, int64_t cap) {
    ScanScratch sc;
    int64_t n = cap;
    do {
        n = (n + kTile - 1) / kTile;
        sc.level.push_back(tmp.alloc<uint32_t>(n));
        sc.size.push_back(n);
    } while (n > 1);
    return sc;
}

template <bool MAX>
void scan(uint32_t* d, int64_t n, const ScanScratch& sc, size_t level, hipStream_t s) {
    if (n <= 0) return;
    const int64_t nb = (n + kTile - 1) / kTile;
    if (level >= sc.level.size() || nb > sc.size[level]) throw Fail{DevicePlanError::kHip, "scan scratch too small"};
    uint32_t* sums = sc.level[level];
    launch(scan_chunk_kernel<MAX>, (unsigned)nb, kT, s, d, n, sums);
    if (nb > 1) {
        scan<MAX>(sums, nb, sc, level + 1, s);
        launch(scan_add_kernel<MAX>, grid_for(n), kT, s, d, n, (const uint32_t*)sums);
    }
}

struct SortBufs {
    uint32_t* k[2];
    int32_t* v[2];
    uint32_t* hist;
    ScanScratch sc;
};

// Stable sort of (k[0], v[0]) by the low `bits` bits of the keys; the result
// ends in (k[0], v[0]) (the buffers are swapped as needed).
void radix_sort(SortBufs& b, int64_t n, int bits, hipStream_t s) {
    if (n <= 0) return;
    const int64_t nt = (n + kTile - 1) / kTile;
    for (int shift = 0; shift < bits; shift += 8) {
        launch(rs_hist_kernel, (unsigned)nt, kT, s, (const uint32_t*)b.k[0], n, shift, b.hist, nt);
        scan<false>(b.hist, 256 * nt, b.sc, 0, s);
        launch(rs_scatter_kernel, (unsigned)nt, kT, s, (const uint32_t*)b.k[0], (const int32_t*)b.v[0],
               b.k[1], b.v[1], n, shift, (const uint32_t*)b.hist, nt);
        std::swap(b.k[0], b.k[1]);
        std::swap(b.v[0], b.v[1]);
    }
}

}  // namespace

DevicePlanError build_plan_device(int N, const int64_t* dims, int64_t nnz, const int32_t* idx,
                                  const float* val, const PlanOptions& opt,
                                  const RecordLayout& lay, int copies, hipStream_t s,
                                  const DeviceAlloc& persist, DevicePlan* out, std::string* msg) {
    try {
        bool range = false;
        std::string shape = validate_shape(N, dims, nnz, idx, &range);
        if (!shape.empty()) {
            *msg = shape;
            return range ? DevicePlanError::kRange : DevicePlanError::kInvalid;
        }
        const int32_t kappa = opt.kappa > 0 ? opt.kappa : default_kappa(nnz);
        int64_t cap;
        if (opt.split_cap < 0)
            cap = 0;
        else if (opt.split_cap == 0)
            cap = std::max<int64_t>(1, (nnz + kappa - 1) / kappa);
        else
            cap = opt.split_cap;
        out->kappa = kappa;
        out->cap = cap;
        auto palloc = [&](size_t bytes) {
            void* p = persist(std::max<size_t>(bytes, 4));
            if (!p) throw Fail{DevicePlanError::kOom, "device allocation failed for the streams"};
            return p;
        };

        Temps tmp;
        tmp.stream = s;
        int64_t maxI = 1;
        for (int w = 0; w < N; ++w) maxI = std::max<int64_t>(maxI, dims[w]);
        int32_t* didx = tmp.alloc<int32_t>(N * nnz);
        float* dval = tmp.alloc<float>(nnz);
        if (nnz > 0) {
            check(hipMemcpyAsync(didx, idx, sizeof(int32_t) * N * nnz, hipMemcpyHostToDevice, s), "upload indices");
            check(hipMemcpyAsync(dval, val, sizeof(float) * nnz, hipMemcpyHostToDevice, s), "upload values");
        }

        // indices in range (the first offender in mode-major order, as the
        // host validator reports it)
        if (nnz > 0) {
            unsigned long long* bad = tmp.alloc<unsigned long long>(1);
            const unsigned long long none = ~0ull;
            check(hipMemcpyAsync(bad, &none, sizeof(none), hipMemcpyHostToDevice, s), "upload");
            Dims8 d8{};
            for (int w = 0; w < N; ++w) d8.d[w] = dims[w];
            launch(validate_kernel, grid_for(N * nnz, kT, 16384), kT, s, (const int32_t*)didx, nnz, N, d8, bad);
            unsigned long long hb = none;
            check(hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, s), "download");
            check(hipStreamSynchronize(s), "validate");
            if (hb != none) {
                const int w = (int)(hb / (unsigned long long)nnz);
                const int64_t e = (int64_t)(hb % (unsigned long long)nnz);
                *msg = "index " + std::to_string(idx[(int64_t)w * nnz + e]) + " of nonzero " + std::to_string(e) +
                       " is outside mode " + std::to_string(w) + " (size " + std::to_string(dims[w]) + ")";
                return DevicePlanError::kRange;
            }
        }

        SortBufs sb;
        sb.k[0] = tmp.alloc<uint32_t>(nnz);
        sb.k[1] = tmp.alloc<uint32_t>(nnz);
        sb.v[0] = tmp.alloc<int32_t>(nnz);
        sb.v[1] = tmp.alloc<int32_t>(nnz);
        const int64_t ntiles = (nnz + kTile - 1) / kTile;
        sb.hist = tmp.alloc<uint32_t>(256 * std::max<int64_t>(1, ntiles));
        sb.sc = make_scan_scratch(tmp, std::max<int64_t>(256 * std::max<int64_t>(1, ntiles), maxI));
        const unsigned g = grid_for(nnz, kT, 16384);

        // ---- degrees and within-row ranks: stable sort of the nonzeros by
        // row, one mode at a time; Alg. 1 for the mode on a host thread
        // while the device sorts the next mode
        std::vector<uint32_t*> rowK(N);
        std::vector<int32_t*> rowE(N);
        std::vector<uint32_t*> ends(N);
        std::vector<RowPieces> pieces(N);
        std::vector<std::vector<int64_t>> deg(N);
        JoinAll lpt;
        for (int w = 0; w < N; ++w) {
            rowK[w] = tmp.alloc<uint32_t>(nnz);
            rowE[w] = tmp.alloc<int32_t>(nnz);
            ends[w] = tmp.alloc<uint32_t>(dims[w]);
            if (nnz > 0) {
                launch(gather_key_kernel, g, kT, s, sb.k[0], (const int32_t*)(didx + w * nnz), (const int32_t*)nullptr, nnz);
                launch(iota_kernel, g, kT, s, sb.v[0], nnz);
                radix_sort(sb, nnz, bit_len(dims[w] - 1), s);
                check(hipMemcpyAsync(rowK[w], sb.k[0], sizeof(uint32_t) * nnz, hipMemcpyDeviceToDevice, s), "copy");
                check(hipMemcpyAsync(rowE[w], sb.v[0], sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s), "copy");
            }
            launch(fill_u32_kernel, grid_for(dims[w]), kT, s, ends[w], dims[w], 0u);
            if (nnz > 0) launch(row_end_kernel, g, kT, s, (const uint32_t*)rowK[w], nnz, ends[w]);
            scan<true>(ends[w], dims[w], sb.sc, 0, s);
            std::vector<uint32_t> he(dims[w]);
            check(hipMemcpyAsync(he.data(), ends[w], sizeof(uint32_t) * dims[w], hipMemcpyDeviceToHost, s), "download");
            check(hipStreamSynchronize(s), "row degrees");
            deg[w].resize(dims[w]);
            for (int64_t i = 0; i < dims[w]; ++i) deg[w][i] = (int64_t)he[i] - (i ? (int64_t)he[i - 1] : 0);
            lpt.th.emplace_back([&, w] { partition_rows(dims[w], deg[w].data(), kappa, cap, out->mode[w], pieces[w]); });
        }
        lpt.join();

        // ---- segment id of every nonzero in every mode
        std::vector<int32_t*> seg(N);
        for (int w = 0; w < N; ++w) {
            seg[w] = tmp.alloc<int32_t>(nnz);
            int64_t* pb = tmp.alloc<int64_t>((int64_t)pieces[w].piece_base.size());
            int32_t* ps = tmp.alloc<int32_t>((int64_t)pieces[w].piece_seg.size());
            check(hipMemcpyAsync(pb, pieces[w].piece_base.data(), sizeof(int64_t) * pieces[w].piece_base.size(),
                                 hipMemcpyHostToDevice, s), "upload");
            check(hipMemcpyAsync(ps, pieces[w].piece_seg.data(), sizeof(int32_t) * pieces[w].piece_seg.size(),
                                 hipMemcpyHostToDevice, s), "upload");
            if (nnz > 0)
                launch(seg_kernel, g, kT, s, (const uint32_t*)rowK[w], (const int32_t*)rowE[w], nnz,
                       (const uint32_t*)ends[w], (const int64_t*)pb, (const int32_t*)ps, seg[w]);
            // the host tables are read by the copies above before they go
            check(hipStreamSynchronize(s), "segments");
        }

        // ---- streams: sorts by seg_1, ..., seg_{N-1}, seg_0 -> mode 0; then
        // one more sort by seg_d for each mode d
        PackArgs pa{};
        pa.idx = didx;
        pa.val = dval;
        pa.nnz = nnz;
        pa.nmodes = N;
        pa.words = lay.words;
        for (int w = 0; w < N; ++w) {
            pa.off[w] = lay.off[w];
            pa.bits[w] = lay.bits[w];
        }
        std::vector<int32_t*> remap(N);
        for (int w = 0; w < N; ++w) remap[w] = tmp.alloc<int32_t>(nnz);
        if (nnz > 0) launch(iota_kernel, g, kT, s, sb.v[0], nnz);
        auto sort_by = [&](int w) {
            if (nnz == 0) return;
            launch(gather_key_kernel, g, kT, s, sb.k[0], (const int32_t*)seg[w], (const int32_t*)sb.v[0], nnz);
            radix_sort(sb, nnz, bit_len(pieces[w].nseg - 1), s);
        };
        for (int k = 1; k <= N; ++k) sort_by(k % N);
        for (int d = 0; d < N; ++d) {
            if (d > 0) sort_by(d);
            if (nnz > 0) launch(scatter_pos_kernel, g, kT, s, (const int32_t*)sb.v[0], nnz, remap[d]);
            if (d == 0) {
                out->order0.resize(nnz);
                if (nnz > 0)
                    check(hipMemcpyAsync(out->order0.data(), sb.v[0], sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s),
                          "download order");
            }
            if (copies || d == 0) {
                uint32_t* r = static_cast<uint32_t*>(palloc(sizeof(uint32_t) * lay.words * nnz));
                if (copies)
                    out->rec_mode[d] = r;
                else
                    out->rec0 = r;
                if (nnz > 0) launch(pack_kernel, g, kT, s, pa, (const int32_t*)sb.v[0], r);
            }
        }
        if (!copies)
            for (int d = 0; d < N; ++d) {
                out->nxt[d] = static_cast<int32_t*>(palloc(sizeof(int32_t) * nnz));
                if (nnz > 0)
                    launch(nxt_kernel, g, kT, s, (const int32_t*)remap[d], (const int32_t*)remap[(d + 1) % N], nnz,
                           out->nxt[d]);
            }

        // ---- ||X||^2 of the coalesced tensor: stable sorts by the index of
        // modes N-1, ..., 0 put equal coordinates together in input order
        out->norm_sq = 0.0;
        if (nnz > 0) {
            launch(iota_kernel, g, kT, s, sb.v[0], nnz);
            for (int w = N - 1; w >= 0; --w) {
                launch(gather_key_kernel, g, kT, s, sb.k[0], (const int32_t*)(didx + w * nnz), (const int32_t*)sb.v[0], nnz);
                radix_sort(sb, nnz, bit_len(dims[w] - 1), s);
            }
            const int64_t nch = (nnz + kRunChunk - 1) / kRunChunk;
            double* hp = tmp.alloc<double>(nch);
            double* in = tmp.alloc<double>(nch);
            double* tl = tmp.alloc<double>(nch);
            int32_t* hh = tmp.alloc<int32_t>(nch);
            launch(run_chunk_kernel, grid_for(nch, kT, 16384), kT, s, (const int32_t*)sb.v[0],
                   (const int32_t*)didx, (const float*)dval, N, nnz, hp, in, tl, hh);
            std::vector<double> h_hp(nch), h_in(nch), h_tl(nch);
            std::vector<int32_t> h_hh(nch);
            check(hipMemcpyAsync(h_hp.data(), hp, sizeof(double) * nch, hipMemcpyDeviceToHost, s), "download");
            check(hipMemcpyAsync(h_in.data(), in, sizeof(double) * nch, hipMemcpyDeviceToHost, s), "download");
            check(hipMemcpyAsync(h_tl.data(), tl, sizeof(double) * nch, hipMemcpyDeviceToHost, s), "download");
            check(hipMemcpyAsync(h_hh.data(), hh, sizeof(int32_t) * nch, hipMemcpyDeviceToHost, s), "download");
            check(hipStreamSynchronize(s), "norm chunks");
            // runs crossing chunk boundaries, joined in chunk order
            double carry = 0.0, total = 0.0;
            for (int64_t c = 0; c < nch; ++c) {
                carry += h_hp[c];
                if (h_hh[c]) {
                    total += carry * carry;
                    total += h_in[c];
                    carry = h_tl[c];
                }
            }
            out->norm_sq = total + carry * carry;
        }
        check(hipStreamSynchronize(s), "device planner");
        return DevicePlanError::kNone;
    } catch (const Fail& f) {
        *msg = f.msg;
        return f.code;
    } catch (const std::bad_alloc&) {
        *msg = "host allocation failed in the device planner";
        return DevicePlanError::kOom;
    }
}

}  // namespace spt
