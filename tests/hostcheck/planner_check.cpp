// Host-only exercise of the planner and the C ABI for the sanitizer build:
// spt_plan_coo over skewed tensors of 2 to 8 modes with several partition
// counts and split caps (checking the invariants of the plan), rejected
// inputs, and spt_tensor_load_coo up to its first device allocation (there
// is no device here), which must fail cleanly.  Exit status 0 = all held.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "spmttkrp.h"

namespace {

uint64_t g_state = 0x9E3779B97F4A7C15ull;
uint64_t next_u64() {  // xorshift64*
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return g_state * 0x2545F4914F6CDD1Dull;
}

int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

// skewed indices: the square of a uniform draw favours low ids
std::vector<int32_t> make_idx(const std::vector<int64_t>& dims, int64_t nnz, bool skew) {
    std::vector<int32_t> idx(dims.size() * nnz);
    for (size_t w = 0; w < dims.size(); ++w)
        for (int64_t e = 0; e < nnz; ++e) {
            double u = (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0);
            if (skew) u = u * u * u;
            int64_t c = (int64_t)(u * (double)dims[w]);
            if (c >= dims[w]) c = dims[w] - 1;
            idx[w * nnz + e] = (int32_t)c;
        }
    return idx;
}

void check_plan(const std::vector<int64_t>& dims, int64_t nnz, int32_t kappa, int64_t cap, bool skew) {
    const int N = (int)dims.size();
    std::vector<int32_t> idx = make_idx(dims, nnz, skew);
    spt_opts o{};
    o.kappa = kappa;
    o.split_cap = cap;
    int32_t k = 0;
    CHECK(spt_plan_coo(N, dims.data(), nnz, idx.data(), &o, nullptr, nullptr, nullptr, &k) == SPT_OK);
    CHECK(k >= 1);
    std::vector<int32_t> part((size_t)N * nnz);
    std::vector<int64_t> remap((size_t)N * nnz), ptr((size_t)N * (k + 1));
    CHECK(spt_plan_coo(N, dims.data(), nnz, idx.data(), &o, part.data(), remap.data(), ptr.data(), &k) == SPT_OK);
    for (int d = 0; d < N; ++d) {
        const int64_t* p = &ptr[(size_t)d * (k + 1)];
        CHECK(p[0] == 0 && p[k] == nnz);
        for (int z = 0; z < k; ++z) CHECK(p[z] <= p[z + 1]);
        std::vector<char> seen(nnz, 0);
        for (int64_t e = 0; e < nnz; ++e) {
            const int64_t b = remap[(size_t)d * nnz + e];
            const int32_t z = part[(size_t)d * nnz + e];
            CHECK(b >= 0 && b < nnz && !seen[b]);
            if (b >= 0 && b < nnz) seen[b] = 1;
            CHECK(z >= 0 && z < k && p[z] <= b && b < p[z + 1]);
        }
    }
}

}  // namespace

int main() {
    check_plan({40, 9}, 3000, 7, 0, true);
    check_plan({30, 20, 10}, 5000, 0, 0, true);
    check_plan({30, 20, 10}, 5000, 13, -1, true);
    check_plan({30, 20, 10}, 5000, 13, 50, false);
    check_plan({12, 9, 7, 5}, 4000, 31, 0, true);
    check_plan({8, 7, 6, 5, 4}, 4000, 97, 0, true);
    check_plan({5, 4, 3, 3, 2, 2}, 3000, 11, 0, true);
    check_plan({9, 8, 7, 6, 5, 4, 3, 2}, 6000, 5, 0, true);
    check_plan({1, 300, 1, 7}, 2000, 16, 0, false);
    check_plan({50, 40, 30}, 37, 200, 0, false);
    check_plan({5, 4, 3}, 0, 0, 0, false);
    check_plan({3000, 2500, 60000}, 200000, 0, 0, true);

    // rejected inputs
    std::vector<int64_t> dims = {5, 4, 3};
    std::vector<int32_t> idx = {0, 5, 0, 1, 0, 1};
    int32_t k = 0;
    CHECK(spt_plan_coo(3, dims.data(), 2, idx.data(), nullptr, nullptr, nullptr, nullptr, &k) ==
          SPT_ERR_OUT_OF_RANGE);
    CHECK(spt_plan_coo(1, dims.data(), 2, idx.data(), nullptr, nullptr, nullptr, nullptr, &k) ==
          SPT_ERR_INVALID_ARG);
    CHECK(spt_plan_coo(9, dims.data(), 2, idx.data(), nullptr, nullptr, nullptr, nullptr, &k) ==
          SPT_ERR_INVALID_ARG);
    CHECK(spt_plan_coo(3, nullptr, 2, idx.data(), nullptr, nullptr, nullptr, nullptr, &k) == SPT_ERR_INVALID_ARG);
    CHECK(spt_plan_coo(3, dims.data(), -1, idx.data(), nullptr, nullptr, nullptr, nullptr, &k) ==
          SPT_ERR_OUT_OF_RANGE);
    spt_opts bad{};
    bad.dr = 2;
    idx[1] = 1;
    CHECK(spt_plan_coo(3, dims.data(), 2, idx.data(), &bad, nullptr, nullptr, nullptr, &k) == SPT_ERR_INVALID_ARG);
    bad = spt_opts{};
    bad.kappa = -3;
    CHECK(spt_plan_coo(3, dims.data(), 2, idx.data(), &bad, nullptr, nullptr, nullptr, &k) == SPT_ERR_INVALID_ARG);
    CHECK(spt_status_str(SPT_ERR_STATE)[0] == 'S');

    // the whole host planner, then the first device allocation fails cleanly
    {
        std::vector<int64_t> d3 = {300, 200, 4000};
        const int64_t nnz = 60000;
        std::vector<int32_t> id3 = make_idx(d3, nnz, true);
        std::vector<float> val(nnz, 0.5f);
        spt_tensor_t t = nullptr;
        const spt_status st = spt_tensor_load_coo(3, d3.data(), nnz, id3.data(), val.data(), nullptr, nullptr, &t);
        CHECK(st != SPT_OK && t == nullptr);
        CHECK(spt_last_error()[0] != 0);
        CHECK(spt_tensor_free(nullptr) == SPT_OK);
    }
    if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
    else std::printf("planner checks passed\n");
    return failures ? 1 : 0;
}
