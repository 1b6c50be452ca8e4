// C ABI of the library (include/spmttkrp.h): handle lifecycle, uploads,
// kernel launches and the CP-ALS sweep.
#include "spmttkrp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "device_plan.hpp"
#include "plan.hpp"

using spt::Plan;
using spt::PlanOptions;
using spt::RecordLayout;

namespace {

thread_local std::string g_last_error;

spt_status fail(spt_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

spt_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? SPT_ERR_OOM : SPT_ERR_HIP;
}

#define HIPCHK(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

bool rank_compiled(int r) { return r == 8 || r == 16 || r == 32 || r == 64 || r == 128; }
bool als_rank(int r) { return r == 8 || r == 16 || r == 32 || r == 64; }
// factor rows and output rows move as 16-byte vectors
bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

struct spt_tensor_s {
    int N = 0;
    int64_t nnz = 0;
    int64_t dims[8] = {};
    int32_t kappa = 0;
    int copies = 0;
    int cur_mode = 0;
    RecordLayout lay;
    // device: record streams.  copies == 0: rec[cur] holds the stream of
    // cur_mode, rec[1-cur] is the remap target.  copies == 1: rec_mode[d].
    uint32_t* rec[2] = {nullptr, nullptr};
    int cur = 0;
    uint32_t* rec_mode[8] = {};
    int32_t* nxt[8] = {};
    int64_t* ptr[8] = {};
    int32_t* psplit_ptr[8] = {};
    int32_t* psplit_row[8] = {};
    int32_t* psplit_slot[8] = {};
    int32_t* split_row[8] = {};
    int32_t* split_ptr[8] = {};
    int32_t* empty_rows[8] = {};
    int dr = 0;                   // 0: staged remap pass after EC; 1: remap fused into EC
    int32_t* ddst[8] = {};        // staged remap tables of mode d -> d+1 (dr == 0)
    uint16_t* doff[8] = {};
    int32_t nsplit[8] = {}, nslots[8] = {}, nempty[8] = {};
    int64_t max_load[8] = {};
    std::vector<int32_t> order0;  // input nonzero at each mode-0 position
    double norm_sq = 0.0;
    double prep_seconds = 0.0;
    int64_t device_bytes = 0;
    std::vector<void*> allocs;
    // workspace
    int ws_rank = 0;
    float* M = nullptr;
    float* carry = nullptr;
    double* grams = nullptr;
    double* gpart = nullptr;
    double* ipart = nullptr;
    double* Vinv = nullptr;
    uint16_t* shadow[8] = {};  // BF16 copies of the factors (CP-ALS with SPT_BF16)
    uint32_t* res[2] = {nullptr, nullptr};  // residual stream + its remap target
    int res_cur = 0;                        // res[res_cur]: residuals in mode 0's order
    int res_rank = 0;                       // rank of the last forward pass (0: none)
    double* loss_part = nullptr;
    double* Gsum = nullptr;
    double* Isum = nullptr;
    double* fitd = nullptr;
    int32_t* status = nullptr;
    int32_t* status_host = nullptr;
    hipEvent_t status_event = nullptr;
    // CP-ALS: the remap pass of a mode on a side stream, beside that mode's
    // fixup and dense update (joined before the next mode's EC)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool join_pending = false;
    bool status_pending = false;
    std::vector<void*> ws_allocs;
    // kernel timing
    struct Timed {
        int mode;
        hipEvent_t ev[5];  // before EC, after EC, after staged remap, after fixup, after ALS step
        bool side;         // the remap ran on the side stream (ev[2] recorded there)
    };
    bool timing = false;
    std::vector<Timed> timed;
    std::vector<hipEvent_t> event_pool;
    size_t events_used = 0;
};

namespace {

template <typename T>
spt_status dalloc(spt_tensor_s* t, T** p, size_t count, std::vector<void*>* list) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    list->push_back(*p);
    t->device_bytes += (int64_t)(count * sizeof(T));
    return SPT_OK;
}

template <typename T>
spt_status upload(spt_tensor_s* t, T** p, const std::vector<T>& v, hipStream_t s) {
    spt_status st = dalloc(t, p, v.size(), &t->allocs);
    if (st != SPT_OK) return st;
    if (!v.empty()) HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return SPT_OK;
}

void release(spt_tensor_s* t) {
    for (hipEvent_t e : t->event_pool) (void)hipEventDestroy(e);
    t->event_pool.clear();
    for (void* p : t->allocs) (void)hipFree(p);
    for (void* p : t->ws_allocs) (void)hipFree(p);
    if (t->status_host) (void)hipHostFree(t->status_host);
    if (t->status_event) (void)hipEventDestroy(t->status_event);
    if (t->side) (void)hipStreamDestroy(t->side);
    if (t->ev_fork) (void)hipEventDestroy(t->ev_fork);
    if (t->ev_join) (void)hipEventDestroy(t->ev_join);
    t->side = nullptr;
    t->ev_fork = t->ev_join = nullptr;
    t->allocs.clear();
    t->ws_allocs.clear();
}

spt_status get_opts(const spt_opts* o, PlanOptions* po, int* copies, int* dr) {
    *copies = 0;
    *dr = 0;
    if (!o) return SPT_OK;
    if (o->reserved != 0) return fail(SPT_ERR_INVALID_ARG, "opts.reserved must be zero");
    if (o->dr != 0 && o->dr != 1) return fail(SPT_ERR_INVALID_ARG, "opts.dr must be 0 or 1");
    *dr = o->dr;
    if (o->layout < 0 || o->layout > 4) return fail(SPT_ERR_INVALID_ARG, "opts.layout must be 0..4");
    po->layout = o->layout;
    if (o->prep != 0 && o->prep != 1) return fail(SPT_ERR_INVALID_ARG, "opts.prep must be 0 or 1");
    po->prep = o->prep;
    if (o->kappa < 0) return fail(SPT_ERR_INVALID_ARG, "opts.kappa must be >= 0");
    if (o->copies != 0 && o->copies != 1) return fail(SPT_ERR_INVALID_ARG, "opts.copies must be 0 or 1");
    if (o->split_cap < -1) return fail(SPT_ERR_INVALID_ARG, "opts.split_cap must be >= -1");
    po->kappa = o->kappa;
    po->split_cap = o->split_cap;
    *copies = o->copies;
    return SPT_OK;
}

spt_status ensure_carry(spt_tensor_s* t, int rank) {
    if (t->ws_rank == rank) return SPT_OK;
    for (void* p : t->ws_allocs) (void)hipFree(p);
    t->ws_allocs.clear();
    t->ws_rank = 0;
    int64_t maxslots = 1, maxrows = 1;
    for (int d = 0; d < t->N; ++d) {
        maxslots = std::max<int64_t>(maxslots, t->nslots[d]);
        maxrows = std::max<int64_t>(maxrows, t->dims[d]);
    }
    spt_status st;
    if ((st = dalloc(t, &t->carry, (size_t)(maxslots * rank), &t->ws_allocs)) != SPT_OK) return st;
    if (als_rank(rank)) {
        const int64_t E = (int64_t)rank * rank;
        const int64_t nb = std::max<int64_t>(spt::solve_blocks(maxrows), spt::gram_blocks(maxrows));
        if ((st = dalloc(t, &t->M, (size_t)(maxrows * rank), &t->ws_allocs)) != SPT_OK) return st;
        if ((st = dalloc(t, &t->grams, (size_t)(t->N * E), &t->ws_allocs)) != SPT_OK) return st;
        if ((st = dalloc(t, &t->gpart, (size_t)(nb * E), &t->ws_allocs)) != SPT_OK) return st;
        if ((st = dalloc(t, &t->ipart, (size_t)(nb * rank), &t->ws_allocs)) != SPT_OK) return st;
        if ((st = dalloc(t, &t->Vinv, (size_t)E, &t->ws_allocs)) != SPT_OK) return st;
        if ((st = dalloc(t, &t->Gsum, (size_t)E, &t->ws_allocs)) != SPT_OK) return st;
        for (int w = 0; w < t->N; ++w)
            if ((st = dalloc(t, &t->shadow[w], (size_t)(t->dims[w] * rank), &t->ws_allocs)) != SPT_OK)
                return st;
        if ((st = dalloc(t, &t->Isum, (size_t)rank, &t->ws_allocs)) != SPT_OK) return st;
        if ((st = dalloc(t, &t->fitd, 1, &t->ws_allocs)) != SPT_OK) return st;
        if ((st = dalloc(t, &t->status, 1, &t->ws_allocs)) != SPT_OK) return st;
        HIPCHK(hipMemset(t->status, 0, sizeof(int32_t)));
    }
    t->ws_rank = rank;
    return SPT_OK;
}

// An event recorded on `s` now (timing only); nullptr if timing is off.
hipEvent_t mark(spt_tensor_s* t, hipStream_t s) {
    if (!t->timing) return nullptr;
    if (t->events_used == t->event_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        t->event_pool.push_back(e);
    }
    hipEvent_t e = t->event_pool[t->events_used++];
    if (hipEventRecord(e, s) != hipSuccess) return nullptr;
    return e;
}

spt_status ensure_side(spt_tensor_s* t) {
    if (t->side) return SPT_OK;
    HIPCHK(hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking));  // default priority
    HIPCHK(hipEventCreateWithFlags(&t->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&t->ev_join, hipEventDisableTiming));
    return SPT_OK;
}

// s waits for the side stream's last remap pass
spt_status join_side(spt_tensor_s* t, hipStream_t s) {
    if (!t->join_pending) return SPT_OK;
    HIPCHK(hipStreamWaitEvent(s, t->ev_join, 0));
    t->join_pending = false;
    return SPT_OK;
}

// EC (+ remap into rec_out when it is not null) and fixup for one mode over
// the stream rec_in, which must be in that mode's order.  With side_remap the
// remap pass runs on the tensor's side stream after EC, and the caller must
// call join_side() before anything on s reads rec_out.
// With noalloc_carry != nullptr the call allocates nothing: the split-row
// partial sums go to that buffer and no timing events are recorded.
spt_status launch_mode(spt_tensor_s* t, int mode, const uint32_t* rec_in, uint32_t* rec_out,
                       const void* const* factors, int fdtype, int rank, float* out, hipStream_t s,
                       bool side_remap = false, float* noalloc_carry = nullptr) {
    if (!spt::pick_ec_exists(t->N, rank, fdtype, t->lay.words, t->lay.kind))
        return fail(SPT_ERR_UNSUPPORTED, "no kernel compiled for this mode count / rank / record size");
    const bool noalloc = noalloc_carry != nullptr;
    spt_status st = join_side(t, s);
    if (st == SPT_OK && !noalloc) st = ensure_carry(t, rank);
    if (st != SPT_OK) return st;
    float* const carry = noalloc ? noalloc_carry : t->carry;
    auto mark_if = [&](hipStream_t on) -> hipEvent_t { return noalloc ? nullptr : mark(t, on); };
    const int N = t->N;
    // the staged pass remaps after EC when its tables exist, else EC stores
    // each record at its next position itself
    const bool staged = rec_out && t->ddst[mode];
    spt::EcArgs a{};
    a.rec_in = rec_in;
    a.rec_out = staged ? nullptr : rec_out;
    a.nxt = a.rec_out ? t->nxt[mode] : nullptr;
    a.ptr = t->ptr[mode];
    a.psplit_ptr = t->psplit_ptr[mode];
    a.psplit_row = t->psplit_row[mode];
    a.psplit_slot = t->psplit_slot[mode];
    a.out = out;
    a.carry = carry;
    for (int k = 0; k < N; ++k) {
        const int w = (mode + k) % N;
        a.fac[k] = factors[w];
        a.rot[k] = w;
        a.foff[k] = t->lay.off[k];
        a.fmask[k] = (uint32_t)((uint64_t(1) << t->lay.bits[k]) - 1);
    }
    spt_tensor_s::Timed tm{mode, {nullptr, nullptr, nullptr, nullptr, nullptr}, false};
    tm.ev[0] = mark_if(s);
    if (!spt::launch_ec(N, rank, fdtype, t->lay.words, t->lay.kind, t->kappa, a, s))
        return fail(SPT_ERR_HIP, "launch of the elementwise kernel failed");
    HIPCHK(hipGetLastError());
    tm.ev[1] = mark_if(s);
    if (staged && side_remap) {
        spt_status st2 = ensure_side(t);
        if (st2 != SPT_OK) return st2;
        HIPCHK(hipEventRecord(t->ev_fork, s));
        HIPCHK(hipStreamWaitEvent(t->side, t->ev_fork, 0));
        spt::launch_remap_staged(t->lay.words, t->nnz, rec_in, rec_out, t->ddst[mode], t->doff[mode], t->side);
        HIPCHK(hipGetLastError());
        tm.ev[2] = mark_if(t->side);
        tm.side = true;
        HIPCHK(hipEventRecord(t->ev_join, t->side));
        t->join_pending = true;
    } else if (staged) {
        spt::launch_remap_staged(t->lay.words, t->nnz, rec_in, rec_out, t->ddst[mode], t->doff[mode], s);
        HIPCHK(hipGetLastError());
        tm.ev[2] = mark_if(s);
    } else {
        tm.ev[2] = tm.ev[1];
    }
    spt::FixupArgs f{};
    f.out = out;
    f.carry = carry;
    f.split_row = t->split_row[mode];
    f.split_ptr = t->split_ptr[mode];
    f.empty_rows = t->empty_rows[mode];
    f.nsplit = t->nsplit[mode];
    f.nempty = t->nempty[mode];
    spt::launch_fixup(rank, f, s);
    HIPCHK(hipGetLastError());
    tm.ev[3] = mark_if(s);
    if (!noalloc && t->timing && tm.ev[0] && tm.ev[1] && tm.ev[2] && tm.ev[3]) t->timed.push_back(tm);
    return SPT_OK;
}

// mode d's stream and, when remapping, the target buffer of the tensor
spt_status run_mttkrp(spt_tensor_s* t, int mode, const void* const* factors, int fdtype, int rank,
                      float* out, bool fuse, hipStream_t s, bool side_remap = false) {
    if (t->copies)
        return launch_mode(t, mode, t->rec_mode[mode], nullptr, factors, fdtype, rank, out, s);
    spt_status st = launch_mode(t, mode, t->rec[t->cur], fuse ? t->rec[1 - t->cur] : nullptr,
                                factors, fdtype, rank, out, s, side_remap);
    if (st != SPT_OK) return st;
    if (fuse) {
        t->cur = 1 - t->cur;
        t->cur_mode = (mode + 1) % t->N;
    }
    return SPT_OK;
}

// Forward pass over `rec_in` (in any mode's order): residual records into
// `rec_res`, loss partials into t->loss_part.
spt_status launch_forward_pass(spt_tensor_s* t, const uint32_t* rec_in, uint32_t* rec_res,
                               const void* const* factors, int rank, hipStream_t s) {
    spt::ForwardArgs f{};
    f.rec_in = rec_in;
    f.rec_res = rec_res;
    for (int w = 0; w < t->N; ++w) {
        f.fac[w] = (const float*)factors[w];
        f.foff[w] = t->lay.off[w];
        f.fmask[w] = (uint32_t)((uint64_t(1) << t->lay.bits[w]) - 1);
    }
    f.loss_part = t->loss_part;
    f.nnz = t->nnz;
    if (!spt::launch_forward(t->N, rank, t->lay.words, t->lay.kind, f, s))
        return fail(SPT_ERR_UNSUPPORTED, "no forward kernel for this mode count / rank / layout");
    HIPCHK(hipGetLastError());
    return SPT_OK;
}

spt_status do_remap(spt_tensor_s* t, int mode, hipStream_t s) {
    spt_status st = join_side(t, s);
    if (st != SPT_OK) return st;
    if (t->copies) {
        t->cur_mode = mode;
        return SPT_OK;
    }
    const int N = t->N;
    const int hops = (mode - t->cur_mode + N) % N;
    if (hops == 0) return SPT_OK;
    if (hops == 1 && t->ddst[t->cur_mode]) {
        // one hop: the chunk-ordered remap pass
        spt::launch_remap_staged(t->lay.words, t->nnz, t->rec[t->cur], t->rec[1 - t->cur], t->ddst[t->cur_mode],
                                 t->doff[t->cur_mode], s);
        HIPCHK(hipGetLastError());
        t->cur = 1 - t->cur;
        t->cur_mode = mode;
        return SPT_OK;
    }
    const int32_t* chain[8];
    for (int h = 0; h < hops; ++h) chain[h] = t->nxt[(t->cur_mode + h) % N];
    spt::launch_remap(t->lay.words, t->nnz, t->rec[t->cur], t->rec[1 - t->cur], chain, hops, s);
    HIPCHK(hipGetLastError());
    t->cur = 1 - t->cur;
    t->cur_mode = mode;
    return SPT_OK;
}

}  // namespace

extern "C" {

const char* spt_status_str(spt_status s) {
    switch (s) {
        case SPT_OK: return "SPT_OK";
        case SPT_ERR_INVALID_ARG: return "SPT_ERR_INVALID_ARG";
        case SPT_ERR_OUT_OF_RANGE: return "SPT_ERR_OUT_OF_RANGE";
        case SPT_ERR_OOM: return "SPT_ERR_OOM";
        case SPT_ERR_HIP: return "SPT_ERR_HIP";
        case SPT_ERR_STATE: return "SPT_ERR_STATE";
        case SPT_ERR_NOT_SPD: return "SPT_ERR_NOT_SPD";
        case SPT_ERR_UNSUPPORTED: return "SPT_ERR_UNSUPPORTED";
    }
    return "SPT_UNKNOWN";
}

const char* spt_last_error(void) { return g_last_error.c_str(); }

spt_status spt_plan_coo(int32_t nmodes, const int64_t* dims, int64_t nnz, const int32_t* indices,
                        const spt_opts* opts, int32_t* part, int64_t* remap, int64_t* ptr,
                        int32_t* kappa_out) {
    g_last_error.clear();
    PlanOptions po;
    int copies = 0, dr = 0;
    spt_status st = get_opts(opts, &po, &copies, &dr);
    if (st != SPT_OK) return st;
    bool range = false;
    std::string msg = spt::validate(nmodes, dims, nnz, indices, &range);
    if (!msg.empty()) return fail(range ? SPT_ERR_OUT_OF_RANGE : SPT_ERR_INVALID_ARG, msg);
    po.remap_ids = remap != nullptr;
    po.norm = false;
    if (!part && !remap && !ptr) {
        if (kappa_out) *kappa_out = po.kappa > 0 ? po.kappa : spt::default_kappa(nnz);
        return SPT_OK;
    }
    try {
        Plan plan;
        spt::build_plan(nmodes, dims, nnz, indices, nullptr, po, &plan);
        for (int d = 0; d < nmodes; ++d) {
            const auto& mp = plan.mode[d];
            if (part) std::memcpy(part + (int64_t)d * nnz, mp.part.data(), sizeof(int32_t) * nnz);
            if (remap)
                for (int64_t e = 0; e < nnz; ++e) remap[(int64_t)d * nnz + e] = mp.remap[e];
            if (ptr)
                std::memcpy(ptr + (int64_t)d * (plan.kappa + 1), mp.ptr.data(),
                            sizeof(int64_t) * (plan.kappa + 1));
        }
        if (kappa_out) *kappa_out = plan.kappa;
    } catch (const std::bad_alloc&) {
        return fail(SPT_ERR_OOM, "host allocation failed in the planner");
    }
    return SPT_OK;
}

namespace {

// Staged remap tables of every mode from its next positions (both planners;
// the tables depend only on nxt_d, so they are identical either way).
spt_status build_stage_tables(spt_tensor_s* t, hipStream_t s) {
    if (t->copies || t->dr != 0) return SPT_OK;
    // the sorted runs before the merge into whole chunks (freed on return)
    std::vector<void*> temps;
    int32_t* tmp_dst = nullptr;
    uint16_t* tmp_off = nullptr;
    spt_status st = SPT_OK;
    const int64_t bytes_before = t->device_bytes;
    st = dalloc(t, &tmp_dst, (size_t)t->nnz, &temps);
    if (st == SPT_OK) st = dalloc(t, &tmp_off, (size_t)t->nnz, &temps);
    const int64_t temp_bytes = t->device_bytes - bytes_before;
    auto free_temps = [&]() {
        for (void* p : temps) (void)hipFree(p);
        t->device_bytes -= temp_bytes;
    };
    for (int d = 0; d < t->N && st == SPT_OK; ++d) {
        st = dalloc(t, &t->ddst[d], (size_t)t->nnz, &t->allocs);
        if (st == SPT_OK) st = dalloc(t, &t->doff[d], (size_t)t->nnz, &t->allocs);
        if (st != SPT_OK) break;
        spt::launch_stage_tables(t->lay.words, t->nxt[d], t->nnz, t->ddst[d], t->doff[d], tmp_dst, tmp_off, s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) st = hip_fail(e, "launch of the remap table kernels");
    }
    if (hipStreamSynchronize(s) != hipSuccess && st == SPT_OK)
        st = fail(SPT_ERR_HIP, "hipStreamSynchronize after the remap tables");
    free_temps();
    return st;
}

// The load with the device planner: streams and next positions are built in
// device memory the handle owns; the per-mode tables come back to the host
// and are uploaded as in the host path.
spt_status load_device(int32_t nmodes, const int64_t* dims, int64_t nnz, const int32_t* indices,
                       const float* values, const PlanOptions& po, int copies, hipStream_t s,
                       spt_tensor_s** out) {
    spt_tensor_s* t = nullptr;
    spt_status st = SPT_OK;
    try {
        t = new spt_tensor_s();
        t->N = nmodes;
        t->nnz = nnz;
        for (int w = 0; w < nmodes; ++w) t->dims[w] = dims[w];
        t->copies = copies;
        if (!spt::choose_layout(nmodes, dims, po.layout, &t->lay)) {
            delete t;
            return fail(SPT_ERR_UNSUPPORTED, "the record layout asked for in opts.layout has no kernel for "
                                             "this mode count and these mode sizes");
        }
        spt::DevicePlan dp;
        std::string msg;
        auto persist = [&](size_t bytes) -> void* {
            uint8_t* p = nullptr;
            return dalloc(t, &p, bytes, &t->allocs) == SPT_OK ? (void*)p : nullptr;
        };
        const spt::DevicePlanError e =
            spt::build_plan_device(nmodes, dims, nnz, indices, values, po, t->lay, copies, s, persist, &dp, &msg);
        if (e != spt::DevicePlanError::kNone) {
            release(t);
            delete t;
            const spt_status code = e == spt::DevicePlanError::kRange  ? SPT_ERR_OUT_OF_RANGE
                                    : e == spt::DevicePlanError::kOom  ? SPT_ERR_OOM
                                    : e == spt::DevicePlanError::kHip  ? SPT_ERR_HIP
                                                                       : SPT_ERR_INVALID_ARG;
            return fail(code, msg);
        }
        t->kappa = dp.kappa;
        t->norm_sq = dp.norm_sq;
        for (int d = 0; d < nmodes && st == SPT_OK; ++d) {
            const auto& mp = dp.mode[d];
            t->nsplit[d] = (int32_t)mp.split_row.size();
            t->nslots[d] = (int32_t)mp.slot_part.size();
            t->nempty[d] = (int32_t)mp.empty_rows.size();
            t->max_load[d] = mp.max_load;
            if ((st = upload(t, &t->ptr[d], mp.ptr, s)) != SPT_OK) break;
            if ((st = upload(t, &t->psplit_ptr[d], mp.psplit_ptr, s)) != SPT_OK) break;
            if ((st = upload(t, &t->psplit_row[d], mp.psplit_row, s)) != SPT_OK) break;
            if ((st = upload(t, &t->psplit_slot[d], mp.psplit_slot, s)) != SPT_OK) break;
            if ((st = upload(t, &t->split_row[d], mp.split_row, s)) != SPT_OK) break;
            if ((st = upload(t, &t->split_ptr[d], mp.split_ptr, s)) != SPT_OK) break;
            if ((st = upload(t, &t->empty_rows[d], mp.empty_rows, s)) != SPT_OK) break;
            if (copies)
                t->rec_mode[d] = dp.rec_mode[d];
            else
                t->nxt[d] = dp.nxt[d];
        }
        if (st == SPT_OK && !copies) {
            t->rec[0] = dp.rec0;
            st = dalloc(t, &t->rec[1], (size_t)std::max<int64_t>(1, nnz) * t->lay.words, &t->allocs);
            // the remap target holds defined records (index 0) until the first remap
            if (st == SPT_OK && hipMemsetAsync(t->rec[1], 0, sizeof(uint32_t) * std::max<int64_t>(1, nnz) * t->lay.words,
                                               s) != hipSuccess)
                st = fail(SPT_ERR_HIP, "hipMemsetAsync of the remap target");
        }
        // the uploads read the plan's host vectors
        if (st == SPT_OK && hipStreamSynchronize(s) != hipSuccess)
            st = fail(SPT_ERR_HIP, "hipStreamSynchronize after upload");
        if (st != SPT_OK) {
            release(t);
            delete t;
            return st;
        }
        t->order0 = std::move(dp.order0);
        t->cur = 0;
        t->cur_mode = 0;
    } catch (const std::bad_alloc&) {
        if (t) {
            release(t);
            delete t;
        }
        return fail(SPT_ERR_OOM, "host allocation failed during preprocessing");
    }
    *out = t;
    return SPT_OK;
}

}  // namespace

spt_status spt_tensor_load_coo(int32_t nmodes, const int64_t* dims, int64_t nnz,
                               const int32_t* indices, const float* values, const spt_opts* opts,
                               void* stream, spt_tensor_t* out) {
    g_last_error.clear();
    if (!out) return fail(SPT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    PlanOptions po;
    int copies = 0, dr = 0;
    spt_status st = get_opts(opts, &po, &copies, &dr);
    if (st != SPT_OK) return st;
    bool range = false;
    std::string msg = po.prep ? spt::validate_shape(nmodes, dims, nnz, indices, &range)
                              : spt::validate(nmodes, dims, nnz, indices, &range);
    if (!msg.empty()) return fail(range ? SPT_ERR_OUT_OF_RANGE : SPT_ERR_INVALID_ARG, msg);
    if (nnz > 0 && !values) return fail(SPT_ERR_INVALID_ARG, "values is NULL");
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    if (po.prep) {
        spt_tensor_s* t = nullptr;
        st = load_device(nmodes, dims, nnz, indices, values, po, copies, s, &t);
        if (st != SPT_OK) return st;
        t->dr = dr;
        if ((st = build_stage_tables(t, s)) != SPT_OK) {
            release(t);
            delete t;
            return st;
        }
        t->prep_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = t;
        return SPT_OK;
    }
    spt_tensor_s* t = nullptr;
    try {
        t = new spt_tensor_s();
        t->N = nmodes;
        t->nnz = nnz;
        for (int w = 0; w < nmodes; ++w) t->dims[w] = dims[w];
        t->copies = copies;
        if (!spt::choose_layout(nmodes, dims, po.layout, &t->lay)) {
            delete t;
            return fail(SPT_ERR_UNSUPPORTED, "the record layout asked for in opts.layout has no kernel for "
                                             "this mode count and these mode sizes");
        }
        Plan plan;
        spt::build_plan(nmodes, dims, nnz, indices, values, po, &plan);
        t->kappa = plan.kappa;
        t->norm_sq = plan.norm_sq;
        const int W = t->lay.words;
        auto pack_stream = [&](const std::vector<int32_t>& order, std::vector<uint32_t>& recs) {
            recs.resize((size_t)nnz * W);
            spt::pack_stream(t->lay, indices, nnz, values, order.data(), recs.data());
        };
        std::vector<uint32_t> recs;
        std::vector<int32_t> nxt;
        for (int d = 0; d < nmodes; ++d) {
            const auto& mp = plan.mode[d];
            t->nsplit[d] = (int32_t)mp.split_row.size();
            t->nslots[d] = (int32_t)mp.slot_part.size();
            t->nempty[d] = (int32_t)mp.empty_rows.size();
            t->max_load[d] = mp.max_load;
            if ((st = upload(t, &t->ptr[d], mp.ptr, s)) != SPT_OK) break;
            if ((st = upload(t, &t->psplit_ptr[d], mp.psplit_ptr, s)) != SPT_OK) break;
            if ((st = upload(t, &t->psplit_row[d], mp.psplit_row, s)) != SPT_OK) break;
            if ((st = upload(t, &t->psplit_slot[d], mp.psplit_slot, s)) != SPT_OK) break;
            if ((st = upload(t, &t->split_row[d], mp.split_row, s)) != SPT_OK) break;
            if ((st = upload(t, &t->split_ptr[d], mp.split_ptr, s)) != SPT_OK) break;
            if ((st = upload(t, &t->empty_rows[d], mp.empty_rows, s)) != SPT_OK) break;
            if (copies) {
                pack_stream(mp.order, recs);
                if ((st = upload(t, &t->rec_mode[d], recs, s)) != SPT_OK) break;
            } else {
                nxt.resize(nnz);
                spt::next_positions(mp.order.data(), plan.mode[(d + 1) % nmodes].remap.data(), nnz,
                                    nxt.data());
                if ((st = upload(t, &t->nxt[d], nxt, s)) != SPT_OK) break;
            }
            // the uploads above read host vectors that are reused next mode
            if (hipStreamSynchronize(s) != hipSuccess) {
                st = fail(SPT_ERR_HIP, "hipStreamSynchronize after upload");
                break;
            }
        }
        if (st == SPT_OK && !copies) {
            pack_stream(plan.mode[0].order, recs);
            if ((st = upload(t, &t->rec[0], recs, s)) == SPT_OK)
                st = dalloc(t, &t->rec[1], recs.size(), &t->allocs);
            // the remap target holds defined records (index 0) until the first remap
            if (st == SPT_OK && !recs.empty() &&
                hipMemsetAsync(t->rec[1], 0, sizeof(uint32_t) * recs.size(), s) != hipSuccess)
                st = fail(SPT_ERR_HIP, "hipMemsetAsync of the remap target");
        }
        if (st == SPT_OK && hipStreamSynchronize(s) != hipSuccess)
            st = fail(SPT_ERR_HIP, "hipStreamSynchronize after upload");
        if (st != SPT_OK) {
            release(t);
            delete t;
            return st;
        }
        t->order0 = plan.mode[0].order;
        t->cur = 0;
        t->cur_mode = 0;
        t->dr = dr;
        if ((st = build_stage_tables(t, s)) != SPT_OK) {
            release(t);
            delete t;
            return st;
        }
    } catch (const std::bad_alloc&) {
        if (t) {
            release(t);
            delete t;
        }
        return fail(SPT_ERR_OOM, "host allocation failed during preprocessing");
    }
    t->prep_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = t;
    return SPT_OK;
}

spt_status spt_timing_control(spt_tensor_t t, int32_t enable, spt_timing* out) {
    g_last_error.clear();
    if (!t) return fail(SPT_ERR_INVALID_ARG, "NULL handle");
    if (out) {
        std::memset(out, 0, sizeof(*out));
        for (const auto& tm : t->timed) {
            HIPCHK(hipEventSynchronize(tm.ev[4] ? tm.ev[4] : tm.ev[3]));
            HIPCHK(hipEventSynchronize(tm.ev[2]));
            float a = 0.f, r = 0.f, b = 0.f, c = 0.f;
            HIPCHK(hipEventElapsedTime(&a, tm.ev[0], tm.ev[1]));
            if (tm.ev[2] != tm.ev[1]) HIPCHK(hipEventElapsedTime(&r, tm.ev[1], tm.ev[2]));
            // a side-stream remap overlaps the fixup: time the fixup from EC's end
            HIPCHK(hipEventElapsedTime(&b, tm.side ? tm.ev[1] : tm.ev[2], tm.ev[3]));
            if (tm.ev[4]) HIPCHK(hipEventElapsedTime(&c, tm.ev[3], tm.ev[4]));
            out->calls[tm.mode] += 1;
            out->ec_ms[tm.mode] += a;
            out->remap_ms[tm.mode] += r;
            out->fixup_ms[tm.mode] += b;
            out->als_ms[tm.mode] += c;
        }
    }
    if (enable) {
        HIPCHK(hipDeviceSynchronize());
        t->timed.clear();
        t->events_used = 0;
    }
    t->timing = enable != 0;
    return SPT_OK;
}

spt_status spt_tensor_free(spt_tensor_t t) {
    g_last_error.clear();
    if (!t) return SPT_OK;
    release(t);
    delete t;
    return SPT_OK;
}

spt_status spt_tensor_info(spt_tensor_t t, spt_info* info) {
    g_last_error.clear();
    if (!t || !info) return fail(SPT_ERR_INVALID_ARG, "NULL handle or info");
    std::memset(info, 0, sizeof(*info));
    info->nmodes = t->N;
    info->cur_mode = t->cur_mode;
    info->kappa = t->kappa;
    info->record_bytes = t->lay.words * 4;
    info->nnz = t->nnz;
    for (int w = 0; w < t->N; ++w) {
        info->dims[w] = t->dims[w];
        info->max_load[w] = t->max_load[w];
        info->split_rows[w] = t->nsplit[w];
    }
    info->norm_sq = t->norm_sq;
    info->prep_seconds = t->prep_seconds;
    info->device_bytes = t->device_bytes;
    info->remap_chunk = t->ddst[0] ? spt::stage_chunk(t->lay.words, t->nnz) : 0;
    return SPT_OK;
}

spt_status spt_remap_for_mode(spt_tensor_t t, int32_t mode, void* stream) {
    g_last_error.clear();
    if (!t) return fail(SPT_ERR_INVALID_ARG, "NULL handle");
    if (mode < 0 || mode >= t->N) return fail(SPT_ERR_INVALID_ARG, "mode out of range");
    return do_remap(t, mode, (hipStream_t)stream);
}

spt_status spt_mttkrp(spt_tensor_t t, int32_t mode, const void* const* factors, spt_dtype fdtype,
                      int32_t rank, float* out, uint32_t flags, void* stream) {
    g_last_error.clear();
    if (!t) return fail(SPT_ERR_INVALID_ARG, "NULL handle");
    if (mode < 0 || mode >= t->N) return fail(SPT_ERR_INVALID_ARG, "mode out of range");
    if (fdtype != SPT_F32 && fdtype != SPT_BF16) return fail(SPT_ERR_UNSUPPORTED, "factor dtype not supported");
    if (!rank_compiled(rank)) return fail(SPT_ERR_UNSUPPORTED, "rank must be 8, 16, 32, 64 or 128");
    if (!factors || !out) return fail(SPT_ERR_INVALID_ARG, "NULL factors or out");
    for (int w = 0; w < t->N; ++w)
        if (w != mode && !factors[w]) return fail(SPT_ERR_INVALID_ARG, "NULL factor matrix");
    for (int w = 0; w < t->N; ++w)
        if (w != mode && !aligned16(factors[w])) return fail(SPT_ERR_INVALID_ARG, "factor matrices must be 16-byte aligned");
    if (!aligned16(out)) return fail(SPT_ERR_INVALID_ARG, "out must be 16-byte aligned");
    if (flags & ~(SPT_FUSE_REMAP_NEXT | SPT_AUTO_REMAP)) return fail(SPT_ERR_INVALID_ARG, "unknown flag");
    hipStream_t s = (hipStream_t)stream;
    if (!t->copies && t->cur_mode != mode) {
        if (!(flags & SPT_AUTO_REMAP))
            return fail(SPT_ERR_STATE, "stream is in mode " + std::to_string(t->cur_mode) +
                                           "'s order, not " + std::to_string(mode) + "'s");
        spt_status st = do_remap(t, mode, s);
        if (st != SPT_OK) return st;
    }
    return run_mttkrp(t, mode, factors, fdtype, rank, out, (flags & SPT_FUSE_REMAP_NEXT) != 0, s);
}

spt_status spt_mttkrp_noalloc(spt_tensor_t t, int32_t mode, const void* const* factors, spt_dtype fdtype,
                              int32_t rank, float* out, uint32_t flags, void* stream) {
    g_last_error.clear();
    if (!t) return fail(SPT_ERR_INVALID_ARG, "NULL handle");
    if (mode < 0 || mode >= t->N) return fail(SPT_ERR_INVALID_ARG, "mode out of range");
    if (fdtype != SPT_F32 && fdtype != SPT_BF16) return fail(SPT_ERR_UNSUPPORTED, "factor dtype not supported");
    if (!rank_compiled(rank)) return fail(SPT_ERR_UNSUPPORTED, "rank must be 8, 16, 32, 64 or 128");
    if (!factors || !out) return fail(SPT_ERR_INVALID_ARG, "NULL factors or out");
    for (int w = 0; w < t->N; ++w)
        if (w != mode && !factors[w]) return fail(SPT_ERR_INVALID_ARG, "NULL factor matrix");
    for (int w = 0; w < t->N; ++w)
        if (w != mode && !aligned16(factors[w])) return fail(SPT_ERR_INVALID_ARG, "factor matrices must be 16-byte aligned");
    if (!aligned16(out)) return fail(SPT_ERR_INVALID_ARG, "out must be 16-byte aligned");
    if (flags & ~(SPT_FUSE_REMAP_NEXT | SPT_AUTO_REMAP)) return fail(SPT_ERR_INVALID_ARG, "unknown flag");
    const int64_t need = (int64_t)t->nslots[mode] * rank * 4;
    if (need > spt::kNoAllocScratchBytes)
        return fail(SPT_ERR_UNSUPPORTED, "the split-row partial sums of this mode need " + std::to_string(need) +
                                             " bytes; the fixed buffer of spt_mttkrp_noalloc holds " +
                                             std::to_string(spt::kNoAllocScratchBytes));
    void* scr = nullptr;
    HIPCHK(spt::noalloc_scratch(&scr));
    hipStream_t s = (hipStream_t)stream;
    if (!t->copies && t->cur_mode != mode) {
        if (!(flags & SPT_AUTO_REMAP))
            return fail(SPT_ERR_STATE, "stream is in mode " + std::to_string(t->cur_mode) + "'s order, not " +
                                           std::to_string(mode) + "'s");
        spt_status st = do_remap(t, mode, s);
        if (st != SPT_OK) return st;
    }
    float* carry = static_cast<float*>(scr);
    if (t->copies) return launch_mode(t, mode, t->rec_mode[mode], nullptr, factors, fdtype, rank, out, s, false, carry);
    const bool fuse = (flags & SPT_FUSE_REMAP_NEXT) != 0;
    spt_status st = launch_mode(t, mode, t->rec[t->cur], fuse ? t->rec[1 - t->cur] : nullptr, factors, fdtype, rank,
                                out, s, false, carry);
    if (st != SPT_OK) return st;
    if (fuse) {
        t->cur = 1 - t->cur;
        t->cur_mode = (mode + 1) % t->N;
    }
    return SPT_OK;
}

spt_status spt_cp_als_iter(spt_tensor_t t, void* const* factors, spt_dtype fdtype, int32_t rank,
                           double* lambda, double* fit, void* stream) {
    g_last_error.clear();
    if (!t) return fail(SPT_ERR_INVALID_ARG, "NULL handle");
    if (fdtype != SPT_F32 && fdtype != SPT_BF16) return fail(SPT_ERR_UNSUPPORTED, "factor dtype not supported");
    if (!als_rank(rank)) return fail(SPT_ERR_UNSUPPORTED, "CP-ALS rank must be 8, 16, 32 or 64");
    if (!factors || !lambda) return fail(SPT_ERR_INVALID_ARG, "NULL factors or lambda");
    for (int w = 0; w < t->N; ++w)
        if (!factors[w]) return fail(SPT_ERR_INVALID_ARG, "NULL factor matrix");
    for (int w = 0; w < t->N; ++w)
        if (!aligned16(factors[w])) return fail(SPT_ERR_INVALID_ARG, "factor matrices must be 16-byte aligned");
    if (!t->copies && t->cur_mode != 0) return fail(SPT_ERR_STATE, "stream must be in mode 0's order");
    if (fit && t->norm_sq <= 0.0) return fail(SPT_ERR_INVALID_ARG, "fit undefined for a zero tensor");
    hipStream_t s = (hipStream_t)stream;
    // a failure flagged by an earlier sweep that was not synchronised
    if (t->status_pending) {
        HIPCHK(hipEventSynchronize(t->status_event));
        t->status_pending = false;
        if (t->status_host[0] != 0) {
            t->status_host[0] = 0;
            return fail(SPT_ERR_NOT_SPD, "normal matrix not positive definite (earlier sweep)");
        }
    }
    spt_status st = ensure_carry(t, rank);
    if (st != SPT_OK) return st;
    if (!t->status_host) {
        HIPCHK(hipHostMalloc((void**)&t->status_host, sizeof(int32_t)));
        t->status_host[0] = 0;
        HIPCHK(hipEventCreateWithFlags(&t->status_event, hipEventDisableTiming));
    }
    const int N = t->N;
    const int64_t E = (int64_t)rank * rank;
    for (int w = 1; w < N; ++w) {
        const int nb = spt::gram_blocks(t->dims[w]);
        spt::launch_gram_partial(rank, (const float*)factors[w], t->dims[w], t->gpart, s);
        spt::launch_reduce_partials(t->gpart, nb, (int)E, t->grams + w * E, s);
    }
    HIPCHK(hipGetLastError());
    const bool bf16 = fdtype == SPT_BF16;
    const void* gath[8];
    for (int w = 0; w < N; ++w) {
        gath[w] = bf16 ? (const void*)t->shadow[w] : (const void*)factors[w];
        if (bf16) spt::launch_to_bf16((const float*)factors[w], t->shadow[w], t->dims[w] * rank, s);
    }
    for (int d = 0; d < N; ++d) {
        // the remap pass of mode d overlaps its fixup and dense update
        st = run_mttkrp(t, d, gath, fdtype, rank, t->M, true, s, true);
        if (st != SPT_OK) return st;
        spt::launch_normal_inverse(rank, N, d, t->grams, t->Vinv, t->status, s);
        const int nb = spt::solve_blocks(t->dims[d]);
        spt::launch_solve_rows(rank, t->M, t->Vinv, t->dims[d], (float*)factors[d], t->gpart,
                               t->ipart, s);
        spt::launch_reduce_partials(t->gpart, nb, (int)E, t->Gsum, s);
        spt::launch_reduce_partials(t->ipart, nb, rank, t->Isum, s);
        spt::launch_als_finish(rank, N, d, t->Gsum, t->Isum, t->grams, lambda, t->norm_sq,
                               (fit && d == N - 1) ? 1 : 0, t->fitd, s);
        spt::launch_scale_cols(rank, (float*)factors[d], t->dims[d], lambda, s);
        if (bf16) spt::launch_to_bf16((const float*)factors[d], t->shadow[d], t->dims[d] * rank, s);
        HIPCHK(hipGetLastError());
        if (t->timing && !t->timed.empty() && t->timed.back().mode == d && !t->timed.back().ev[4])
            t->timed.back().ev[4] = mark(t, s);
        if ((st = join_side(t, s)) != SPT_OK) return st;
    }
    if (t->copies) t->cur_mode = 0;
    HIPCHK(hipMemcpyAsync(t->status_host, t->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    spt::launch_zero_i32(t->status, 1, s);
    HIPCHK(hipEventRecord(t->status_event, s));
    t->status_pending = true;
    if (fit) {
        HIPCHK(hipMemcpyAsync(fit, t->fitd, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        t->status_pending = false;
        if (t->status_host[0] != 0) {
            t->status_host[0] = 0;
            return fail(SPT_ERR_NOT_SPD, "normal matrix not positive definite");
        }
    }
    return SPT_OK;
}

namespace {

// Checks shared by the loss, the adjoint and the gradient.
spt_status grad_args(spt_tensor_t t, const void* const* factors, spt_dtype fdtype, int32_t rank) {
    if (!t) return fail(SPT_ERR_INVALID_ARG, "NULL handle");
    if (fdtype != SPT_F32) return fail(SPT_ERR_UNSUPPORTED, "gradient supports FP32 factors");
    if (!als_rank(rank)) return fail(SPT_ERR_UNSUPPORTED, "gradient rank must be 8, 16, 32 or 64");
    if (!factors) return fail(SPT_ERR_INVALID_ARG, "NULL factors");
    for (int w = 0; w < t->N; ++w)
        if (!factors[w]) return fail(SPT_ERR_INVALID_ARG, "NULL factor matrix");
    for (int w = 0; w < t->N; ++w)
        if (!aligned16(factors[w])) return fail(SPT_ERR_INVALID_ARG, "factor matrices must be 16-byte aligned");
    if (!t->copies && t->cur_mode != 0) return fail(SPT_ERR_STATE, "stream must be in mode 0's order");
    spt_status st = ensure_carry(t, rank);
    if (st != SPT_OK) return st;
    if (!t->res[0]) {
        const int nres = t->copies ? 1 : 2;
        for (int k = 0; k < nres; ++k)
            if ((st = dalloc(t, &t->res[k], (size_t)(t->nnz * t->lay.words), &t->allocs)) != SPT_OK) return st;
        if ((st = dalloc(t, &t->loss_part, (size_t)spt::forward_blocks(t->nnz), &t->allocs)) != SPT_OK)
            return st;
    }
    return SPT_OK;
}

// Forward pass over the mode-0 stream: the residual stream into res[0] and
// the loss into loss[0].
spt_status run_loss(spt_tensor_t t, const void* const* factors, int32_t rank, double* loss, hipStream_t s) {
    const uint32_t* src = t->copies ? t->rec_mode[0] : t->rec[t->cur];
    spt_status st = launch_forward_pass(t, src, t->res[0], factors, rank, s);
    if (st != SPT_OK) return st;
    spt::launch_reduce_partials(t->loss_part, spt::forward_blocks(t->nnz), 1, loss, s);
    HIPCHK(hipGetLastError());
    t->res_rank = rank;
    t->res_cur = 0;
    return SPT_OK;
}

// The adjoint of every mode from the residual stream of the last forward
// pass (res[res_cur], mode 0's order), remapped mode to mode and back to
// mode 0's order.  With one copy per mode each mode's residuals are formed
// again from that mode's own stream.
spt_status run_adjoint(spt_tensor_t t, const void* const* factors, int32_t rank, void* const* grads,
                       hipStream_t s) {
    const int N = t->N;
    spt_status st;
    if (t->copies) {
        for (int d = 0; d < N; ++d) {
            if (d > 0 && (st = launch_forward_pass(t, t->rec_mode[d], t->res[0], factors, rank, s)) != SPT_OK)
                return st;
            if ((st = launch_mode(t, d, t->res[0], nullptr, factors, SPT_F32, rank, (float*)grads[d], s)) != SPT_OK)
                return st;
        }
        // res[0] now holds the last mode's residuals: form mode 0's again
        if (N > 1) return launch_forward_pass(t, t->rec_mode[0], t->res[0], factors, rank, s);
        return SPT_OK;
    }
    int cur = t->res_cur;
    for (int d = 0; d < N; ++d) {
        if ((st = launch_mode(t, d, t->res[cur], t->res[1 - cur], factors, SPT_F32, rank, (float*)grads[d],
                              s)) != SPT_OK)
            return st;
        cur = 1 - cur;
    }
    t->res_cur = cur;  // N remaps: mode 0's order again
    return SPT_OK;
}

}  // namespace

spt_status spt_cp_loss(spt_tensor_t t, const void* const* factors, spt_dtype fdtype, int32_t rank,
                       double* loss, void* stream) {
    g_last_error.clear();
    spt_status st = grad_args(t, factors, fdtype, rank);
    if (st != SPT_OK) return st;
    if (!loss) return fail(SPT_ERR_INVALID_ARG, "NULL loss");
    return run_loss(t, factors, rank, loss, (hipStream_t)stream);
}

spt_status spt_cp_adjoint(spt_tensor_t t, const void* const* factors, spt_dtype fdtype, int32_t rank,
                          void* const* grads, void* stream) {
    g_last_error.clear();
    spt_status st = grad_args(t, factors, fdtype, rank);
    if (st != SPT_OK) return st;
    if (!grads) return fail(SPT_ERR_INVALID_ARG, "NULL grads");
    for (int w = 0; w < t->N; ++w)
        if (!grads[w]) return fail(SPT_ERR_INVALID_ARG, "NULL gradient matrix");
    for (int w = 0; w < t->N; ++w)
        if (!aligned16(grads[w])) return fail(SPT_ERR_INVALID_ARG, "gradient matrices must be 16-byte aligned");
    if (t->res_rank != rank) return fail(SPT_ERR_STATE, "no residual stream of this rank: call spt_cp_loss first");
    return run_adjoint(t, factors, rank, grads, (hipStream_t)stream);
}

spt_status spt_cp_gradient(spt_tensor_t t, const void* const* factors, spt_dtype fdtype,
                           int32_t rank, void* const* grads, double* loss, void* stream) {
    g_last_error.clear();
    spt_status st = grad_args(t, factors, fdtype, rank);
    if (st != SPT_OK) return st;
    if (!grads || !loss) return fail(SPT_ERR_INVALID_ARG, "NULL grads or loss");
    for (int w = 0; w < t->N; ++w)
        if (!grads[w]) return fail(SPT_ERR_INVALID_ARG, "NULL gradient matrix");
    for (int w = 0; w < t->N; ++w)
        if (!aligned16(grads[w])) return fail(SPT_ERR_INVALID_ARG, "gradient matrices must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if ((st = run_loss(t, factors, rank, loss, s)) != SPT_OK) return st;
    return run_adjoint(t, factors, rank, grads, s);
}

spt_status spt_copy_probe(const void* src, void* dst, int64_t bytes, void* stream) {
    g_last_error.clear();
    if (bytes < 0 || bytes % 16 != 0) return fail(SPT_ERR_INVALID_ARG, "bytes must be a non-negative multiple of 16");
    if (bytes > 0 && (!src || !dst)) return fail(SPT_ERR_INVALID_ARG, "NULL src or dst");
    if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return fail(SPT_ERR_INVALID_ARG, "src and dst must be 16-byte aligned");
    spt::launch_copy_probe(src, dst, bytes, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return SPT_OK;
}

spt_status spt_tensor_get_remap(spt_tensor_t t, int32_t mode, int64_t* b_host) {
    g_last_error.clear();
    if (!t || !b_host) return fail(SPT_ERR_INVALID_ARG, "NULL handle or output");
    if (mode < 0 || mode >= t->N) return fail(SPT_ERR_INVALID_ARG, "mode out of range");
    if (t->copies) return fail(SPT_ERR_UNSUPPORTED, "no remap ids are held with one copy per mode");
    const int64_t nnz = t->nnz;
    try {
        // b_0 from the mode-0 stream, then follow the device's next-position
        // arrays mode by mode
        std::vector<int32_t> pos(nnz), nx(nnz);
        for (int64_t p = 0; p < nnz; ++p) pos[t->order0[p]] = (int32_t)p;
        for (int d = 0; d < mode; ++d) {
            if (nnz) HIPCHK(hipMemcpy(nx.data(), t->nxt[d], sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
            for (int64_t e = 0; e < nnz; ++e) pos[e] = nx[pos[e]];
        }
        for (int64_t e = 0; e < nnz; ++e) b_host[e] = pos[e];
    } catch (const std::bad_alloc&) {
        return fail(SPT_ERR_OOM, "host allocation failed");
    }
    return SPT_OK;
}

spt_status spt_tensor_get_records(spt_tensor_t t, int32_t* idx_host, float* val_host,
                                  int32_t* cur_mode) {
    g_last_error.clear();
    if (!t || !idx_host || !val_host) return fail(SPT_ERR_INVALID_ARG, "NULL handle or output");
    const int64_t nnz = t->nnz;
    const int W = t->lay.words;
    const uint32_t* src = t->copies ? t->rec_mode[t->cur_mode] : t->rec[t->cur];
    try {
        std::vector<uint32_t> recs((size_t)nnz * W);
        HIPCHK(hipDeviceSynchronize());
        if (nnz) HIPCHK(hipMemcpy(recs.data(), src, recs.size() * 4, hipMemcpyDeviceToHost));
        int32_t c[8];
        for (int64_t p = 0; p < nnz; ++p) {
            spt::unpack_record(t->lay, &recs[(size_t)p * W], c, &val_host[p]);
            for (int w = 0; w < t->N; ++w) idx_host[(int64_t)w * nnz + p] = c[w];
        }
    } catch (const std::bad_alloc&) {
        return fail(SPT_ERR_OOM, "host allocation failed");
    }
    if (cur_mode) *cur_mode = t->cur_mode;
    return SPT_OK;
}

}  // extern "C"
