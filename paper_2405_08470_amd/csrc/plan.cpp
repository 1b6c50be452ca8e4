// Host-side preprocessing: Algorithm 1 (Sec. 3.4) with the piece split of
// heavy rows, remap ids, record packing and the tables the kernels use.
// Multithreaded with std::thread; every result is independent of the
// thread count.
#include "plan.hpp"

#include <algorithm>
#include <cstring>
#include <functional>
#include <queue>
#include <thread>
#include <utility>

namespace spt {

namespace {

int bit_length(int64_t v) {
    int b = 0;
    while (v > 0) {
        ++b;
        v >>= 1;
    }
    return b;
}

int num_threads() {
    unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, h ? h : 1u));
}

// Runs fn(begin, end, part) over [0, n) split into `parts` contiguous spans.
void parallel_for(int64_t n, int parts, const std::function<void(int64_t, int64_t, int)>& fn) {
    parts = (int)std::max<int64_t>(1, std::min<int64_t>(parts, n / 65536 + 1));
    if (parts == 1) {
        fn(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < parts; ++t) {
        const int64_t b = n * t / parts, e = n * (t + 1) / parts;
        th.emplace_back(fn, b, e, t);
    }
    for (auto& x : th) x.join();
}

// Stable counting sort of the permutation `in` (n entries) by key[in[p]] in
// [0, nkeys); result in `out`.  Each thread histograms and scatters its own
// contiguous span; spans are placed in order, so the sort is stable.
void counting_sort(const int32_t* in, int64_t n, const int32_t* key, int64_t nkeys, int32_t* out) {
    int T = num_threads();
    T = (int)std::max<int64_t>(1, std::min<int64_t>(T, n / 65536 + 1));
    // bound the histogram memory for very many keys
    while (T > 1 && (int64_t)T * nkeys > (int64_t)1 << 27) --T;
    std::vector<std::vector<int64_t>> hist(T, std::vector<int64_t>(nkeys, 0));
    auto span = [&](int t, int64_t* b, int64_t* e) {
        *b = n * t / T;
        *e = n * (t + 1) / T;
    };
    {
        std::vector<std::thread> th;
        for (int t = 0; t < T; ++t)
            th.emplace_back([&, t] {
                int64_t b, e;
                span(t, &b, &e);
                int64_t* h = hist[t].data();
                for (int64_t p = b; p < e; ++p) ++h[key[in[p]]];
            });
        for (auto& x : th) x.join();
    }
    int64_t run = 0;
    for (int64_t k = 0; k < nkeys; ++k)
        for (int t = 0; t < T; ++t) {
            const int64_t c = hist[t][k];
            hist[t][k] = run;
            run += c;
        }
    {
        std::vector<std::thread> th;
        for (int t = 0; t < T; ++t)
            th.emplace_back([&, t] {
                int64_t b, e;
                span(t, &b, &e);
                int64_t* h = hist[t].data();
                for (int64_t p = b; p < e; ++p) out[h[key[in[p]]]++] = in[p];
            });
        for (auto& x : th) x.join();
    }
}

struct Item {
    int64_t size;
    int32_t row;
    int32_t piece;
};

}  // namespace

void partition_rows(int64_t I, const int64_t* deg, int32_t kappa, int64_t cap, ModePlan& mp,
                    RowPieces& rp) {
    std::vector<int64_t>& piece_base = rp.piece_base;
    std::vector<int32_t>& piece_part = rp.piece_part;
    std::vector<int32_t>& piece_seg = rp.piece_seg;
    // items: each vertex, or its pieces when heavier than cap
    piece_base.assign(I + 1, 0);
    for (int64_t i = 0; i < I; ++i) {
        int64_t k = (cap > 0 && deg[i] > cap) ? (deg[i] + cap - 1) / cap : 1;
        piece_base[i + 1] = piece_base[i] + k;
    }
    const int64_t nitems = piece_base[I];
    std::vector<Item> items(nitems);
    for (int64_t i = 0; i < I; ++i) {
        int64_t k = piece_base[i + 1] - piece_base[i];
        int64_t q = deg[i] / k, rem = deg[i] % k;
        for (int64_t j = 0; j < k; ++j)
            items[piece_base[i] + j] = Item{q + (j < rem ? 1 : 0), (int32_t)i, (int32_t)j};
    }
    // decreasing size, then row, then piece
    std::sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
        if (a.size != b.size) return a.size > b.size;
        if (a.row != b.row) return a.row < b.row;
        return a.piece < b.piece;
    });
    // least-filled block first, ties to the lowest block id: a min-heap on
    // (load, id)
    using LoadId = std::pair<int64_t, int32_t>;
    std::priority_queue<LoadId, std::vector<LoadId>, std::greater<LoadId>> heap;
    for (int32_t z = 0; z < kappa; ++z) heap.push(LoadId(0, z));
    piece_part.assign(nitems, 0);
    mp.loads.assign(kappa, 0);
    for (const Item& it : items) {
        LoadId top = heap.top();
        heap.pop();
        piece_part[piece_base[it.row] + it.piece] = top.second;
        top.first += it.size;
        mp.loads[top.second] = top.first;
        heap.push(top);
    }
    items.clear();
    items.shrink_to_fit();
    mp.ptr.assign(kappa + 1, 0);
    for (int32_t z = 0; z < kappa; ++z) mp.ptr[z + 1] = mp.ptr[z] + mp.loads[z];
    mp.max_load = *std::max_element(mp.loads.begin(), mp.loads.end());

    // segments = distinct (partition, row) pairs in (partition, row) order
    std::vector<std::pair<int32_t, int32_t>> pairs;
    pairs.reserve(nitems);
    for (int64_t i = 0; i < I; ++i)
        for (int64_t j = piece_base[i]; j < piece_base[i + 1]; ++j)
            pairs.push_back({piece_part[j], (int32_t)i});
    std::sort(pairs.begin(), pairs.end());
    pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
    rp.nseg = (int64_t)pairs.size();
    piece_seg.assign(nitems, 0);
    for (int64_t i = 0; i < I; ++i)
        for (int64_t j = piece_base[i]; j < piece_base[i + 1]; ++j) {
            auto it = std::lower_bound(pairs.begin(), pairs.end(),
                                       std::make_pair(piece_part[j], (int32_t)i));
            piece_seg[j] = (int32_t)(it - pairs.begin());
        }
    pairs.clear();
    pairs.shrink_to_fit();

    // split rows: pieces in two or more partitions
    mp.split_row.clear();
    mp.split_ptr.assign(1, 0);
    mp.slot_part.clear();
    std::vector<std::vector<std::pair<int32_t, int32_t>>> per_part(kappa);
    std::vector<int32_t> parts;
    for (int64_t i = 0; i < I; ++i) {
        const int64_t k = piece_base[i + 1] - piece_base[i];
        if (k < 2) continue;
        parts.assign(piece_part.begin() + piece_base[i], piece_part.begin() + piece_base[i + 1]);
        std::sort(parts.begin(), parts.end());
        parts.erase(std::unique(parts.begin(), parts.end()), parts.end());
        if (parts.size() < 2) continue;
        mp.split_row.push_back((int32_t)i);
        for (int32_t z : parts) {
            int32_t slot = (int32_t)mp.slot_part.size();
            mp.slot_part.push_back(z);
            per_part[z].push_back({(int32_t)i, slot});
        }
        mp.split_ptr.push_back((int32_t)mp.slot_part.size());
    }
    mp.psplit_ptr.assign(kappa + 1, 0);
    mp.psplit_row.clear();
    mp.psplit_slot.clear();
    for (int32_t z = 0; z < kappa; ++z) {
        for (auto& rs : per_part[z]) {
            mp.psplit_row.push_back(rs.first);
            mp.psplit_slot.push_back(rs.second);
        }
        mp.psplit_ptr[z + 1] = (int32_t)mp.psplit_row.size();
    }
    mp.empty_rows.clear();
    for (int64_t i = 0; i < I; ++i)
        if (deg[i] == 0) mp.empty_rows.push_back((int32_t)i);
}

int64_t piece_of_rank(int64_t deg, int64_t k, int64_t rank) {
    if (k <= 1) return 0;
    const int64_t q = deg / k, rem = deg % k, big = rem * (q + 1);
    return rank < big ? rank / (q + 1) : rem + (rank - big) / q;
}

namespace {

// Partitions one mode: Alg. 1 over the rows (or their pieces), then the
// partition and the (partition, row) segment of every nonzero.
void plan_mode(int d, const int64_t* dims, int64_t nnz, const int32_t* idx, int32_t kappa,
               int64_t cap, ModePlan& mp, std::vector<int32_t>& seg, int64_t* nseg) {
    const int64_t I = dims[d];
    const int32_t* c = idx + (int64_t)d * nnz;
    std::vector<int64_t> deg(I, 0);
    for (int64_t e = 0; e < nnz; ++e) ++deg[c[e]];
    RowPieces rp;
    partition_rows(I, deg.data(), kappa, cap, mp, rp);
    *nseg = rp.nseg;
    const std::vector<int64_t>& piece_base = rp.piece_base;
    // partition and segment of every nonzero: its row's piece, pieces taking
    // the row's nonzeros in input order
    mp.part.resize(nnz);
    seg.resize(nnz);
    std::vector<int64_t> seen(I, 0);
    for (int64_t e = 0; e < nnz; ++e) {
        const int32_t i = c[e];
        const int64_t k = piece_base[i + 1] - piece_base[i];
        const int64_t j = k > 1 ? piece_of_rank(deg[i], k, seen[i]++) : 0;
        mp.part[e] = rp.piece_part[piece_base[i] + j];
        seg[e] = rp.piece_seg[piece_base[i] + j];
    }
}

}  // namespace

int32_t default_kappa(int64_t nnz) {
    // about 2048 nonzeros per partition, at most 8192 partitions: fewer, larger
    // partitions give the remap longer runs of adjacent destinations, and 8192
    // one-wave workgroups still fill the chip (measured over kappa 2048..65536
    // on 50M..100M-nonzero tensors)
    int64_t k = (nnz + 2047) / 2048;
    return (int32_t)std::min<int64_t>(8192, std::max<int64_t>(1, k));
}

std::string validate(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                     bool* range_error) {
    std::string m = validate_shape(nmodes, dims, nnz, idx, range_error);
    if (!m.empty()) return m;
    for (int w = 0; w < nmodes; ++w) {
        const int32_t* c = idx + (int64_t)w * nnz;
        const int64_t I = dims[w];
        for (int64_t e = 0; e < nnz; ++e) {
            if (c[e] < 0 || c[e] >= I) {
                *range_error = true;
                return "index " + std::to_string(c[e]) + " of nonzero " + std::to_string(e) +
                       " is outside mode " + std::to_string(w) + " (size " + std::to_string(I) +
                       ")";
            }
        }
    }
    return "";
}

std::string validate_shape(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                           bool* range_error) {
    *range_error = false;
    if (nmodes < 2 || nmodes > kMaxModes) return "nmodes must be in [2, 8]";
    if (!dims) return "dims is NULL";
    for (int w = 0; w < nmodes; ++w) {
        if (dims[w] < 1 || dims[w] >= (int64_t(1) << 31)) {
            *range_error = true;
            return "dims[" + std::to_string(w) + "] = " + std::to_string(dims[w]) +
                   " is outside [1, 2^31)";
        }
    }
    if (nnz < 0 || nnz >= (int64_t(1) << 31)) {
        *range_error = true;
        return "nnz = " + std::to_string(nnz) + " is outside [0, 2^31)";
    }
    if (nnz > 0 && !idx) return "indices is NULL";
    return "";
}

bool choose_layout(int nmodes, const int64_t* dims, int pref, RecordLayout* lay) {
    lay->nmodes = nmodes;
    int packed_bits = 0;
    bool small = true;
    for (int w = 0; w < nmodes; ++w) {
        packed_bits += std::max(1, bit_length(dims[w] - 1));
        small = small && dims[w] <= 65536;
    }
    auto set = [&](int kind, int words) {
        lay->kind = kind;
        lay->words = words;
        int o = 0;
        for (int w = 0; w < nmodes; ++w) {
            const int b = kind == kWord32 ? 32 : kind == kHalf16 ? 16
                                                                 : std::max(1, bit_length(dims[w] - 1));
            lay->bits[w] = b;
            lay->off[w] = o;
            o += b;
        }
    };
    if (nmodes < 1 || nmodes > kMaxModes) return false;
    // 12-byte records: the indices in the first 64 bits, in the cheapest
    // decode that fits (whole words, 16-bit fields, else bit fields)
    auto compact = [&]() {
        if (nmodes <= 2)
            set(kWord32, 3);
        else if (nmodes == 4 && small)
            set(kHalf16, 3);
        else if (packed_bits <= 64)
            set(kPacked, 3);
        else
            return false;
        return true;
    };
    const int word32_words = nmodes <= 3 ? 4 : nmodes <= 7 ? 8 : 12;
    switch (pref) {
        case kLayoutCompact:
            return compact();
        case kLayoutWord32:
            set(kWord32, word32_words);
            return true;
        case kLayoutHalf16:
            // 16-bit fields exist for 4..6 modes (16 B) and 8 modes (32 B)
            if (!small || nmodes <= 3 || nmodes == 7) return false;
            set(kHalf16, nmodes <= 6 ? 4 : 8);
            return true;
        case kLayoutPacked:
            if (nmodes <= 3 || nmodes > 6 || packed_bits > 96) return false;
            set(kPacked, 4);
            return true;
        default:
            break;
    }
    if (compact())
        return true;
    if (nmodes <= 3)
        set(kWord32, 4);
    else if (small && nmodes <= 6)
        set(kHalf16, 4);
    else if (packed_bits <= 96 && nmodes <= 6)
        set(kPacked, 4);
    else if (nmodes <= 7)
        set(kWord32, 8);
    else if (small)
        set(kHalf16, 8);
    else
        set(kWord32, 12);
    return true;
}

void pack_record(const RecordLayout& lay, const int32_t* idx, int64_t nnz, const float* val,
                 int64_t e, uint32_t* out) {
    for (int k = 0; k < lay.words; ++k) out[k] = 0;
    for (int w = 0; w < lay.nmodes; ++w) {
        const uint64_t v = (uint32_t)idx[(int64_t)w * nnz + e];
        const int o = lay.off[w];
        const int wi = o >> 5, sh = o & 31;
        out[wi] |= (uint32_t)(v << sh);
        if (sh + lay.bits[w] > 32) out[wi + 1] |= (uint32_t)(v >> (32 - sh));
    }
    float f = val ? val[e] : 0.0f;
    std::memcpy(&out[lay.words - 1], &f, 4);
}

void unpack_record(const RecordLayout& lay, const uint32_t* rec, int32_t* c, float* v) {
    for (int w = 0; w < lay.nmodes; ++w) {
        const int o = lay.off[w];
        const int wi = o >> 5, sh = o & 31;
        const uint64_t lo = rec[wi];
        const uint64_t hi = (wi + 1 < lay.words - 1) ? rec[wi + 1] : 0;
        const uint64_t x = ((hi << 32) | lo) >> sh;
        c[w] = (int32_t)(x & ((uint64_t(1) << lay.bits[w]) - 1));
    }
    std::memcpy(v, &rec[lay.words - 1], 4);
}

void pack_stream(const RecordLayout& lay, const int32_t* idx, int64_t nnz, const float* val,
                 const int32_t* order, uint32_t* out) {
    const int W = lay.words;
    parallel_for(nnz, num_threads(), [&](int64_t b, int64_t e, int) {
        for (int64_t p = b; p < e; ++p) pack_record(lay, idx, nnz, val, order[p], out + p * W);
    });
}

void next_positions(const int32_t* order, const int32_t* remap_next, int64_t nnz, int32_t* nxt) {
    parallel_for(nnz, num_threads(), [&](int64_t b, int64_t e, int) {
        for (int64_t p = b; p < e; ++p) nxt[p] = remap_next[order[p]];
    });
}

void build_plan(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                const float* val, const PlanOptions& opt, Plan* plan) {
    const int N = nmodes;
    plan->nmodes = N;
    plan->nnz = nnz;
    plan->dims.assign(dims, dims + N);
    plan->kappa = opt.kappa > 0 ? opt.kappa : default_kappa(nnz);
    const int32_t kappa = plan->kappa;
    int64_t cap;
    if (opt.split_cap < 0)
        cap = 0;  // never split
    else if (opt.split_cap == 0)
        cap = std::max<int64_t>(1, (nnz + kappa - 1) / kappa);
    else
        cap = opt.split_cap;
    plan->cap = cap;

    // modes are independent: one thread each
    std::vector<std::vector<int32_t>> seg(N);
    std::vector<int64_t> nseg(N, 0);
    {
        std::vector<std::thread> th;
        for (int d = 0; d < N; ++d)
            th.emplace_back([&, d] { plan_mode(d, dims, nnz, idx, kappa, cap, plan->mode[d], seg[d], &nseg[d]); });
        for (auto& x : th) x.join();
    }

    if (opt.remap_ids) {
        // Stream of mode d: sorted by (z_d, c_d, z_{d-1}, c_{d-1}, ...,
        // z_{d+1}, c_{d+1}, e).  Segment ids order the pairs (z_w, c_w), so
        // the stream is built least significant key first by stable sorts
        // on seg_w for w = 1, 2, ..., N-1, 0; after that each further stable
        // sort by seg_d yields mode d's stream.
        std::vector<int32_t> order(nnz), tmp(nnz);
        for (int64_t e = 0; e < nnz; ++e) order[e] = (int32_t)e;
        auto sort_by = [&](int w) {
            counting_sort(order.data(), nnz, seg[w].data(), nseg[w], tmp.data());
            order.swap(tmp);
        };
        for (int k = 1; k <= N; ++k) sort_by(k % N);
        for (int d = 0; d < N; ++d) {
            if (d > 0) sort_by(d);
            ModePlan& mp = plan->mode[d];
            mp.order = order;
            mp.remap.resize(nnz);
            parallel_for(nnz, num_threads(), [&](int64_t b, int64_t e, int) {
                for (int64_t p = b; p < e; ++p) mp.remap[order[p]] = (int32_t)p;
            });
        }
    }
    seg.clear();

    if (opt.norm) {
        // ||X||^2 with repeated coordinates summed first: sort by the full
        // coordinate (stable passes over modes N-1 .. 0), then FP64 sums of
        // each run in input order, totalled in coordinate order.
        std::vector<int32_t> order(nnz), tmp(nnz);
        for (int64_t e = 0; e < nnz; ++e) order[e] = (int32_t)e;
        for (int w = N - 1; w >= 0; --w) {
            counting_sort(order.data(), nnz, idx + (int64_t)w * nnz, dims[w], tmp.data());
            order.swap(tmp);
        }
        auto same = [&](int64_t a, int64_t b) {
            for (int w = 0; w < N; ++w)
                if (idx[(int64_t)w * nnz + a] != idx[(int64_t)w * nnz + b]) return false;
            return true;
        };
        double total = 0.0;
        int64_t p = 0;
        while (p < nnz) {
            int64_t q = p + 1;
            double s = val ? (double)val[order[p]] : 0.0;
            while (q < nnz && same(order[p], order[q])) {
                s += val ? (double)val[order[q]] : 0.0;
                ++q;
            }
            total += s * s;
            p = q;
        }
        plan->norm_sq = total;
    }
}

}  // namespace spt
