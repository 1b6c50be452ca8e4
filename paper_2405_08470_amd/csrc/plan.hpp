// Host-side preprocessing of a COO tensor: per-mode partitioning (Alg. 1,
// Sec. 3.4), remap ids (Sec. 3.4-3.5) and the packed record stream.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace spt {

constexpr int kMaxModes = 8;

// Layout of one record <c_0..c_{N-1}, val>: the indices fill words
// 0 .. words-2, the last word holds the FP32 value.  Index w occupies bits
// [off[w], off[w] + bits[w]) of the little-endian index words.  Kinds:
//   kWord32  index w is word w                      (N <= words - 1)
//   kHalf16  index w is the half-word w (dims <= 2^16)
//   kPacked  indices packed back to back, each ceil(log2 I_w) bits, in the
//            first 64 bits (12-byte records) or 96 bits (16-byte records)
// A 12-byte record (words = 3) holds its indices in 64 bits: kWord32 for
// N <= 2, kHalf16 for N = 4, kPacked otherwise.
enum LayoutKind : int { kWord32 = 0, kHalf16 = 1, kPacked = 2 };

struct RecordLayout {
    int nmodes = 0;
    int words = 0;            // 3 (12 B), 4 (16 B), 8 (32 B) or 12 (48 B)
    int kind = kWord32;
    int bits[kMaxModes] = {};
    int off[kMaxModes] = {};
};

struct ModePlan {
    std::vector<int32_t> part;        // [nnz] partition of each nonzero (z_d)
    std::vector<int64_t> loads;       // [kappa]
    std::vector<int64_t> ptr;         // [kappa+1]
    std::vector<int32_t> order;       // [nnz] nonzero at each stream position
    std::vector<int32_t> remap;       // [nnz] b_d(e): position of e
    // rows whose pieces landed in >= 2 partitions ("split rows"); one carry
    // slot per (row, partition), slots ordered by (row, partition)
    std::vector<int32_t> split_row;   // [nsplit]
    std::vector<int32_t> split_ptr;   // [nsplit+1] slot ranges per split row
    std::vector<int32_t> slot_part;   // [nslots]
    // per partition: its split rows and their slots (CSR over partitions)
    std::vector<int32_t> psplit_ptr;  // [kappa+1]
    std::vector<int32_t> psplit_row;  // [nslots]
    std::vector<int32_t> psplit_slot; // [nslots]
    std::vector<int32_t> empty_rows;  // rows with no nonzero
    int64_t max_load = 0;
};

struct Plan {
    int nmodes = 0;
    int64_t nnz = 0;
    int32_t kappa = 0;
    int64_t cap = 0;
    std::vector<int64_t> dims;
    ModePlan mode[kMaxModes];
    RecordLayout layout;
    double norm_sq = 0.0;
};

struct PlanOptions {
    int32_t kappa = 0;       // 0 -> default_kappa(nnz)
    int64_t split_cap = 0;   // 0 -> ceil(nnz/kappa); <0 -> never split
    bool remap_ids = true;   // build orders / remap ids
    bool norm = true;        // compute ||X||^2 of the coalesced tensor
    int prep = 0;            // 0: host planner, 1: device planner (load only)
    int layout = 0;          // kLayout* record layout preference (load only)
};

// Items of one mode after Alg. 1: rows, or pieces of rows heavier than the
// cap.  Item j of row i is piece_base[i] + j; its partition and its segment
// (rank of the distinct (partition, row) pair) are piece_part / piece_seg.
struct RowPieces {
    std::vector<int64_t> piece_base;  // [I+1]
    std::vector<int32_t> piece_part;  // [nitems]
    std::vector<int32_t> piece_seg;   // [nitems]
    int64_t nseg = 0;
};

// Alg. 1 from the degrees of one mode's rows: least-loaded assignment of the
// items (pieces of at most `cap` nonzeros; cap 0: whole rows), partition
// loads and offsets, split-row and empty-row tables.  Fills mp (all but
// part/order/remap) and rp.
void partition_rows(int64_t I, const int64_t* deg, int32_t kappa, int64_t cap, ModePlan& mp,
                    RowPieces& rp);

// Piece of the nonzero of input-order rank `rank` within a row of degree
// `deg` cut into k pieces (the first deg mod k pieces one larger).
int64_t piece_of_rank(int64_t deg, int64_t k, int64_t rank);

int32_t default_kappa(int64_t nnz);

// Validates the input; returns "" or a message (and sets *range_error when
// the failure is an index or size out of range).
std::string validate(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                     bool* range_error);

// The checks of validate() that do not read the indices.
std::string validate_shape(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                           bool* range_error);

// Computes the whole plan.  Throws std::bad_alloc on allocation failure.
void build_plan(int nmodes, const int64_t* dims, int64_t nnz, const int32_t* idx,
                const float* val, const PlanOptions& opt, Plan* plan);

// Chooses the smallest record, preferring layouts the kernels decode with
// fixed shifts; returns false if no layout fits.
// Record layout preference (spt_opts.layout): automatic, or one kind forced.
enum { kLayoutAuto = 0, kLayoutWord32 = 1, kLayoutHalf16 = 2, kLayoutPacked = 3, kLayoutCompact = 4 };
// false if the preferred kind has no kernel for this mode count or these dims
bool choose_layout(int nmodes, const int64_t* dims, int pref, RecordLayout* lay);

// Packs nonzero e into `words` 32-bit words.
void pack_record(const RecordLayout& lay, const int32_t* idx, int64_t nnz, const float* val,
                 int64_t e, uint32_t* out);
void unpack_record(const RecordLayout& lay, const uint32_t* rec, int32_t* c, float* v);

// out[p] = packed record of nonzero order[p], p < nnz (multithreaded).
void pack_stream(const RecordLayout& lay, const int32_t* idx, int64_t nnz, const float* val,
                 const int32_t* order, uint32_t* out);
// nxt[p] = remap_next[order[p]] (multithreaded).
void next_positions(const int32_t* order, const int32_t* remap_next, int64_t nnz, int32_t* nxt);

}  // namespace spt
