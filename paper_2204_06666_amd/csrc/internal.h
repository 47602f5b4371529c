// Internal definitions shared by the host preprocessing (C++) and the device
// launch code (HIP).  Not part of the public ABI.
#pragma once

#include <atomic>
#include <cstdint>
#include <exception>
#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "ehyb.h"

namespace ehyb {

constexpr int kWave = 64;              // gfx950 wavefront width
// ELL entries per lane per load step: 16 bytes of values (FP64 2, FP32 4, BF16 8)
// How a plan's values are stored (the ACC64 types store like F32 / BF16).
constexpr int storage_dtype(int value_dtype) {
    return value_dtype == EHYB_F32_ACC64 ? EHYB_F32 : (value_dtype == EHYB_BF16_ACC64 ? EHYB_BF16 : value_dtype);
}
constexpr int kc_for(int value_dtype) {
    return storage_dtype(value_dtype) == EHYB_F64 ? 2 : (storage_dtype(value_dtype) == EHYB_F32 ? 4 : 8);
}
constexpr int value_bytes(int value_dtype) {
    return storage_dtype(value_dtype) == EHYB_F64 ? 8 : (storage_dtype(value_dtype) == EHYB_F32 ? 4 : 2);
}
constexpr int x_bytes(int value_dtype) { return value_dtype == EHYB_F64 ? 8 : 4; }
// bytes of one residual accumulator in LDS
constexpr int acc_bytes(int value_dtype) {
    return (value_dtype == EHYB_F64 || value_dtype == EHYB_F32_ACC64 || value_dtype == EHYB_BF16_ACC64) ? 8 : 4;
}
constexpr bool valid_dtype(int value_dtype) { return value_dtype >= EHYB_F64 && value_dtype <= EHYB_BF16_ACC64; }
constexpr size_t kBlobAlign = 256;
constexpr int kStaticLds = 64;         // LDS the SpMV kernel keeps for its queue counters
// A residual row that would need more than kWideSteps load steps on its L
// lanes gets a residual slice of its own, processed by all 64 lanes of a
// wavefront ("wide" slice, flagged by bit 31 of its step count).
constexpr int kWideSteps = 32;
// The automatic ELL width cap: a row-slice lane group loads at most this many
// steps of one row (256 FP64 entries per lane at one lane per row).
constexpr int kAutoCapSteps = 128;
constexpr uint32_t kErWide = 1u << 31;
// ehyb_spmv sums every wide residual slice before the product, spread over
// the whole device in pieces of at most kPieceSteps steps (one wavefront
// each); the partition's workgroup then adds its row's pieces in order.
constexpr int kPieceSteps = 8;  // 8 was 3% faster than 16 on power-law graphs, 32 slower

// An exception must not leave an OpenMP region or task: the process would
// terminate.  Bodies that allocate run through run(): the first exception is
// kept (later bodies are skipped, but every thread still reaches every
// barrier of the region), and rethrow() raises it after the region, where
// the entry point turns std::bad_alloc into EHYB_ENOMEM.
class OmpGuard {
public:
    template <class F>
    void run(F&& f) noexcept {
        if (failed_.load(std::memory_order_relaxed)) return;
        try {
            f();
        } catch (...) {
            bool expected = false;
            if (failed_.compare_exchange_strong(expected, true)) error_ = std::current_exception();
        }
    }
    void rethrow() const {
        if (failed_.load(std::memory_order_acquire)) std::rethrow_exception(error_);
    }
    bool failed() const { return failed_.load(std::memory_order_relaxed); }

private:
    std::atomic<bool> failed_{false};
    std::exception_ptr error_;
};

// Allocator whose resize() leaves new elements uninitialised, so that large
// arrays filled by parallel loops are not first zeroed by one thread.
template <class T>
struct NoInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <class U>
    NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
    template <class U>
    void construct(U* p) noexcept {
        ::new ((void*)p) U;
    }
    template <class U, class... Args>
    void construct(U* p, Args&&... args) {
        ::new ((void*)p) U(std::forward<Args>(args)...);
    }
};
template <class T>
using uvec = std::vector<T, NoInitAlloc<T>>;

// Undirected graph in CSR form with vertex and edge weights.
struct Graph {
    int32_t n = 0;
    uvec<int64_t> xadj;   // [n+1]
    uvec<int32_t> adj;    // [xadj[n]]
    uvec<int32_t> ew;     // edge weights, parallel to adj
    uvec<int32_t> vw;     // vertex weights [n]
    int64_t total_vw() const;
};

// Sets err and returns a status.
struct Error {
    ehyb_status status = EHYB_OK;
    std::string msg;
    bool ok() const { return status == EHYB_OK; }
};

// Multilevel k-way graph partitioning with a hard cap on part weight.
// part[v] in [0, nparts_out); every part non-empty and of weight <= cap.
Error partition_multilevel(const Graph& g, int32_t nparts, int64_t cap, uint64_t seed,
                           std::vector<int32_t>& part, int32_t& nparts_out);

// Byte offsets of each array inside the device blob.
struct BlobLayout {
    size_t part_start = 0, slice_start = 0, er_slice_start = 0, ell_free = 0;
    size_t halo_start = 0, halo_idx = 0;
    size_t ell_meta = 0, er_meta = 0, er_row = 0;
    size_t ell_val = 0, ell_col = 0, er_val = 0, er_col = 0;
    size_t perm = 0, xp = 0, yp = 0;
    size_t piece_start = 0, piece_nwide = 0, pieces = 0, ypart = 0;  // wide residual slices in pieces
    size_t total = 0;
};

}  // namespace ehyb

struct ehyb_plan {
    int64_t n = 0, nnz = 0;
    ehyb_params params{};          // resolved parameters
    int32_t L = 1, C = 64, kc = 2;
    int32_t nparts = 0, nslices = 0, ner_slices = 0;
    int32_t value_dtype = EHYB_F64;
    int32_t vbytes = 8;            // bytes per stored value
    int32_t xbytes = 8;            // bytes per x element
    int32_t eq1_K = 1;
    int32_t max_part_rows = 0;
    std::vector<int32_t> perm;            // new -> old
    std::vector<int32_t> iperm;           // old -> new (the reorder table)
    std::vector<int32_t> part_start;      // [nparts+1]
    std::vector<int32_t> slice_start;     // [nparts+1] ELL slices
    std::vector<int32_t> er_slice_start;  // [nparts+1] residual slices
    std::vector<int32_t> ell_free;        // [nparts] leading ELL slices without residual rows
    std::vector<int32_t> halo_start;      // [nparts+1]
    std::vector<int32_t> halo_idx;        // cached neighbour x entries (permuted global indices)
    std::vector<uint32_t> ell_meta;       // [4*nslices] off, steps | index << 16, er mask lo, hi
    std::vector<uint32_t> er_meta;        // [2*ner_slices] off, steps
    std::vector<uint16_t> er_row;         // [C*ner_slices] local row, 0xFFFF = none
    std::vector<int32_t> er_pos;          // [n] permuted row -> e*C + r in the residual part, -1
    std::vector<unsigned char> ell_val;   // ell_slots * vbytes
    std::vector<uint16_t> ell_col;        // ell_slots
    std::vector<unsigned char> er_val;    // er_slots * vbytes
    std::vector<int32_t> er_col;          // er_slots
    std::vector<int32_t> row_ell_len, row_er_len;  // [n], permuted rows
    // pieces of the wide residual slices (derived from er_meta): piece_start
    // [ner_slices+1] gives each slice's first piece (none for other slices),
    // piece_nwide [nparts] the number of wide slices, which lead each
    // partition's residual slices, pieces [3*n_pieces] = (slice, first step,
    // end step)
    std::vector<int32_t> piece_start, piece_nwide, pieces;
    int32_t n_pieces = 0;
    int64_t ell_slots = 0, er_slots = 0;
    int64_t nnz_ell = 0, nnz_er = 0, n_er_rows = 0, nnz_halo = 0;
    int32_t n_er_wide = 0;                // residual slices processed by all 64 lanes
    int32_t max_halo = 0;
    double t_graph = 0, t_partition = 0, t_reorder = 0, t_encode = 0;
    int32_t n_rhs = 1;             // right-hand sides the LDS budget is sized for
    int32_t launch_waves = 0;      // 0 = automatic launch shape
    int32_t load_mode = 0;         // ehyb_load_mode of ehyb_spmv
    // device binding (non-owning)
    void* dev_blob = nullptr;
    size_t dev_bytes = 0;
    ehyb::BlobLayout layout;
};

// A batch of plans for ehyb_spmm_batched (host side).
struct ehyb_batch {
    std::vector<const ehyb_plan*> plans;
    int32_t n_rhs = 1, value_dtype = EHYB_F64, L = 1;
    std::vector<int32_t> items;      // (matrix, partition) pairs, by matrix, then partition
    std::vector<int32_t> range;      // [9] items of each XCD's queue
    std::vector<int32_t> pitems;     // (matrix, residual slice, first step, end step) of every piece
    std::vector<int64_t> pbase;      // [n_plans + 1] first piece of each matrix
    size_t off_desc = 0, off_items = 0, off_counters = 0, off_pitems = 0, off_part = 0, total = 0;
    void* dev_blob = nullptr;
    int64_t lds_bytes = 0;           // dynamic LDS of one workgroup
    int64_t algorithmic_bytes = 0;   // sum over matrices, n_rhs-wide x and y
    int32_t load_mode = 0;           // ehyb_load_mode of ehyb_spmm_batched
};

namespace ehyb {
// Set the thread-local error message and return the status.
ehyb_status fail(ehyb_status st, const std::string& msg);
ehyb_status ok();
BlobLayout compute_layout(const ehyb_plan& p);
int64_t algorithmic_bytes(const ehyb_plan& p);
int64_t lds_bytes_used(const ehyb_plan& p, int n_rhs = 1);
}  // namespace ehyb
