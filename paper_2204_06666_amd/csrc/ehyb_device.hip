// Device side of the EHYB library for gfx950 (CDNA4, wave64): the EHYB SpMV
// kernel, the plain CSR baseline, bandwidth probes and vector permutations,
// plus the C-ABI entry points that upload plans and launch kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>

#include "internal.h"

using namespace ehyb;

// Scalar buffer loads (s_buffer_load) of 8 and 16 bytes: LLVM intrinsics
// without a clang builtin, declared by their intrinsic names.
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
__device__ i32x2 llvm_s_buffer_load_x2(i32x4 rsrc, int32_t offset, int32_t policy) __asm("llvm.amdgcn.s.buffer.load.v2i32");
__device__ i32x4 llvm_s_buffer_load_x4(i32x4 rsrc, int32_t offset, int32_t policy) __asm("llvm.amdgcn.s.buffer.load.v4i32");

namespace {

constexpr int kXcds = 8;  // MI355X: workgroups are dealt round-robin to 8 XCDs

// The dispatcher hands workgroup b to XCD (b mod 8).  Renumber so that each
// XCD receives a contiguous range of logical ids: the workgroups of one
// partition, and neighbouring partitions, then share one XCD's L2.
__device__ __forceinline__ int xcd_logical_id(int b, int nblocks) {
    const int xcd = b % kXcds, idx = b / kXcds;
    const int q = nblocks / kXcds, r = nblocks % kXcds;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Device arrays of one plan (one matrix).
struct PartArrays {
    const int32_t* part_start;      // [nparts+1] first permuted row of each partition
    const int32_t* slice_start;     // [nparts+1] first ELL row-slice of each partition
    const int32_t* er_slice_start;  // [nparts+1] first residual row-slice of each partition
    const int32_t* ell_free;        // [nparts] leading ELL slices without residual rows
    const int32_t* halo_start;      // [nparts+1]
    const int32_t* halo_idx;        // cached neighbour x entries (permuted indices)
    const uint4* ell_meta;          // slot offset, width | index << 16, residual-row mask (lo, hi)
    const uint2* er_meta;           // slot offset, steps
    const uint16_t* er_row;         // local row of each residual slice row, 0xFFFF = none
    // Wide residual slices summed beforehand (ehyb_spmv, one right-hand side):
    // slice e's pieces are er_piece[e] .. er_piece[e+1]-1, their sums in
    // er_part; the first er_nwide[p] residual slices of partition p are the
    // wide ones.  Null: every slice is summed by its partition's workgroup.
    const int32_t* er_piece;
    const int32_t* er_nwide;
    const void* er_part;
    const void* ell_val;            // value type of the plan
    const uint16_t* ell_col;
    const void* er_val;
    const int32_t* er_col;
    int32_t lds_rows;               // LDS rows before the residual accumulators
    int32_t n;                      // rows
};

PartArrays part_arrays(const ehyb_plan& P) {
    const char* blob = (const char*)P.dev_blob;
    const BlobLayout& Ly = P.layout;
    PartArrays a;
    a.part_start = (const int32_t*)(blob + Ly.part_start);
    a.slice_start = (const int32_t*)(blob + Ly.slice_start);
    a.er_slice_start = (const int32_t*)(blob + Ly.er_slice_start);
    a.ell_free = (const int32_t*)(blob + Ly.ell_free);
    a.halo_start = (const int32_t*)(blob + Ly.halo_start);
    a.halo_idx = (const int32_t*)(blob + Ly.halo_idx);
    a.ell_meta = (const uint4*)(blob + Ly.ell_meta);
    a.er_meta = (const uint2*)(blob + Ly.er_meta);
    a.er_row = (const uint16_t*)(blob + Ly.er_row);
    a.ell_val = blob + Ly.ell_val;
    a.ell_col = (const uint16_t*)(blob + Ly.ell_col);
    a.er_val = blob + Ly.er_val;
    a.er_col = (const int32_t*)(blob + Ly.er_col);
    a.lds_rows = P.max_part_rows + P.max_halo;
    a.n = (int32_t)P.n;
    a.er_piece = nullptr;
    a.er_nwide = nullptr;
    a.er_part = nullptr;
    return a;
}

struct SpmvArgs {
    PartArrays m;
    const void* x;                  // permuted order, x type of the plan
    void* y;                        // permuted order
};

// The batched product's work queue is split in one queue per XCD: queue k
// hands out the items [range[k], range[k+1]) in order, and its counter sits
// on a cache line of its own.
constexpr int kCtrStride = 32;  // ints between two queue counters (128 bytes)

struct BatchArgs {
    const PartArrays* mats;         // [n_mats]
    const int2* items;              // (matrix, partition), by matrix, then partition
    int32_t n_items;
    int32_t range[kXcds + 1];       // items of each XCD's queue
    int32_t* counters;              // [k * kCtrStride] next item of queue k; [kXcds * kCtrStride] workgroups finished
    const void* X[EHYB_BATCH_MAX];  // row-major [n_i][NRHS], permuted order
    void* Y[EHYB_BATCH_MAX];
};

constexpr int kErChunk = 16;    // residual steps whose loads are issued before any is used
constexpr int kPieceLoads = 8;  // pieces of a wide slice each lane loads per round
constexpr int kStageRegs = 4;   // x-slice rows per thread kept in flight
constexpr int kHaloRegs = 4;    // halo gathers per thread kept in flight

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// Per value type: storage (V), x and accumulator types (X, A), ELL entries
// per lane per step (KC: 16 bytes of values), the per-step value and column
// loads (VL, CL), how many steps are loaded before use (kEll), and the
// unpacking of one step into KC (value, local column) pairs.
template <int DT> struct Prec;

template <> struct Prec<EHYB_F64> {
    using V = double;
    using X = double;
    using A = double;
    using VL = double2;
    using CL = uint32_t;
    static constexpr int KC = 2;
    static constexpr int kEll = 16;
    __device__ static __forceinline__ void unpack(const VL& v, CL c, A (&val)[KC], uint32_t (&col)[KC]) {
        val[0] = v.x; val[1] = v.y;
        col[0] = c & 0xFFFFu; col[1] = c >> 16;
    }
    __device__ static __forceinline__ A value(V v) { return v; }
};

template <> struct Prec<EHYB_F32> {
    using V = float;
    using X = float;
    using A = float;
    using VL = float4;
    using CL = uint2;
    static constexpr int KC = 4;
    static constexpr int kEll = 16;
    __device__ static __forceinline__ void unpack(const VL& v, CL c, A (&val)[KC], uint32_t (&col)[KC]) {
        val[0] = v.x; val[1] = v.y; val[2] = v.z; val[3] = v.w;
        col[0] = c.x & 0xFFFFu; col[1] = c.x >> 16; col[2] = c.y & 0xFFFFu; col[3] = c.y >> 16;
    }
    __device__ static __forceinline__ A value(V v) { return v; }
};

template <> struct Prec<EHYB_BF16> {
    using V = uint16_t;  // bfloat16 bits
    using X = float;
    using A = float;
    using VL = uint4;    // eight bfloat16 values
    using CL = uint4;    // eight 16-bit columns
    static constexpr int KC = 8;
    static constexpr int kEll = 8;
    __device__ static __forceinline__ void unpack(const VL& v, CL c, A (&val)[KC], uint32_t (&col)[KC]) {
        val[0] = bf16_lo(v.x); val[1] = bf16_hi(v.x); val[2] = bf16_lo(v.y); val[3] = bf16_hi(v.y);
        val[4] = bf16_lo(v.z); val[5] = bf16_hi(v.z); val[6] = bf16_lo(v.w); val[7] = bf16_hi(v.w);
        col[0] = c.x & 0xFFFFu; col[1] = c.x >> 16; col[2] = c.y & 0xFFFFu; col[3] = c.y >> 16;
        col[4] = c.z & 0xFFFFu; col[5] = c.z >> 16; col[6] = c.w & 0xFFFFu; col[7] = c.w >> 16;
    }
    __device__ static __forceinline__ A value(V v) { return __uint_as_float((uint32_t)v << 16); }
};

// binary32 or bfloat16 values and binary32 x with binary64 accumulation:
// the stored values widen exactly, every product and sum is FP64, and y is
// rounded to binary32 once.
template <int BASE> struct PrecAcc64 : Prec<BASE> {
    using B = Prec<BASE>;
    using A = double;
    __device__ static __forceinline__ void unpack(const typename B::VL& v, typename B::CL c, A (&val)[B::KC],
                                                  uint32_t (&col)[B::KC]) {
        float f[B::KC];
        B::unpack(v, c, f, col);
#pragma unroll
        for (int k = 0; k < B::KC; ++k) val[k] = (double)f[k];
    }
    __device__ static __forceinline__ A value(typename B::V v) { return (double)B::value(v); }
};
template <> struct Prec<EHYB_F32_ACC64> : PrecAcc64<EHYB_F32> {};
template <> struct Prec<EHYB_BF16_ACC64> : PrecAcc64<EHYB_BF16> {};

// NRHS consecutive elements (one row of a row-major multi-vector).
template <class T, int N> struct Row {
    typedef T type __attribute__((ext_vector_type(N)));
};
template <class T> struct Row<T, 1> {
    typedef T type;
};
template <class T, int N>
__device__ __forceinline__ T lane_of(const typename Row<T, N>::type& r, int k) {
    if constexpr (N == 1) return r;
    else return r[k];
}

// Load of data read exactly once per product (the value and column streams):
// a non-temporal load, which on gfx950 sustains about 9% more read bandwidth
// than a plain load (measured 7.1 vs 6.5 TB/s on a streaming probe) and does
// not displace reused lines (x, halo) from the caches.
template <class T>
__device__ __forceinline__ T stream_load(const T* p) {
    typedef uint32_t u32v4 __attribute__((ext_vector_type(4)));
    typedef uint32_t u32v2 __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(T) == 16) {
        return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const u32v4*>(p)));
    } else if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const u32v2*>(p)));
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p)));
    } else {
        static_assert(sizeof(T) == 2, "stream_load: 2, 4, 8 or 16 bytes");
        return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p)));
    }
}

template <bool NT, class T>
__device__ __forceinline__ T ld(const T* p) {
    if constexpr (NT) return stream_load(p);
    else return *p;
}

template <int L, class T>
__device__ __forceinline__ T reduce_lanes(T v) {
    if constexpr (L > 1) {
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    }
    return v;
}

// Raw buffer view of `bytes` bytes at p (stride 0, no swizzle): a load at
// byte offset `off` reads p[off..], and one at or past `bytes` reads zeros
// without touching memory.  x, the halo index lists and the residual columns
// are read through such views, with 32-bit offsets; the library rejects
// vectors of 4 GiB or more.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kBufferConfig = 0x00020000;  // gfx9 buffer descriptor word 3: 32-bit data format
__device__ __forceinline__ Rsrc make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kBufferConfig);
}
// The address is the view's base + `off` (per lane) + `soff` (the same for
// the wavefront, kept in a scalar register).  aux = 2 sets the non-temporal
// bit (as __builtin_nontemporal_load does).
template <class T, bool NT = false>
__device__ __forceinline__ T buf_load(Rsrc r, uint32_t off, uint32_t soff = 0) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    constexpr int aux = NT ? 2 : 0;
    if constexpr (sizeof(T) == 2) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, aux));
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, aux));
    } else if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, aux));
    } else {
        static_assert(sizeof(T) % 16 == 0, "buf_load: 2, 4, 8 or a multiple of 16 bytes");
        struct W {
            u32x4 w[sizeof(T) / 16];
        } v;
#pragma unroll
        for (int k = 0; k < (int)(sizeof(T) / 16); ++k)
            v.w[k] = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u * k, soff, aux);
        return __builtin_bit_cast(T, v);
    }
}

// Scalar buffer loads of the per-slice metadata, which is the same for the whole wavefront: the load goes
// through the scalar data cache into scalar registers, and the wavefront waits
// for it on the scalar counter alone.  A vector load of the same data is
// waited for on the vector counter, which also counts the wavefront's y
// stores, so every slice would wait for its own y store to complete.  The
// view is range-checked like a vector buffer view: an offset at or past its
// end reads zeros.
__device__ __forceinline__ i32x4 scalar_rsrc(const void* p, uint32_t bytes) {
    const uint64_t a = (uint64_t)(uintptr_t)p;
    i32x4 r;
    r.x = (int32_t)(uint32_t)a;
    r.y = (int32_t)((uint32_t)(a >> 32) & 0xFFFFu);  // stride 0
    r.z = (int32_t)bytes;
    r.w = kBufferConfig;
    return r;
}
__device__ __forceinline__ uint4 sload4(i32x4 rsrc, uint32_t off) {
    const i32x4 v = llvm_s_buffer_load_x4(rsrc, (int32_t)off, 0);
    return make_uint4((uint32_t)v.x, (uint32_t)v.y, (uint32_t)v.z, (uint32_t)v.w);
}
__device__ __forceinline__ uint2 sload2(i32x4 rsrc, uint32_t off) {
    const i32x2 v = llvm_s_buffer_load_x2(rsrc, (int32_t)off, 0);
    return make_uint2((uint32_t)v.x, (uint32_t)v.y);
}

// Metadata is the same for the whole wavefront: keep it in scalar registers.
__device__ __forceinline__ uint4 uniform4(uint4 v) {
    return make_uint4(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y),
                      __builtin_amdgcn_readfirstlane(v.z), __builtin_amdgcn_readfirstlane(v.w));
}

__device__ __forceinline__ int wave_fetch_add(int* ctr, int lane) {
    int v = 0;
    if (lane == 0) v = atomicAdd(ctr, 1);
    return __builtin_amdgcn_readfirstlane(v);
}

// Release this wave's LDS writes, then count it in `ctr` (`n` times).
__device__ __forceinline__ void wave_signal_n(int* ctr, int lane, int n) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) atomicAdd(ctr, n);
}
__device__ __forceinline__ void wave_signal(int* ctr, int lane) { wave_signal_n(ctr, lane, 1); }

// Wait (sleeping) until `ctr` reaches `target`, then acquire the LDS writes
// released before each increment.  Every increment is made by a wavefront of
// this workgroup that waits on nothing before making it, so the wait ends.
__device__ __forceinline__ void wave_wait(int* ctr, int target) {
    while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(ctr, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP)) < target)
        __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The loads of one round of an ELL slice: up to N full steps (KC entries per
// lane each) and, in the slice's last round, its single-entry tail steps, all
// issued before any is used.
template <int DT, int N>
struct EllRound {
    static constexpr int kSteps = N;
    typename Prec<DT>::VL v[N];
    typename Prec<DT>::CL c[N];
    typename Prec<DT>::V tv[Prec<DT>::KC - 1];
    uint16_t tc[Prec<DT>::KC - 1];
};

// Counters of the two workgroup queues of one partition.
struct Queues {
    int q_er, q_ell, n_staged, n_er_done;
};

// One partition of one matrix, processed by one workgroup (Alg. 3); its
// wavefronts pull work from two workgroup queues (the balancing of Alg. 3):
//  1. the workgroup loads the partition's x-slice into LDS (the cached vector
//     of Alg. 3) followed by its halo, the x entries of other partitions that
//     the partition's ELL entries reference;
//  2. residual queue: a wavefront takes a residual row-slice, loads all its
//     columns and values (up to kErChunk steps at once), gathers x from
//     device memory for all of them, and leaves each row's sums in LDS
//     accumulators (each residual row belongs to one lane group: plain
//     store), then counts the slice.  A residual row too long for its lane
//     group has a wide slice of its own, which all 64 lanes take and reduce
//     (so a hub row of a power-law matrix is not left to L lanes).  The next
//     slice's metadata is fetched while the current one is processed;
//  3. ELL queue (slices without residual rows first): a wavefront takes a
//     row-slice, issues all its loads (up to kEll steps of 16 bytes of values
//     and KC columns per lane) before using any, then the slice's last
//     entries (fewer than KC per lane, one value and column per step),
//     multiply-adds against the LDS vector (x-slice and halo) and stores y
//     once.  A slice with residual
//     rows first waits until the residual queue is drained, then adds the
//     residual sums.
// Wavefronts that leave the residual queue early stream ELL slices while
// others still gather, so the latency-bound residual work overlaps the
// streaming.  With NRHS right-hand sides, x, y and the LDS vector are
// row-major [row][NRHS] and every entry updates NRHS sums.  The sum of a row
// is (ELL entries in column order) + (residual entries in column order),
// fixed by the plan: results are bitwise reproducible.
// The caller initialises nothing and must not touch LDS or `Q` until every
// thread has returned (a barrier).
template <int DT, int L, int NRHS, bool NT, bool PREFETCH = false>
__device__ __forceinline__ void process_partition(const PartArrays& a, int p,
                                                  const typename Prec<DT>::X* __restrict__ x,
                                                  typename Prec<DT>::X* __restrict__ y,
                                                  unsigned char* lds_raw, Queues& Q) {
    using P = Prec<DT>;
    using V = typename P::V;
    using X = typename P::X;
    using Acc = typename P::A;
    using VL = typename P::VL;
    using CL = typename P::CL;
    using XR = typename Row<X, NRHS>::type;
    constexpr int KC = P::KC;
    constexpr int kEll = NRHS >= 4 ? (P::kEll > 8 ? P::kEll / 2 : 4) : P::kEll;
    // Steps of each wavefront's first slice loaded during the staging, whose
    // registers are live at the same time: a whole round for FP64 products
    // of one workgroup per partition (PREFETCH), none otherwise.  The other
    // value types need more registers per step, and the batched kernel runs
    // several workgroups per CU, so that one's staging overlaps another's
    // streaming anyway.
    constexpr int kPre = (PREFETCH && NRHS == 1 && DT == EHYB_F64) ? kEll : 0;
    // residual gathers in flight: whole rows of NRHS elements, about 16 registers' worth each way
    constexpr int kEr = NRHS == 1 ? kErChunk : (sizeof(X) * NRHS >= 32 ? 4 : 8);
    constexpr int XV = 16 / (int)sizeof(X);  // x elements per 16-byte load
    constexpr int C = kWave / L;
    X* xs = reinterpret_cast<X*>(lds_raw);
    // residual accumulators after the x-slice and halo, aligned to their size
    const size_t yer_off = ((size_t)a.lds_rows * NRHS * sizeof(X) + sizeof(Acc) - 1) / sizeof(Acc) * sizeof(Acc);
    Acc* yer = reinterpret_cast<Acc*>(lds_raw + yer_off);
    const int ps = a.part_start[p];
    const int sz = a.part_start[p + 1] - ps;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & (kWave - 1);
    const int nwaves = nthr >> 6;
    const int r = lane / L;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s0 = a.slice_start[p];
    const int ns = a.slice_start[p + 1] - s0;
    // Wavefront w's first ELL slice is slice w when that slice has no residual
    // rows (the leading ell_free[p] slices): its loads are issued during the
    // staging below, so that they stream while the staging round trips and
    // the barrier are waited for.  The ELL queue starts after those slices.
    const int nfirst = kPre > 0 ? min(min(nwaves, a.ell_free[p]), ns) : 0;
    const int e0 = a.er_slice_start[p];
    const int ner = a.er_slice_start[p + 1] - e0;
    if (tid == 0) {
        Q.q_er = 0;
        Q.q_ell = nfirst;
        Q.n_staged = 0;
        Q.n_er_done = 0;
    }
    const V* ell_val = static_cast<const V*>(a.ell_val);
    const i32x4 r_ell_meta = scalar_rsrc(a.ell_meta + s0, (uint32_t)ns * 16u);

    using Round = EllRound<DT, kEll>;
    // Every load of a round is issued unconditionally through views of the
    // slice's full steps and (last round only) of its tail steps: a load past
    // a view's end reads 0 without a memory access, so no load sits under a
    // branch (whose untaken path would leave its registers undefined and keep
    // them live across the queue loop).
    auto ell_issue = [&](const uint4& mu, uint32_t t0, auto& R) {
        constexpr int N = std::remove_reference_t<decltype(R)>::kSteps;
        const uint32_t width = mu.y & 0xFFFFu;  // entries per lane
        const uint32_t steps = width / KC;      // steps of KC entries, then
        const uint32_t tail = width % KC;       // single-entry steps
        const Rsrc rv = make_rsrc(ell_val + mu.x, steps * (uint32_t)(kWave * sizeof(VL)));
        const Rsrc rc = make_rsrc(a.ell_col + mu.x, steps * (uint32_t)(kWave * sizeof(CL)));
        // the tail: one value and one column per lane per step, so that rows
        // are not padded to a multiple of KC
        const uint32_t tl = t0 + N >= steps ? tail : 0u;
        const size_t tb = (size_t)mu.x + (size_t)steps * kWave * KC;
        const Rsrc rtv = make_rsrc(ell_val + tb, tl * (uint32_t)(kWave * sizeof(V)));
        const Rsrc rtc = make_rsrc(a.ell_col + tb, tl * (uint32_t)(kWave * sizeof(uint16_t)));
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const uint32_t t = t0 + j;
            R.v[j] = buf_load<VL, NT>(rv, lane * (uint32_t)sizeof(VL), t * (uint32_t)(kWave * sizeof(VL)));
            R.c[j] = buf_load<CL, NT>(rc, lane * (uint32_t)sizeof(CL), t * (uint32_t)(kWave * sizeof(CL)));
        }
#pragma unroll
        for (int j = 0; j < KC - 1; ++j) {
            R.tv[j] = buf_load<V, NT>(rtv, lane * (uint32_t)sizeof(V), j * (uint32_t)(kWave * sizeof(V)));
            R.tc[j] = buf_load<uint16_t, NT>(rtc, lane * 2u, j * (uint32_t)(kWave * 2));
        }
    };
    // multiply-add one round against the LDS vector (x-slice and halo)
    auto ell_consume = [&](const uint4& mu, uint32_t t0, const auto& R, Acc (&acc)[NRHS]) {
        constexpr int N = std::remove_reference_t<decltype(R)>::kSteps;
        const XR* xsr = reinterpret_cast<const XR*>(xs);
        const uint32_t width = mu.y & 0xFFFFu;
        const uint32_t steps = width / KC;
        const uint32_t tail = width % KC;
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (t0 + j < steps) {
                Acc val[KC];
                uint32_t col[KC];
                P::unpack(R.v[j], R.c[j], val, col);
#pragma unroll
                for (int e = 0; e < KC; ++e) {
                    const XR xv = xsr[col[e]];
#pragma unroll
                    for (int k = 0; k < NRHS; ++k) acc[k] = fma(val[e], (Acc)lane_of<X, NRHS>(xv, k), acc[k]);
                }
            }
        if (t0 + N >= steps && tail != 0) {
#pragma unroll
            for (int j = 0; j < KC - 1; ++j)
                if (j < (int)tail) {
                    const Acc vv = P::value(R.tv[j]);
                    const XR xv = xsr[R.tc[j]];
#pragma unroll
                    for (int k = 0; k < NRHS; ++k) acc[k] = fma(vv, (Acc)lane_of<X, NRHS>(xv, k), acc[k]);
                }
        }
    };
    EllRound<DT, (kPre > 0 ? kPre : 1)> first;  // unused when kPre == 0
    uint4 m_first = make_uint4(0, 0, 0, 0);

    // 1. x-slice into LDS, then the halo
    {
        const int hs = a.halo_start[p];
        const int hn = a.halo_start[p + 1] - hs;
        XR* xsr = reinterpret_cast<XR*>(xs);
        // Two dependent round trips to device memory for slices and halos
        // that fit the registers: the halo index loads and the x-slice loads,
        // then (once the indices are in) the halo gathers, before any LDS
        // store.  Nothing here branches per lane: a load under a branch, or
        // one the compiler sinks into the branch of its store, is waited for
        // there, and the vector counter drains in order, so that wait would
        // also wait for every load issued before it (the first slice's
        // round, below).  Loads are buffer loads (32-bit offsets, no 64-bit
        // address arithmetic) at indices clamped to the last valid element,
        // and stores go to the same clamped indices: surplus lanes rewrite
        // the last element with its own value.
        const Rsrc r_xs = make_rsrc(x + (size_t)ps * NRHS, (uint32_t)sz * (uint32_t)sizeof(XR));
        const Rsrc r_hidx = make_rsrc(a.halo_idx + hs, (uint32_t)hn * 4u);
        const Rsrc r_x = make_rsrc(x, (uint32_t)((size_t)a.n * sizeof(XR)));
        const uint32_t sz_last = (uint32_t)max(sz - 1, 0);
        const uint32_t hn_last = (uint32_t)max(hn - 1, 0);
        // Without a halo the gathers re-read the slice's last element and
        // store it in its own place (the LDS may end right after the slice).
        const bool has_halo = hn > 0;
        const uint32_t own_last = (uint32_t)ps + sz_last;
        uint32_t hi[kHaloRegs];
#pragma unroll
        for (int j = 0; j < kHaloRegs; ++j)
            hi[j] = buf_load<uint32_t>(r_hidx, min((uint32_t)(tid + j * nthr), hn_last) * 4u);
        XR xv[kStageRegs];
#pragma unroll
        for (int j = 0; j < kStageRegs; ++j)
            xv[j] = buf_load<XR>(r_xs, min((uint32_t)(tid + j * nthr), sz_last) * (uint32_t)sizeof(XR));
        XR hv[kHaloRegs];
#pragma unroll
        for (int j = 0; j < kHaloRegs; ++j) hv[j] = buf_load<XR>(r_x, (has_halo ? hi[j] : own_last) * (uint32_t)sizeof(XR));
        // The first ELL slice's first round, after the gathers, so that
        // waiting for the gathers does not wait for it.  Issued by every
        // wavefront, without a branch: one without a first slice reads
        // metadata past the view's end (zeros: a slice of width 0, whose
        // loads read nothing from memory).
        if constexpr (kPre > 0) {
            m_first = sload4(r_ell_meta, wave < nfirst ? (uint32_t)wave * 16u : 0xFFFFFFF0u);
            ell_issue(m_first, 0, first);
        }
#pragma unroll
        for (int j = 0; j < kStageRegs; ++j) xsr[min((uint32_t)(tid + j * nthr), sz_last)] = xv[j];
#pragma unroll
        for (int j = 0; j < kHaloRegs; ++j)
            xsr[has_halo ? sz + min((uint32_t)(tid + j * nthr), hn_last) : sz_last] = hv[j];
        // Partitions or halos beyond that first pass (large LDS budgets, the
        // long halos of power-law matrices): the rest in chunks of kRest rows
        // per thread, each chunk's loads (index loads, then gathers) issued
        // before any of its stores, with the same clamping.
        constexpr int kRest = NRHS == 1 ? 8 : kHaloRegs;
        for (uint32_t b = (uint32_t)(kStageRegs * nthr); b < (uint32_t)sz; b += (uint32_t)(kRest * nthr)) {
            XR v2[kRest];
#pragma unroll
            for (int j = 0; j < kRest; ++j)
                v2[j] = buf_load<XR>(r_xs, min(b + (uint32_t)(tid + j * nthr), sz_last) * (uint32_t)sizeof(XR));
#pragma unroll
            for (int j = 0; j < kRest; ++j) xsr[min(b + (uint32_t)(tid + j * nthr), sz_last)] = v2[j];
        }
        for (uint32_t b = (uint32_t)(kHaloRegs * nthr); b < (uint32_t)hn; b += (uint32_t)(kRest * nthr)) {
            uint32_t h2[kRest];
#pragma unroll
            for (int j = 0; j < kRest; ++j)
                h2[j] = buf_load<uint32_t>(r_hidx, min(b + (uint32_t)(tid + j * nthr), hn_last) * 4u);
            XR v2[kRest];
#pragma unroll
            for (int j = 0; j < kRest; ++j) v2[j] = buf_load<XR>(r_x, h2[j] * (uint32_t)sizeof(XR));
#pragma unroll
            for (int j = 0; j < kRest; ++j) xsr[sz + min(b + (uint32_t)(tid + j * nthr), hn_last)] = v2[j];
        }
    }
    bool er_ready = ner == 0;
    // the rest of a slice after its first round, the residual sums of its
    // rows (waiting, if needed, until the residual queue is drained) and
    // one store of y per row
    auto ell_finish = [&](const uint4& mu, uint32_t t_done, Acc (&acc)[NRHS]) {
        const uint32_t steps = (mu.y & 0xFFFFu) / KC;
        for (uint32_t t0 = t_done; t0 < steps; t0 += kEll) {
            Round R;
            ell_issue(mu, t0, R);
            ell_consume(mu, t0, R, acc);
        }
#pragma unroll
        for (int k = 0; k < NRHS; ++k) acc[k] = reduce_lanes<L>(acc[k]);
        const uint64_t mask = ((uint64_t)mu.w << 32) | mu.z;
        if (mask != 0 && !er_ready) {
            wave_wait(&Q.n_er_done, ner);
            er_ready = true;
        }
        const int lr = (int)(mu.y >> 16) * C + r;
        if ((lane & (L - 1)) == 0 && lr < sz) {
            if ((mask >> r) & 1u) {
#pragma unroll
                for (int k = 0; k < NRHS; ++k) acc[k] += yer[(size_t)lr * NRHS + k];
            }
            if constexpr (NRHS == 1) {
                y[ps + lr] = (X)acc[0];
            } else {
                XR out;
#pragma unroll
                for (int k = 0; k < NRHS; ++k) out[k] = (X)acc[k];
                reinterpret_cast<XR*>(y)[ps + lr] = out;
            }
        }
    };
    __syncthreads();  // counters initialised, x-slice and halo in LDS

    // the prefetched first slice (it has no residual rows: nothing to wait for)
    if (wave < nfirst) {
        Acc acc[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) acc[k] = 0;
        ell_consume(m_first, 0, first, acc);
        ell_finish(m_first, kPre, acc);
    }

    // 2. residual queue.  When the wide slices (which lead the partition's
    // residual slices) were summed beforehand in pieces, their items are
    // groups of 64 slices, one per lane, each lane adding its slice's pieces
    // in piece order; the other items are single slices.
    {
        const V* er_val = static_cast<const V*>(a.er_val);
        const Rsrc r_xg = make_rsrc(x, (uint32_t)((size_t)a.n * sizeof(XR)));
        const i32x4 r_meta = scalar_rsrc(a.er_meta + e0, (uint32_t)ner * 8u);
        const int nw = a.er_piece != nullptr ? a.er_nwide[p] : 0;
        const int ngr = (nw + kWave - 1) / kWave;
        const int nitems = ngr + ner - nw;
        // residual slice of item i >= ngr (clamped below for group items, whose metadata is not used)
        auto slice_of = [&](int i) { return (uint32_t)max(i - ngr + nw, 0); };
        int it = wave_fetch_add(&Q.q_er, lane);
        uint2 m = sload2(r_meta, slice_of(it) * 8u);
        while (it < nitems) {
            const int itn = wave_fetch_add(&Q.q_er, lane);
            const uint2 mn = sload2(r_meta, slice_of(itn) * 8u);
            if (it < ngr) {
                // pieces loaded per round: kPieceLoads, fewer when each is
                // a row of NRHS sums, to stay within about 32 registers
                constexpr int kPR = 128 / (NRHS * (int)sizeof(Acc));
                constexpr int kPL = NRHS == 1 || kPR > kPieceLoads ? kPieceLoads : (kPR > 1 ? kPR : 1);
                const int k = it * kWave + lane;  // this lane's wide slice
                const int e = e0 + min(k, nw - 1);
                const int q0 = a.er_piece[e];
                const int nq = a.er_piece[e + 1] - q0;  // at least 1
                const uint16_t lw = a.er_row[(size_t)e * C];
                const Acc* part = static_cast<const Acc*>(a.er_part) + (size_t)q0 * NRHS;
                Acc sum[NRHS];
#pragma unroll
                for (int kk = 0; kk < NRHS; ++kk) sum[kk] = 0;
                // all lanes load kPL pieces per round (clamped to their last
                // piece), so the loads are issued together
                for (int j0 = 0; __builtin_amdgcn_ballot_w64(j0 < nq) != 0; j0 += kPL) {
                    Acc pv[kPL][NRHS];
#pragma unroll
                    for (int u = 0; u < kPL; ++u)
#pragma unroll
                        for (int kk = 0; kk < NRHS; ++kk) pv[u][kk] = part[(size_t)min(j0 + u, nq - 1) * NRHS + kk];
#pragma unroll
                    for (int u = 0; u < kPL; ++u)
                        if (j0 + u < nq) {
#pragma unroll
                            for (int kk = 0; kk < NRHS; ++kk) sum[kk] += pv[u][kk];
                        }
                }
                if (k < nw && lw != 0xFFFF) {
#pragma unroll
                    for (int kk = 0; kk < NRHS; ++kk) yer[(size_t)lw * NRHS + kk] = sum[kk];
                }
                wave_signal_n(&Q.n_er_done, lane, min(kWave, nw - it * kWave));
                it = itn;
                m = mn;
                continue;
            }
            const int es = (int)slice_of(it);
            const uint32_t off = __builtin_amdgcn_readfirstlane(m.x);
            const uint32_t my = __builtin_amdgcn_readfirstlane(m.y);
            const uint32_t steps = my & ~kErWide;
            const bool wide = (my & kErWide) != 0;  // one long row on all 64 lanes
            const uint16_t lr = a.er_row[(size_t)(e0 + es) * C + (wide ? 0 : r)];
            Acc acc[NRHS];
#pragma unroll
            for (int k = 0; k < NRHS; ++k) acc[k] = 0;
            // Every load of a batch of kEr steps is issued unconditionally
            // (through views of the slice: a step past its end reads column
            // 0 and value 0 without a memory access, and gathers x[0]); only
            // the multiply-adds of real steps are guarded.  A load under a
            // branch is waited for at the branch's end, which would issue the
            // steps' gathers one round trip at a time.
            const Rsrc r_ec = make_rsrc(a.er_col + off, steps * (uint32_t)(kWave * sizeof(int32_t)));
            const Rsrc r_ev = make_rsrc(er_val + off, steps * (uint32_t)(kWave * sizeof(V)));
            for (uint32_t t0 = 0; t0 < steps; t0 += kEr) {
                int32_t c[kEr];
                V v[kEr];
                XR xg[kEr];
#pragma unroll
                for (int j = 0; j < kEr; ++j) {
                    c[j] = buf_load<int32_t, NT>(r_ec, lane * (uint32_t)sizeof(int32_t),
                                                 (t0 + j) * (uint32_t)(kWave * sizeof(int32_t)));
                    v[j] = buf_load<V, NT>(r_ev, lane * (uint32_t)sizeof(V), (t0 + j) * (uint32_t)(kWave * sizeof(V)));
                }
#pragma unroll
                for (int j = 0; j < kEr; ++j) xg[j] = buf_load<XR>(r_xg, (uint32_t)c[j] * (uint32_t)sizeof(XR));
#pragma unroll
                for (int j = 0; j < kEr; ++j)
                    if (t0 + j < steps) {
                        const Acc vv = P::value(v[j]);
#pragma unroll
                        for (int k = 0; k < NRHS; ++k) acc[k] = fma(vv, (Acc)lane_of<X, NRHS>(xg[j], k), acc[k]);
                    }
            }
            if (wide) {
#pragma unroll
                for (int k = 0; k < NRHS; ++k) acc[k] = reduce_lanes<kWave>(acc[k]);
            } else {
#pragma unroll
                for (int k = 0; k < NRHS; ++k) acc[k] = reduce_lanes<L>(acc[k]);
            }
            if ((wide ? lane == 0 : (lane & (L - 1)) == 0) && lr != 0xFFFF) {
#pragma unroll
                for (int k = 0; k < NRHS; ++k) yer[(size_t)lr * NRHS + k] = acc[k];
            }
            wave_signal(&Q.n_er_done, lane);
            it = itn;
            m = mn;
        }
    }

    // 3. ELL queue
    int item = wave_fetch_add(&Q.q_ell, lane);
    uint4 m = sload4(r_ell_meta, (uint32_t)item * 16u);
    while (item < ns) {
        const int nxt = wave_fetch_add(&Q.q_ell, lane);
        // the next slice's metadata travels while this slice streams
        const uint4 mn = sload4(r_ell_meta, (uint32_t)nxt * 16u);
        const uint4 mu = uniform4(m);
        Acc acc[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) acc[k] = 0;
        Round R;
        ell_issue(mu, 0, R);
        ell_consume(mu, 0, R, acc);
        ell_finish(mu, kEll, acc);
        item = nxt;
        m = mn;
    }
}

// y = A x: one workgroup per partition.
template <int DT, int L, bool NT>
__global__ void __launch_bounds__(1024) ehyb_spmv_kernel(SpmvArgs a) {
    using X = typename Prec<DT>::X;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Queues Q;
    const int p = xcd_logical_id(blockIdx.x, gridDim.x);
    process_partition<DT, L, 1, NT, true>(a.m, p, static_cast<const X*>(a.x), static_cast<X*>(a.y), lds_raw, Q);
}

// Y_i = A_i X_i for a batch: persistent workgroups take (matrix, partition)
// items from a queue (the global queue of Alg. 3, spread over matrices), first
// from their own XCD's queue, then, once it is empty, from the other XCDs'
// queues in turn.  Each XCD's queue holds a contiguous run of items in
// partition order: partitions numbered close together are neighbours (the
// partitioner bisects recursively), so the x rows one partition loads as its
// halo are mostly those its neighbours load as theirs or as their x-slice,
// on the same XCD at about the same time, and are found in that XCD's L2.
// The last workgroup to leave resets the counters, so the next launch (or
// graph replay) starts from zero.
template <int DT, int L, int NRHS, bool NT>
__global__ void __launch_bounds__(1024) ehyb_spmm_batched_kernel(BatchArgs args) {
    using X = typename Prec<DT>::X;
    // Read the argument block in place (it is the first and only kernel
    // argument): the per-matrix pointer tables are indexed at run time, which
    // on a by-value copy would go through private memory.
    const BatchArgs& a = *(const BatchArgs*)__builtin_amdgcn_kernarg_segment_ptr();
    (void)args;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Queues Q;
    __shared__ int s_item;
    int32_t* counters = a.counters;
    const int home = (int)(blockIdx.x % kXcds);
    int visited = 0;  // queues found empty so far (used by thread 0 only)
    for (;;) {
        if (threadIdx.x == 0) {
            int it = -1;
            while (visited < kXcds) {
                const int q = (home + visited) % kXcds;
                const int i = atomicAdd(&counters[q * kCtrStride], 1);
                if (i < a.range[q + 1] - a.range[q]) {
                    it = a.range[q] + i;
                    break;
                }
                ++visited;
            }
            s_item = it;
        }
        __syncthreads();
        const int it = s_item;
        if (it < 0) break;
        const int2 w = a.items[it];
        const int mi = __builtin_amdgcn_readfirstlane(w.x);
        const int pi = __builtin_amdgcn_readfirstlane(w.y);
        process_partition<DT, L, NRHS, NT>(a.mats[mi], pi, static_cast<const X*>(a.X[mi]),
                                       static_cast<X*>(a.Y[mi]), lds_raw, Q);
        __syncthreads();  // LDS, Q and s_item are reused by the next item
    }
    // Every workgroup has seen all queues empty before it counts itself
    // here, and waited for the result of each of its queue increments.
    if (threadIdx.x == 0 && atomicAdd(&counters[kXcds * kCtrStride], 1) == (int)gridDim.x - 1) {
        for (int q = 0; q <= kXcds; ++q)
            __hip_atomic_store(&counters[q * kCtrStride], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The wide residual slices, summed before the product over the whole device:
// one wavefront per piece of at most kPieceSteps steps.  Entry k of a wide
// slice is at slot off + k, so piece (e, t0, t1) holds slots off + 64*t0 ..
// off + 64*t1 - 1, one per lane per step; each lane sums its entries in step
// order, then the wavefront adds its lanes in a fixed tree.  The partition's
// workgroup adds the pieces of its row in a fixed order, so results do not
// depend on timing.  All loads are issued unconditionally through views of
// the piece (steps past its end read column 0 and value 0 without a memory
// access, and gather x[0]), so that the gathers are in flight together; only
// the multiply-adds of real steps are guarded.  With NRHS right-hand sides
// each gather is a row of NRHS elements and lane 0 writes NRHS sums.
template <int DT, int NRHS, bool NT>
__device__ __forceinline__ void piece_sum(const uint2* __restrict__ er_meta, const void* __restrict__ er_val_,
                                          const int32_t* __restrict__ er_col, int e, int t0, int t1,
                                          const void* __restrict__ x, uint32_t x_bytes, void* __restrict__ out) {
    using P = Prec<DT>;
    using V = typename P::V;
    using X = typename P::X;
    using Acc = typename P::A;
    using XR = typename Row<X, NRHS>::type;
    // steps whose gathers are in flight together: the whole piece, or half
    // of it when each gather is a row of 32 bytes or more (fewer registers,
    // so more wavefronts per SIMD: 1.5% faster for FP32 x 8)
    constexpr int kPS = sizeof(XR) >= 32 ? kPieceSteps / 2 : kPieceSteps;
    const V* er_val = static_cast<const V*>(er_val_);
    const int lane = threadIdx.x & (kWave - 1);
    const size_t base = (size_t)__builtin_amdgcn_readfirstlane(er_meta[e].x) + (size_t)t0 * kWave;
    const uint32_t nst = (uint32_t)(t1 - t0);
    const Rsrc rc = make_rsrc(er_col + base, nst * (uint32_t)(kWave * sizeof(int32_t)));
    const Rsrc rv = make_rsrc(er_val + base, nst * (uint32_t)(kWave * sizeof(V)));
    const Rsrc rx = make_rsrc(x, x_bytes);
    Acc acc[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) acc[k] = 0;
#pragma unroll
    for (int s0 = 0; s0 < kPieceSteps; s0 += kPS) {
        int32_t c[kPS];
        V v[kPS];
#pragma unroll
        for (int j = 0; j < kPS; ++j) {
            c[j] = buf_load<int32_t, NT>(rc, lane * (uint32_t)sizeof(int32_t),
                                         (uint32_t)(s0 + j) * (uint32_t)(kWave * sizeof(int32_t)));
            v[j] = buf_load<V, NT>(rv, lane * (uint32_t)sizeof(V), (uint32_t)(s0 + j) * (uint32_t)(kWave * sizeof(V)));
        }
        XR xg[kPS];
#pragma unroll
        for (int j = 0; j < kPS; ++j) xg[j] = buf_load<XR>(rx, (uint32_t)c[j] * (uint32_t)sizeof(XR));
#pragma unroll
        for (int j = 0; j < kPS; ++j)
            if (t0 + s0 + j < t1) {
                const Acc vv = P::value(v[j]);
#pragma unroll
                for (int k = 0; k < NRHS; ++k) acc[k] = fma(vv, (Acc)lane_of<X, NRHS>(xg[j], k), acc[k]);
            }
    }
#pragma unroll
    for (int k = 0; k < NRHS; ++k) acc[k] = reduce_lanes<kWave>(acc[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NRHS; ++k) static_cast<Acc*>(out)[k] = acc[k];
    }
}

// ehyb_spmv: the pieces of one plan, sums in piece order.  One wavefront
// per workgroup: on a power-law graph the product was 1.4% faster than
// with four per workgroup, and 4% slower with sixteen.
template <int DT, bool NT>
__global__ void __launch_bounds__(64) er_pieces_kernel(const uint2* __restrict__ er_meta,
                                                        const void* __restrict__ er_val,
                                                        const int32_t* __restrict__ er_col,
                                                        const int32_t* __restrict__ pieces, int n_pieces,
                                                        const void* __restrict__ x, uint32_t x_bytes,
                                                        void* __restrict__ part) {
    using Acc = typename Prec<DT>::A;
    const int q = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    if (q >= n_pieces) return;
    const int e = __builtin_amdgcn_readfirstlane(pieces[3 * (size_t)q]);
    const int t0 = __builtin_amdgcn_readfirstlane(pieces[3 * (size_t)q + 1]);
    const int t1 = __builtin_amdgcn_readfirstlane(pieces[3 * (size_t)q + 2]);
    piece_sum<DT, 1, NT>(er_meta, er_val, er_col, e, t0, t1, x, x_bytes, static_cast<Acc*>(part) + q);
}

// ehyb_spmm_batched: the pieces of every matrix of the batch in one launch.
struct BatchPieceArgs {
    const PartArrays* mats;         // [n_mats]
    const int4* items;              // (matrix, residual slice, first step, end step), by matrix, then piece
    int32_t n_items;
    void* part;                     // [n_items][NRHS] sums, item order
    const void* X[EHYB_BATCH_MAX];  // row-major [n_i][NRHS], permuted order
};

template <int DT, int NRHS, bool NT>
__global__ void __launch_bounds__(256) er_pieces_batched_kernel(BatchPieceArgs args) {
    using X = typename Prec<DT>::X;
    using Acc = typename Prec<DT>::A;
    // read in place: X is indexed at run time (see ehyb_spmm_batched_kernel)
    const BatchPieceArgs& a = *(const BatchPieceArgs*)__builtin_amdgcn_kernarg_segment_ptr();
    (void)args;
    const int q = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    if (q >= a.n_items) return;
    const int4 w = a.items[q];
    const int mi = __builtin_amdgcn_readfirstlane(w.x);
    const PartArrays& m = a.mats[mi];
    const uint32_t xb = (uint32_t)((size_t)m.n * NRHS * sizeof(X));  // below 4 GiB: checked by ehyb_spmm_batched
    piece_sum<DT, NRHS, NT>(m.er_meta, m.er_val, m.er_col, __builtin_amdgcn_readfirstlane(w.y),
                            __builtin_amdgcn_readfirstlane(w.z), __builtin_amdgcn_readfirstlane(w.w), a.X[mi], xb,
                            static_cast<Acc*>(a.part) + (size_t)q * NRHS);
}

template <int DT>
void launch_pieces(const ehyb_plan& P, bool nt, const void* x, hipStream_t s) {
    const char* blob = (const char*)P.dev_blob;
    const BlobLayout& Ly = P.layout;
    const int nblocks = P.n_pieces;  // one wavefront per workgroup
    const uint2* meta = (const uint2*)(blob + Ly.er_meta);
    const int32_t* col = (const int32_t*)(blob + Ly.er_col);
    const int32_t* pc = (const int32_t*)(blob + Ly.pieces);
    void* part = (void*)(blob + Ly.ypart);
    const uint32_t xb = (uint32_t)((size_t)P.n * P.xbytes);  // below 4 GiB: checked by ehyb_spmv
    if (nt)
        hipLaunchKernelGGL((er_pieces_kernel<DT, true>), dim3(nblocks), dim3(64), 0, s, meta, blob + Ly.er_val, col, pc,
                           P.n_pieces, x, xb, part);
    else
        hipLaunchKernelGGL((er_pieces_kernel<DT, false>), dim3(nblocks), dim3(64), 0, s, meta, blob + Ly.er_val, col,
                           pc, P.n_pieces, x, xb, part);
}

template <int DT, int NRHS>
void launch_pieces_batched_r(bool nt, const BatchPieceArgs& a, hipStream_t s) {
    const int nblocks = (a.n_items + 3) / 4;  // four wavefronts per 256-thread workgroup
    if (nt)
        hipLaunchKernelGGL((er_pieces_batched_kernel<DT, NRHS, true>), dim3(nblocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((er_pieces_batched_kernel<DT, NRHS, false>), dim3(nblocks), dim3(256), 0, s, a);
}

template <int DT>
bool launch_pieces_batched(int nrhs, bool nt, const BatchPieceArgs& a, hipStream_t s) {
    switch (nrhs) {
        case 1: launch_pieces_batched_r<DT, 1>(nt, a, s); return true;
        case 2: launch_pieces_batched_r<DT, 2>(nt, a, s); return true;
        case 4: launch_pieces_batched_r<DT, 4>(nt, a, s); return true;
        case 8: launch_pieces_batched_r<DT, 8>(nt, a, s); return true;
        default: return false;
    }
}

// Plain CSR SpMV, the comparator (CSR-vector): L lanes per row, rows of a
// wavefront consecutive.  Each lane takes kCsrU entries per batch, L apart,
// and issues all their column, value and x loads before using any (through
// range-checked buffer views, so that no load sits under a branch); lanes
// past the row's end gather x[0] and add nothing.  A wavefront that holds a
// row longer than kCsrLong entries instead sums its rows one at a time on
// all 64 lanes, so that a hub row is not left to L lanes.  The sum of a row
// is a fixed function of L: results are reproducible.
constexpr int kCsrU = 4;
constexpr int kCsrLong = 1024;

__device__ __forceinline__ double csr_batch_sum(Rsrc rc, Rsrc rv, Rsrc rx, int32_t b, int32_t len, int32_t t,
                                                int sub, int stride, double acc) {
    int32_t c[kCsrU];
    double v[kCsrU];
    double xg[kCsrU];
#pragma unroll
    for (int k = 0; k < kCsrU; ++k) {
        const uint32_t q = (uint32_t)(b + t + sub + stride * k);
        c[k] = buf_load<int32_t>(rc, q * 4u);
        v[k] = buf_load<double>(rv, q * 8u);
    }
#pragma unroll
    for (int k = 0; k < kCsrU; ++k) {
        const bool in = t + sub + stride * k < len;
        xg[k] = buf_load<double>(rx, in ? (uint32_t)c[k] * 8u : 0u);
    }
#pragma unroll
    for (int k = 0; k < kCsrU; ++k)
        if (t + sub + stride * k < len) acc = fma(v[k], xg[k], acc);
    return acc;
}

template <int L>
__global__ void __launch_bounds__(256) csr_spmv_f64_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const double* __restrict__ v,
                                                           const double* __restrict__ x,
                                                           double* __restrict__ y) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid / L;
    const int sub = (int)(gid & (L - 1));
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const Rsrc rc = make_rsrc(ci, (uint32_t)(nnz * 4));
    const Rsrc rv = make_rsrc(v, (uint32_t)(nnz * 8));
    const Rsrc rx = make_rsrc(x, (uint32_t)(n * 8));
    int32_t b = 0, len = 0;
    if (row < n) {
        b = rp[row];
        len = rp[row + 1] - b;
    }
    int mx = len;  // the wavefront's longest row
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, kWave));
    mx = __builtin_amdgcn_readfirstlane(mx);
    if (mx <= kCsrLong) {
        double acc = 0.0;
        for (int32_t t = 0; t < mx; t += L * kCsrU) acc = csr_batch_sum(rc, rv, rx, b, len, t, sub, L, acc);
        if constexpr (L > 1) {
#pragma unroll
            for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        }
        if (sub == 0 && row < n) y[row] = acc;
        return;
    }
    // one row at a time on the whole wavefront
    const int64_t row0 = (gid - lane) / L;
    for (int r = 0; r < kWave / L; ++r) {
        const int64_t rr = row0 + r;
        if (rr >= n) break;
        const int32_t br = __builtin_amdgcn_readfirstlane(rp[rr]);
        const int32_t lr = __builtin_amdgcn_readfirstlane(rp[rr + 1]) - br;
        double acc = 0.0;
        for (int32_t t = 0; t < lr; t += kWave * kCsrU) acc = csr_batch_sum(rc, rv, rx, br, lr, t, lane, kWave, acc);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) y[rr] = acc;
    }
}

// Read-stream probe: every byte of buf is loaded once with 16-byte
// non-temporal loads; one partial per workgroup keeps the loads alive.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Four independent 16-byte non-temporal loads per thread in flight, 512
// threads per workgroup: the best of the read-stream shapes measured on
// gfx950 (about 7.1 TB/s over a 2 GiB buffer).
// NT = false: ordinary loads, which allocate in L2 and the Infinity Cache;
// reading a buffer larger than both this way evicts what they held (the
// cache flush of cold timings).  Non-temporal loads do not displace it.
template <bool NT>
__global__ void __launch_bounds__(512) probe_read_kernel(const u32x4* __restrict__ buf, size_t n16,
                                                         uint64_t* __restrict__ sink) {
    uint32_t acc = 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 v0 = ld<NT>(buf + i);
        const u32x4 v1 = ld<NT>(buf + i + stride);
        const u32x4 v2 = ld<NT>(buf + i + 2 * stride);
        const u32x4 v3 = ld<NT>(buf + i + 3 * stride);
        acc ^= (v0.x ^ v0.y ^ v0.z ^ v0.w) ^ (v1.x ^ v1.y ^ v1.z ^ v1.w) ^ (v2.x ^ v2.y ^ v2.z ^ v2.w) ^
               (v3.x ^ v3.y ^ v3.z ^ v3.w);
    }
    for (; i < n16; i += stride) {
        const u32x4 v = ld<NT>(buf + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    // wave-level combine, then one store per workgroup
    for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, kWave);
    __shared__ uint32_t part[8];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t ^= part[w];
        sink[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(256) probe_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                         size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

template <class T>
__global__ void __launch_bounds__(256) gather_kernel(int64_t n, const int32_t* __restrict__ perm,
                                                     const T* __restrict__ x, T* __restrict__ xp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) xp[i] = x[perm[i]];
}

template <class T>
__global__ void __launch_bounds__(256) scatter_kernel(int64_t n, const int32_t* __restrict__ perm,
                                                      const T* __restrict__ yp, T* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[perm[i]] = yp[i];
}

ehyb_status launch_status(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(EHYB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return EHYB_OK;
}

// Wavefronts per workgroup: 16 (1024 threads) unless the plan sets another
// shape; never more wavefronts than the largest partition has ELL row-slices.
int launch_waves(const ehyb_plan& P) {
    if (P.launch_waves > 0) return P.launch_waves;
    const int64_t max_slices = (P.max_part_rows + P.C - 1) / P.C;
    if (max_slices <= 4) return 4;
    if (max_slices <= 8) return 8;
    return 16;
}

// Allow a kernel the full 160 KiB of gfx950 LDS as dynamic shared memory
// (HIP's default limit is 64 KiB), once per kernel and device.  Thread-safe;
// a failure is reported (EHYB_EDEVICE with HIP's message) and retried on the
// next launch.
template <class K>
ehyb_status raise_lds_limit(K* kernel, size_t lds) {
    if (lds <= 64 * 1024) return EHYB_OK;
    static std::atomic<uint64_t> done{0};  // one bit per device
    static std::mutex mu;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(EHYB_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return fail(EHYB_EUNSUPPORTED, "device index above 63");
    const uint64_t bit = 1ull << dev;
    if (done.load(std::memory_order_acquire) & bit) return EHYB_OK;
    std::lock_guard<std::mutex> lock(mu);
    if (done.load(std::memory_order_relaxed) & bit) return EHYB_OK;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024 - kStaticLds);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(EHYB_EDEVICE, std::string("raising the kernel's LDS limit to 160 KiB: ") + hipGetErrorString(e));
    }
    done.fetch_or(bit, std::memory_order_release);
    return EHYB_OK;
}

// The launchers return false when no kernel is instantiated for the
// requested shape, else true with the launch's status in `st`.
template <int DT, int L, bool NT>
ehyb_status launch_spmv(const SpmvArgs& a, int nblocks, int threads, size_t lds, hipStream_t s) {
    const ehyb_status st = raise_lds_limit(&ehyb_spmv_kernel<DT, L, NT>, lds);
    if (st != EHYB_OK) return st;
    hipLaunchKernelGGL((ehyb_spmv_kernel<DT, L, NT>), dim3(nblocks), dim3(threads), lds, s, a);
    return EHYB_OK;
}

template <int DT, bool NT>
bool launch_spmv_l(int L, const SpmvArgs& a, int nblocks, int threads, size_t lds, hipStream_t s, ehyb_status& st) {
    switch (L) {
        case 1: st = launch_spmv<DT, 1, NT>(a, nblocks, threads, lds, s); return true;
        case 2: st = launch_spmv<DT, 2, NT>(a, nblocks, threads, lds, s); return true;
        case 4: st = launch_spmv<DT, 4, NT>(a, nblocks, threads, lds, s); return true;
        case 8: st = launch_spmv<DT, 8, NT>(a, nblocks, threads, lds, s); return true;
        case 16: st = launch_spmv<DT, 16, NT>(a, nblocks, threads, lds, s); return true;
        case 32: st = launch_spmv<DT, 32, NT>(a, nblocks, threads, lds, s); return true;
        case 64: st = launch_spmv<DT, 64, NT>(a, nblocks, threads, lds, s); return true;
        default: return false;
    }
}

template <int DT>
bool launch_spmv_dt(int L, bool nt, const SpmvArgs& a, int nblocks, int threads, size_t lds, hipStream_t s,
                    ehyb_status& st) {
    return nt ? launch_spmv_l<DT, true>(L, a, nblocks, threads, lds, s, st)
              : launch_spmv_l<DT, false>(L, a, nblocks, threads, lds, s, st);
}

template <int DT, int L, int NRHS, bool NT>
ehyb_status launch_batched(const BatchArgs& a, int nblocks, int threads, size_t lds, hipStream_t s) {
    const ehyb_status st = raise_lds_limit(&ehyb_spmm_batched_kernel<DT, L, NRHS, NT>, lds);
    if (st != EHYB_OK) return st;
    hipLaunchKernelGGL((ehyb_spmm_batched_kernel<DT, L, NRHS, NT>), dim3(nblocks), dim3(threads), lds, s, a);
    return EHYB_OK;
}

template <int DT, int NRHS, bool NT>
bool launch_batched_l(int L, const BatchArgs& a, int nblocks, int threads, size_t lds, hipStream_t s,
                      ehyb_status& st) {
    switch (L) {
        case 1: st = launch_batched<DT, 1, NRHS, NT>(a, nblocks, threads, lds, s); return true;
        case 4: st = launch_batched<DT, 4, NRHS, NT>(a, nblocks, threads, lds, s); return true;
        case 16: st = launch_batched<DT, 16, NRHS, NT>(a, nblocks, threads, lds, s); return true;
        default: return false;
    }
}

template <int DT, bool NT>
bool launch_batched_r(int L, int nrhs, const BatchArgs& a, int nblocks, int threads, size_t lds, hipStream_t s,
                      ehyb_status& st) {
    switch (nrhs) {
        case 1: return launch_batched_l<DT, 1, NT>(L, a, nblocks, threads, lds, s, st);
        case 2: return launch_batched_l<DT, 2, NT>(L, a, nblocks, threads, lds, s, st);
        case 4: return launch_batched_l<DT, 4, NT>(L, a, nblocks, threads, lds, s, st);
        case 8: return launch_batched_l<DT, 8, NT>(L, a, nblocks, threads, lds, s, st);
        default: return false;
    }
}

template <int DT>
bool launch_batched_dt(int L, int nrhs, bool nt, const BatchArgs& a, int nblocks, int threads, size_t lds,
                       hipStream_t s, ehyb_status& st) {
    return nt ? launch_batched_r<DT, true>(L, nrhs, a, nblocks, threads, lds, s, st)
              : launch_batched_r<DT, false>(L, nrhs, a, nblocks, threads, lds, s, st);
}

// Streaming (non-temporal) loads of the value and column arrays pay when the
// product's bytes exceed the 256 MB Infinity Cache by a margin: back-to-back
// products then re-read nothing from it, and plain loads cost ~9% of the read
// bandwidth.  Below that, plain loads let repeated products hit the cache.
constexpr int64_t kStreamThresholdBytes = 384ll << 20;

bool use_stream_loads(int mode, int64_t bytes) {
    return mode == EHYB_LOAD_STREAM || (mode == EHYB_LOAD_AUTO && bytes > kStreamThresholdBytes);
}

bool is_aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// The kernels read x through buffer views with 32-bit byte offsets.
constexpr size_t kMaxVectorBytes = 0xFFFFFFFFull;

}  // namespace

extern "C" {

ehyb_status ehyb_plan_upload(ehyb_plan* P, void* dev_blob, size_t bytes, void* stream) {
    if (!P || !dev_blob) return fail(EHYB_EINVAL, "null argument");
    const BlobLayout L = compute_layout(*P);
    if (bytes < L.total) return fail(EHYB_EINVAL, "device blob smaller than ehyb_plan_device_bytes");
    if (!is_aligned(dev_blob, kBlobAlign)) return fail(EHYB_EINVAL, "device blob must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char* b = (char*)dev_blob;
    struct Piece {
        size_t off;
        const void* src;
        size_t bytes;
    } pieces[] = {
        {L.part_start, P->part_start.data(), P->part_start.size() * 4},
        {L.slice_start, P->slice_start.data(), P->slice_start.size() * 4},
        {L.er_slice_start, P->er_slice_start.data(), P->er_slice_start.size() * 4},
        {L.ell_free, P->ell_free.data(), P->ell_free.size() * 4},
        {L.halo_start, P->halo_start.data(), P->halo_start.size() * 4},
        {L.halo_idx, P->halo_idx.data(), P->halo_idx.size() * 4},
        {L.ell_meta, P->ell_meta.data(), P->ell_meta.size() * 4},
        {L.er_meta, P->er_meta.data(), P->er_meta.size() * 4},
        {L.er_row, P->er_row.data(), P->er_row.size() * 2},
        {L.ell_val, P->ell_val.data(), P->ell_val.size()},
        {L.ell_col, P->ell_col.data(), P->ell_col.size() * 2},
        {L.er_val, P->er_val.data(), P->er_val.size()},
        {L.er_col, P->er_col.data(), P->er_col.size() * 4},
        {L.perm, P->perm.data(), P->perm.size() * 4},
        {L.piece_start, P->piece_start.data(), P->piece_start.size() * 4},
        {L.piece_nwide, P->piece_nwide.data(), P->piece_nwide.size() * 4},
        {L.pieces, P->pieces.data(), P->pieces.size() * 4},
    };
    for (const Piece& pc : pieces) {
        if (pc.bytes == 0) continue;
        hipError_t e = hipMemcpyAsync(b + pc.off, pc.src, pc.bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return fail(EHYB_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(EHYB_EDEVICE, std::string("upload sync: ") + hipGetErrorString(e));
    P->dev_blob = dev_blob;
    P->dev_bytes = bytes;
    P->layout = L;
    return EHYB_OK;
}

ehyb_status ehyb_plan_set_launch(ehyb_plan* P, int32_t waves_per_wg) {
    if (!P) return fail(EHYB_EINVAL, "null argument");
    if (waves_per_wg != 0 && waves_per_wg != 4 && waves_per_wg != 8 && waves_per_wg != 16)
        return fail(EHYB_EINVAL, "waves_per_wg must be 0, 4, 8 or 16");
    P->launch_waves = waves_per_wg;
    return EHYB_OK;
}

ehyb_status ehyb_plan_set_load_mode(ehyb_plan* P, int32_t mode) {
    if (!P) return fail(EHYB_EINVAL, "null plan");
    if (mode < EHYB_LOAD_AUTO || mode > EHYB_LOAD_STREAM) return fail(EHYB_EINVAL, "unknown load mode");
    P->load_mode = mode;
    return EHYB_OK;
}

ehyb_status ehyb_batch_set_load_mode(ehyb_batch* B, int32_t mode) {
    if (!B) return fail(EHYB_EINVAL, "null batch");
    if (mode < EHYB_LOAD_AUTO || mode > EHYB_LOAD_STREAM) return fail(EHYB_EINVAL, "unknown load mode");
    B->load_mode = mode;
    return EHYB_OK;
}

ehyb_status ehyb_permute_x(const ehyb_plan* P, const void* x, void* xp, void* stream) {
    if (!P || !x || !xp) return fail(EHYB_EINVAL, "null argument");
    if (!P->dev_blob) return fail(EHYB_ESTATE, "plan not uploaded");
    if (P->n == 0) return EHYB_OK;
    const int32_t* perm = (const int32_t*)((const char*)P->dev_blob + P->layout.perm);
    const int nb = (int)((P->n + 255) / 256);
    if (P->xbytes == 8)
        hipLaunchKernelGGL(gather_kernel<double>, dim3(nb), dim3(256), 0, (hipStream_t)stream, P->n, perm,
                           (const double*)x, (double*)xp);
    else
        hipLaunchKernelGGL(gather_kernel<float>, dim3(nb), dim3(256), 0, (hipStream_t)stream, P->n, perm,
                           (const float*)x, (float*)xp);
    return launch_status("permute_x");
}

ehyb_status ehyb_unpermute_y(const ehyb_plan* P, const void* yp, void* y, void* stream) {
    if (!P || !y || !yp) return fail(EHYB_EINVAL, "null argument");
    if (!P->dev_blob) return fail(EHYB_ESTATE, "plan not uploaded");
    if (P->n == 0) return EHYB_OK;
    const int32_t* perm = (const int32_t*)((const char*)P->dev_blob + P->layout.perm);
    const int nb = (int)((P->n + 255) / 256);
    if (P->xbytes == 8)
        hipLaunchKernelGGL(scatter_kernel<double>, dim3(nb), dim3(256), 0, (hipStream_t)stream, P->n, perm,
                           (const double*)yp, (double*)y);
    else
        hipLaunchKernelGGL(scatter_kernel<float>, dim3(nb), dim3(256), 0, (hipStream_t)stream, P->n, perm,
                           (const float*)yp, (float*)y);
    return launch_status("unpermute_y");
}

ehyb_status ehyb_spmv(const ehyb_plan* P, const void* x, void* y, uint32_t flags, void* stream) {
    if (!P || !x || !y) return fail(EHYB_EINVAL, "null argument");
    if (flags & ~EHYB_VEC_PERMUTED) return fail(EHYB_EINVAL, "unknown flag");
    if (!P->dev_blob) return fail(EHYB_ESTATE, "plan not uploaded");
    const size_t xb = (size_t)P->xbytes;
    if (!is_aligned(x, xb) || !is_aligned(y, xb)) return fail(EHYB_EINVAL, "x and y must be aligned to their element size");
    const size_t vb = (size_t)P->n * xb;
    if ((const char*)x < (const char*)y + vb && (const char*)y < (const char*)x + vb)
        return fail(EHYB_EINVAL, "x and y must not overlap");
    if (P->n == 0) return EHYB_OK;
    if (vb > kMaxVectorBytes) return fail(EHYB_EUNSUPPORTED, "x and y are limited to 4 GiB - 1 bytes");
    hipStream_t s = (hipStream_t)stream;
    const char* blob = (const char*)P->dev_blob;
    const BlobLayout& Ly = P->layout;
    const void* xin = x;
    void* yout = y;
    if (!(flags & EHYB_VEC_PERMUTED)) {
        ehyb_status st = ehyb_permute_x(P, x, (void*)(blob + Ly.xp), stream);
        if (st != EHYB_OK) return st;
        xin = blob + Ly.xp;
        yout = (void*)(blob + Ly.yp);
    }
    SpmvArgs a;
    a.m = part_arrays(*P);
    a.x = xin;
    a.y = yout;
    const int nblocks = P->nparts;
    const size_t lds = (size_t)lds_bytes_used(*P);
    if (lds > 160 * 1024 - kStaticLds) return fail(EHYB_EUNSUPPORTED, "partition and halo larger than the LDS budget");
    if (P->kc != kc_for(P->value_dtype)) return fail(EHYB_EINVAL, "plan chunk width does not match its value type");
    const int threads = launch_waves(*P) * kWave;
    const bool nt = use_stream_loads(P->load_mode, algorithmic_bytes(*P));
    if (P->n_pieces > 0) {
        // hub rows: their wide residual slices are summed first, over the whole device
        switch (P->value_dtype) {
            case EHYB_F64: launch_pieces<EHYB_F64>(*P, nt, xin, s); break;
            case EHYB_F32: launch_pieces<EHYB_F32>(*P, nt, xin, s); break;
            case EHYB_BF16: launch_pieces<EHYB_BF16>(*P, nt, xin, s); break;
            case EHYB_F32_ACC64: launch_pieces<EHYB_F32_ACC64>(*P, nt, xin, s); break;
            case EHYB_BF16_ACC64: launch_pieces<EHYB_BF16_ACC64>(*P, nt, xin, s); break;
            default: return fail(EHYB_EINVAL, "bad value type");
        }
        a.m.er_piece = (const int32_t*)(blob + Ly.piece_start);
        a.m.er_nwide = (const int32_t*)(blob + Ly.piece_nwide);
        a.m.er_part = blob + Ly.ypart;
    }
    bool ok = false;
    ehyb_status st = EHYB_OK;
    switch (P->value_dtype) {
        case EHYB_F64: ok = launch_spmv_dt<EHYB_F64>(P->L, nt, a, nblocks, threads, lds, s, st); break;
        case EHYB_F32: ok = launch_spmv_dt<EHYB_F32>(P->L, nt, a, nblocks, threads, lds, s, st); break;
        case EHYB_BF16: ok = launch_spmv_dt<EHYB_BF16>(P->L, nt, a, nblocks, threads, lds, s, st); break;
        case EHYB_F32_ACC64: ok = launch_spmv_dt<EHYB_F32_ACC64>(P->L, nt, a, nblocks, threads, lds, s, st); break;
        case EHYB_BF16_ACC64: ok = launch_spmv_dt<EHYB_BF16_ACC64>(P->L, nt, a, nblocks, threads, lds, s, st); break;
        default: break;
    }
    if (!ok) return fail(EHYB_EINVAL, "bad lanes per row or value type");
    if (st != EHYB_OK) return st;
    st = launch_status("ehyb_spmv");
    if (st != EHYB_OK) return st;
    if (!(flags & EHYB_VEC_PERMUTED)) return ehyb_unpermute_y(P, yout, y, stream);
    return EHYB_OK;
}

ehyb_status ehyb_batch_create(const ehyb_plan* const* plans, int32_t n_plans, int32_t n_rhs, ehyb_batch** out) {
    try {
        if (!plans || !out) return fail(EHYB_EINVAL, "null argument");
        *out = nullptr;
        if (n_plans < 1 || n_plans > EHYB_BATCH_MAX) return fail(EHYB_EINVAL, "a batch holds 1 to 128 plans");
        if (n_rhs != 1 && n_rhs != 2 && n_rhs != 4 && n_rhs != 8) return fail(EHYB_EINVAL, "n_rhs must be 1, 2, 4 or 8");
        auto B = std::unique_ptr<ehyb_batch>(new ehyb_batch());
        B->n_rhs = n_rhs;
        for (int32_t i = 0; i < n_plans; ++i) {
            const ehyb_plan* P = plans[i];
            if (!P) return fail(EHYB_EINVAL, "null plan in batch");
            if (i == 0) {
                B->value_dtype = P->value_dtype;
                B->L = P->L;
            }
            if (P->value_dtype != B->value_dtype || P->L != B->L)
                return fail(EHYB_EINVAL, "batched plans must share value type and rows_per_wave");
            if (P->n_rhs != n_rhs) return fail(EHYB_EINVAL, "plan was not built for this n_rhs");
            B->plans.push_back(P);
        }
        if (B->L != 1 && B->L != 4 && B->L != 16)
            return fail(EHYB_EUNSUPPORTED, "batched products support rows_per_wave 64, 16 or 4");
        // work items by matrix, then partition, with the bytes each streams;
        // cut into one run per XCD queue of about equal bytes
        struct Item {
            int64_t cost;
            int32_t m, p;
        };
        std::vector<Item> items;
        int64_t total_cost = 0;
        for (int32_t i = 0; i < n_plans; ++i) {
            const ehyb_plan& P = *B->plans[i];
            for (int32_t p = 0; p < P.nparts; ++p) {
                int64_t c = 0;
                for (int32_t sl = P.slice_start[p]; sl < P.slice_start[p + 1]; ++sl)
                    c += (int64_t)(P.ell_meta[4 * (size_t)sl + 1] & 0xFFFFu) * kWave * (P.vbytes + 2);
                const int32_t ew = P.er_slice_start[p] + (P.n_pieces > 0 ? P.piece_nwide[p] : 0);
                for (int32_t e = P.er_slice_start[p]; e < P.er_slice_start[p + 1]; ++e)
                    c += e < ew ? (int64_t)(P.piece_start[e + 1] - P.piece_start[e]) * 8 * n_rhs
                                : (int64_t)P.er_meta[2 * (size_t)e + 1] * kWave * (P.vbytes + 4);
                c += 2LL * (P.part_start[p + 1] - P.part_start[p]) * P.xbytes * n_rhs;
                items.push_back({c, i, p});
                total_cost += c;
            }
            B->lds_bytes = std::max<int64_t>(B->lds_bytes, lds_bytes_used(P, n_rhs));
            B->algorithmic_bytes += algorithmic_bytes(P) + 2LL * (n_rhs - 1) * (P.n * P.xbytes + 8LL * P.n_pieces);
        }
        // the pieces of every matrix's wide residual slices, summed in one
        // launch before the product
        B->pbase.assign((size_t)n_plans + 1, 0);
        for (int32_t i = 0; i < n_plans; ++i) {
            const ehyb_plan& P = *B->plans[i];
            B->pbase[i + 1] = B->pbase[i] + P.n_pieces;
            for (int32_t q = 0; q < P.n_pieces; ++q) {
                B->pitems.push_back(i);
                for (int j = 0; j < 3; ++j) B->pitems.push_back(P.pieces[3 * (size_t)q + j]);
            }
        }
        if (B->pbase[n_plans] > INT32_MAX / 4) return fail(EHYB_EUNSUPPORTED, "more than 2^29 pieces of wide slices");
        if (B->lds_bytes > 160 * 1024 - kStaticLds) return fail(EHYB_EINVAL, "a plan needs more LDS than a workgroup has");
        if (items.size() > (size_t)INT32_MAX) return fail(EHYB_EUNSUPPORTED, "more than 2^31 work items");
        B->items.reserve(items.size() * 2);
        B->range.assign(kXcds + 1, 0);
        int64_t run = 0;
        int32_t q = 1;
        for (size_t k = 0; k < items.size(); ++k) {
            // item k starts queue q once the items before it hold q/8 of the bytes
            while (q < kXcds && run * kXcds >= total_cost * q) B->range[q++] = (int32_t)k;
            B->items.push_back(items[k].m);
            B->items.push_back(items[k].p);
            run += items[k].cost;
        }
        while (q <= kXcds) B->range[q++] = (int32_t)items.size();
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t at = off;
            off += (bytes + kBlobAlign - 1) / kBlobAlign * kBlobAlign;
            return at;
        };
        B->off_desc = take(sizeof(PartArrays) * (size_t)n_plans);
        B->off_items = take(B->items.size() * 4);
        B->off_counters = take((kXcds + 1) * kCtrStride * sizeof(int32_t));
        B->off_pitems = take(B->pitems.size() * 4);
        B->off_part = take((size_t)B->pbase[n_plans] * n_rhs * acc_bytes(B->value_dtype));
        B->total = off;
        *out = B.release();
        return EHYB_OK;
    } catch (const std::bad_alloc&) {
        return fail(EHYB_ENOMEM, "host allocation failed while building a batch");
    }
}

ehyb_status ehyb_batch_device_bytes(const ehyb_batch* B, size_t* bytes) {
    if (!B || !bytes) return fail(EHYB_EINVAL, "null argument");
    *bytes = B->total;
    return EHYB_OK;
}

ehyb_status ehyb_batch_upload(ehyb_batch* B, void* dev_blob, size_t bytes, void* stream) {
    if (!B || !dev_blob) return fail(EHYB_EINVAL, "null argument");
    if (bytes < B->total) return fail(EHYB_EINVAL, "device blob smaller than ehyb_batch_device_bytes");
    if (!is_aligned(dev_blob, kBlobAlign)) return fail(EHYB_EINVAL, "device blob must be 256-byte aligned");
    std::vector<PartArrays> desc;
    char* b = (char*)dev_blob;
    for (size_t i = 0; i < B->plans.size(); ++i) {
        const ehyb_plan* P = B->plans[i];
        if (!P->dev_blob) return fail(EHYB_ESTATE, "every plan of a batch must be uploaded first");
        desc.push_back(part_arrays(*P));
        if (P->n_pieces > 0) {
            // wide slices: piece ranges from the plan, sums in the batch's blob
            const char* pb = (const char*)P->dev_blob;
            desc.back().er_piece = (const int32_t*)(pb + P->layout.piece_start);
            desc.back().er_nwide = (const int32_t*)(pb + P->layout.piece_nwide);
            desc.back().er_part = b + B->off_part + (size_t)B->pbase[i] * B->n_rhs * acc_bytes(B->value_dtype);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    const std::vector<int32_t> zeros((kXcds + 1) * kCtrStride, 0);
    hipError_t e = hipMemcpyAsync(b + B->off_desc, desc.data(), desc.size() * sizeof(PartArrays),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B->items.empty())
        e = hipMemcpyAsync(b + B->off_items, B->items.data(), B->items.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b + B->off_counters, zeros.data(), zeros.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !B->pitems.empty())
        e = hipMemcpyAsync(b + B->off_pitems, B->pitems.data(), B->pitems.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(EHYB_EDEVICE, std::string("batch upload: ") + hipGetErrorString(e));
    B->dev_blob = dev_blob;
    return EHYB_OK;
}

ehyb_status ehyb_spmm_batched(const ehyb_batch* B, int32_t n_rhs, const void* const* X, void* const* Y,
                              uint32_t flags, void* stream) {
    if (!B || !X || !Y) return fail(EHYB_EINVAL, "null argument");
    if (!B->dev_blob) return fail(EHYB_ESTATE, "batch not uploaded");
    if (n_rhs != B->n_rhs) return fail(EHYB_EINVAL, "n_rhs differs from the batch's");
    if (flags != EHYB_VEC_PERMUTED) return fail(EHYB_EUNSUPPORTED, "batched products take permuted vectors only");
    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    const char* b = (const char*)B->dev_blob;
    a.mats = (const PartArrays*)(b + B->off_desc);
    a.items = (const int2*)(b + B->off_items);
    a.n_items = (int32_t)(B->items.size() / 2);
    a.counters = (int32_t*)(b + B->off_counters);
    for (int q = 0; q <= kXcds; ++q) a.range[q] = B->range[q];
    const size_t eb = (B->value_dtype == EHYB_F64 ? 8 : 4);
    for (size_t i = 0; i < B->plans.size(); ++i) {
        if (!X[i] || !Y[i]) return fail(EHYB_EINVAL, "null vector in batch");
        if (!is_aligned(X[i], eb * n_rhs) || !is_aligned(Y[i], eb * n_rhs))
            return fail(EHYB_EINVAL, "batched vectors must be aligned to a whole row (n_rhs elements)");
        const size_t vb = (size_t)B->plans[i]->n * eb * n_rhs;
        if (vb > kMaxVectorBytes) return fail(EHYB_EUNSUPPORTED, "each X and Y is limited to 4 GiB - 1 bytes");
        const char* xi = (const char*)X[i];
        const char* yi = (const char*)Y[i];
        if (xi < yi + vb && yi < xi + vb) return fail(EHYB_EINVAL, "X and Y of a matrix must not overlap");
        a.X[i] = X[i];
        a.Y[i] = Y[i];
    }
    if (a.n_items == 0) return EHYB_OK;
    // Up to four workgroups per CU when their partitions' LDS fits, so that
    // one workgroup's staging (latency-bound gathers) overlaps the others'
    // streaming; the CU's 16 wavefronts are split among them (16, 8, 5 or
    // 4 per workgroup, within what the kernels' register use allows).
    const int per_cu = (int)std::max<int64_t>(
        1, std::min<int64_t>(4, (160 * 1024) / std::max<int64_t>(1, B->lds_bytes + kStaticLds)));
    const int threads = 64 * (16 / per_cu);
    const bool nt = use_stream_loads(B->load_mode, B->algorithmic_bytes);
    const int nblocks = std::min(a.n_items, 256 * per_cu);
    bool ok = false;
    ehyb_status st = EHYB_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t lds = (size_t)B->lds_bytes;
    if (!B->pitems.empty()) {
        // hub rows: their wide residual slices are summed first, over the whole device
        BatchPieceArgs pa;
        std::memset(&pa, 0, sizeof(pa));
        pa.mats = a.mats;
        pa.items = (const int4*)(b + B->off_pitems);
        pa.n_items = (int32_t)(B->pitems.size() / 4);
        pa.part = (void*)(b + B->off_part);
        for (size_t i = 0; i < B->plans.size(); ++i) pa.X[i] = X[i];
        bool pok = false;
        switch (B->value_dtype) {
            case EHYB_F64: pok = launch_pieces_batched<EHYB_F64>(n_rhs, nt, pa, s); break;
            case EHYB_F32: pok = launch_pieces_batched<EHYB_F32>(n_rhs, nt, pa, s); break;
            case EHYB_BF16: pok = launch_pieces_batched<EHYB_BF16>(n_rhs, nt, pa, s); break;
            case EHYB_F32_ACC64: pok = launch_pieces_batched<EHYB_F32_ACC64>(n_rhs, nt, pa, s); break;
            case EHYB_BF16_ACC64: pok = launch_pieces_batched<EHYB_BF16_ACC64>(n_rhs, nt, pa, s); break;
            default: break;
        }
        if (!pok) return fail(EHYB_EUNSUPPORTED, "no batched piece kernel for this value type and n_rhs");
    }
    switch (B->value_dtype) {
        case EHYB_F64: ok = launch_batched_dt<EHYB_F64>(B->L, n_rhs, nt, a, nblocks, threads, lds, s, st); break;
        case EHYB_F32: ok = launch_batched_dt<EHYB_F32>(B->L, n_rhs, nt, a, nblocks, threads, lds, s, st); break;
        case EHYB_BF16: ok = launch_batched_dt<EHYB_BF16>(B->L, n_rhs, nt, a, nblocks, threads, lds, s, st); break;
        case EHYB_F32_ACC64: ok = launch_batched_dt<EHYB_F32_ACC64>(B->L, n_rhs, nt, a, nblocks, threads, lds, s, st); break;
        case EHYB_BF16_ACC64:
            ok = launch_batched_dt<EHYB_BF16_ACC64>(B->L, n_rhs, nt, a, nblocks, threads, lds, s, st);
            break;
        default: break;
    }
    if (!ok) return fail(EHYB_EUNSUPPORTED, "no batched kernel for this value type, rows_per_wave and n_rhs");
    if (st != EHYB_OK) return st;
    return launch_status("ehyb_spmm_batched");
}

void ehyb_batch_destroy(ehyb_batch* B) { delete B; }

ehyb_status ehyb_csr_spmv_f64(int64_t n_rows, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                              const double* val, const double* x, double* y, int32_t lanes_per_row,
                              void* stream) {
    if (n_rows < 0 || nnz < 0) return fail(EHYB_EINVAL, "negative size");
    if (n_rows == 0) return EHYB_OK;
    if (!row_ptr || !x || !y || (nnz > 0 && (!col_idx || !val))) return fail(EHYB_EINVAL, "null argument");
    if (nnz >= (1ll << 29) || n_rows >= (1ll << 29))
        return fail(EHYB_EUNSUPPORTED, "the CSR kernel addresses values and x with 32-bit byte offsets (below 2^29 entries)");
    int L = lanes_per_row;
    if (L == 0) {
        const double mean = (double)nnz / (double)n_rows;
        // the fewest lanes whose first batch covers a row of mean length
        L = 1;
        while (L < 64 && L * kCsrU < mean) L *= 2;
    }
    if (L < 1 || L > 64 || (L & (L - 1))) return fail(EHYB_EINVAL, "lanes_per_row must be a power of two <= 64");
    const int64_t threads = n_rows * L;
    const int64_t nb = (threads + 255) / 256;
    if (nb > INT32_MAX) return fail(EHYB_EUNSUPPORTED, "too many workgroups");
    hipStream_t s = (hipStream_t)stream;
#define EHYB_CSR_CASE(LL)                                                                            \
    case LL:                                                                                         \
        hipLaunchKernelGGL(csr_spmv_f64_kernel<LL>, dim3((unsigned)nb), dim3(256), 0, s, n_rows, nnz, row_ptr, \
                           col_idx, val, x, y);                                                      \
        break;
    switch (L) {
        EHYB_CSR_CASE(1)
        EHYB_CSR_CASE(2)
        EHYB_CSR_CASE(4)
        EHYB_CSR_CASE(8)
        EHYB_CSR_CASE(16)
        EHYB_CSR_CASE(32)
        EHYB_CSR_CASE(64)
    }
#undef EHYB_CSR_CASE
    return launch_status("csr_spmv");
}

static ehyb_status probe_read_launch(bool nt, const void* buf, size_t bytes, void* sink, void* stream) {
    if (!buf || !sink) return fail(EHYB_EINVAL, "null argument");
    if (bytes % 16 || !is_aligned(buf, 16)) return fail(EHYB_EINVAL, "bytes and buf must be 16-byte multiples");
    if (bytes == 0) return EHYB_OK;
    const size_t n16 = bytes / 16;
    const int nb = (int)std::min<size_t>(16384, std::max<size_t>(1, n16 / (512 * 4)));
    if (nt)
        hipLaunchKernelGGL(probe_read_kernel<true>, dim3(nb), dim3(512), 0, (hipStream_t)stream, (const u32x4*)buf,
                           n16, (uint64_t*)sink);
    else
        hipLaunchKernelGGL(probe_read_kernel<false>, dim3(nb), dim3(512), 0, (hipStream_t)stream, (const u32x4*)buf,
                           n16, (uint64_t*)sink);
    return launch_status(nt ? "probe_read" : "cache_flush");
}

ehyb_status ehyb_probe_read(const void* buf, size_t bytes, void* sink, void* stream) {
    return probe_read_launch(true, buf, bytes, sink, stream);
}

ehyb_status ehyb_cache_flush(const void* buf, size_t bytes, void* sink, void* stream) {
    return probe_read_launch(false, buf, bytes, sink, stream);
}

ehyb_status ehyb_probe_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst) return fail(EHYB_EINVAL, "null argument");
    if (bytes % 16 || !is_aligned(src, 16) || !is_aligned(dst, 16))
        return fail(EHYB_EINVAL, "bytes and pointers must be 16-byte multiples");
    if (bytes == 0) return EHYB_OK;
    const size_t n16 = bytes / 16;
    const int nb = (int)std::min<size_t>(65536, std::max<size_t>(1, n16 / (256 * 8)));
    hipLaunchKernelGGL(probe_copy_kernel, dim3(nb), dim3(256), 0, (hipStream_t)stream, (const uint4*)src,
                       (uint4*)dst, n16);
    return launch_status("probe_copy");
}

ehyb_status ehyb_device_info_get(ehyb_device_info* out) {
    if (!out) return fail(EHYB_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(EHYB_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail(EHYB_EDEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
    out->device = dev;
    out->num_cus = prop.multiProcessorCount;
    out->lds_per_block = (int32_t)prop.sharedMemPerBlock;
    out->warp_size = prop.warpSize;
    out->clock_khz = prop.clockRate;
    out->mem_clock_khz = prop.memoryClockRate;
    out->mem_bus_width = prop.memoryBusWidth;
    out->l2_bytes = prop.l2CacheSize;
    std::strncpy(out->arch, prop.gcnArchName, sizeof(out->arch) - 1);
    return EHYB_OK;
}

}  // extern "C"
