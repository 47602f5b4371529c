// Device side of the EHYB library for gfx950 (CDNA4, wave64): the EHYB SpMV
// kernel, the plain CSR baseline, bandwidth probes and vector permutations,
// plus the C-ABI entry points that upload plans and launch kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "internal.h"

using namespace ehyb;

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

struct SpmvF64Args {
    const int32_t* part_start;
    const int32_t* slice_start;
    const uint4* slice_meta;   // ell_off, ell_steps, er_off, er_steps
    const double* ell_val;
    const uint16_t* ell_col;
    const double* er_val;
    const int32_t* er_col;
    const double* x;           // permuted order
    double* y;                 // permuted order
    int32_t nparts;
    int32_t wgs_per_part;      // workgroups sharing one partition
};

// One workgroup stages its partition's x-slice in LDS (Alg. 3: the cached
// vector), then each wavefront sweeps row-slices of that partition: 64 lanes,
// L lanes per row, two ELL entries per lane per step (a 16-byte value load and
// a 4-byte load of two 16-bit columns), multiply-add against the LDS copy,
// then the row's residual entries against x in device memory, a reduction
// over the L lanes of a row, and one store per row.  Row-slices are dealt to
// wavefronts statically; the ELL and residual parts of a row are summed by the
// same lane group, so y needs no atomics and the result is deterministic.
template <int L>
__global__ void __launch_bounds__(512) ehyb_spmv_f64_kernel(SpmvF64Args a) {
    extern __shared__ double xs[];
    constexpr int C = kWave / L;
    const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
    const int p = logical / a.wgs_per_part;
    const int sub = logical - p * a.wgs_per_part;
    const int ps = a.part_start[p];
    const int sz = a.part_start[p + 1] - ps;

    // stage the x-slice: 16-byte loads over the aligned body, scalar edges
    {
        const double* src = a.x + ps;
        const int head = (int)(((uintptr_t)src >> 3) & 1);  // 1 if src is 8- but not 16-byte aligned
        const int h = head < sz ? head : sz;
        const int nvec = (sz - h) >> 1;
        const double2* src2 = reinterpret_cast<const double2*>(src + h);
        for (int i = threadIdx.x; i < nvec; i += blockDim.x) {
            const double2 v = src2[i];
            xs[h + 2 * i] = v.x;
            xs[h + 2 * i + 1] = v.y;
        }
        if (threadIdx.x < h) xs[0] = src[0];
        const int tail = h + 2 * nvec;
        if ((int)threadIdx.x < sz - tail) xs[tail + threadIdx.x] = src[tail + threadIdx.x];
    }
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    const int s0 = a.slice_start[p], s1 = a.slice_start[p + 1];
    const int stride = a.wgs_per_part * nwaves;
    const int r = lane / L;
    for (int s = s0 + sub * nwaves + wave; s < s1; s += stride) {
        const uint4 m = a.slice_meta[s];
        double acc = 0.0;
        const double2* v2 = reinterpret_cast<const double2*>(a.ell_val + m.x) + lane;
        const uint32_t* c2 = reinterpret_cast<const uint32_t*>(a.ell_col + m.x) + lane;
        uint32_t t = 0;
        for (; t + 2 <= m.y; t += 2) {
            const double2 va = v2[(size_t)t * kWave];
            const uint32_t ca = c2[(size_t)t * kWave];
            const double2 vb = v2[(size_t)(t + 1) * kWave];
            const uint32_t cb = c2[(size_t)(t + 1) * kWave];
            acc = fma(va.x, xs[ca & 0xFFFFu], acc);
            acc = fma(va.y, xs[ca >> 16], acc);
            acc = fma(vb.x, xs[cb & 0xFFFFu], acc);
            acc = fma(vb.y, xs[cb >> 16], acc);
        }
        if (t < m.y) {
            const double2 va = v2[(size_t)t * kWave];
            const uint32_t ca = c2[(size_t)t * kWave];
            acc = fma(va.x, xs[ca & 0xFFFFu], acc);
            acc = fma(va.y, xs[ca >> 16], acc);
        }
        const double* ev = a.er_val + m.z + lane;
        const int32_t* ec = a.er_col + m.z + lane;
        for (uint32_t k = 0; k < m.w; ++k) acc = fma(ev[(size_t)k * kWave], a.x[ec[(size_t)k * kWave]], acc);
        if constexpr (L > 1) {
#pragma unroll
            for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        }
        const int row = ps + (s - s0) * C + r;
        if ((lane & (L - 1)) == 0 && row < ps + sz) a.y[row] = acc;
    }
}

// Plain CSR SpMV: L lanes per row (rows of a wavefront are consecutive),
// strided loop over the row's entries, reduction over the L lanes.
template <int L>
__global__ void __launch_bounds__(256) csr_spmv_f64_kernel(int64_t n, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const double* __restrict__ v,
                                                           const double* __restrict__ x,
                                                           double* __restrict__ y) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = gid / L;
    const int sub = (int)(gid & (L - 1));
    double acc = 0.0;
    if (row < n) {
        const int32_t b = rp[row], e = rp[row + 1];
        for (int32_t q = b + sub; q < e; q += L) acc = fma(v[q], x[ci[q]], acc);
    }
    if constexpr (L > 1) {
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    }
    if (sub == 0 && row < n) y[row] = acc;
}

// Read-stream probe: every byte of buf is loaded once with 16-byte
// non-temporal loads; one partial per workgroup keeps the loads alive.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) probe_read_kernel(const u32x4* __restrict__ buf, size_t n16,
                                                         uint64_t* __restrict__ sink) {
    uint32_t acc = 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const u32x4 v = __builtin_nontemporal_load(buf + i);
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

struct LaunchShape {
    int waves_per_wg;
    int wgs_per_part;
};

// Waves per workgroup and workgroups per partition: enough wavefronts to keep
// every CU busy (about 16 per CU), never more wavefronts on a partition than
// it has row-slices.
LaunchShape launch_shape(const ehyb_plan& P) {
    LaunchShape sh{8, 1};
    if (P.nparts == 0) return sh;
    const int64_t per_part = (P.nslices + P.nparts - 1) / P.nparts;
    sh.waves_per_wg = (int)std::max<int64_t>(1, std::min<int64_t>(8, per_part));
    const int64_t target_waves = 256LL * 16;
    int64_t w = (target_waves + (int64_t)P.nparts * sh.waves_per_wg - 1) / ((int64_t)P.nparts * sh.waves_per_wg);
    const int64_t max_w = std::max<int64_t>(1, per_part / sh.waves_per_wg);
    sh.wgs_per_part = (int)std::max<int64_t>(1, std::min<int64_t>(w, max_w));
    return sh;
}

template <int L>
void launch_spmv_f64(const SpmvF64Args& a, int nblocks, int threads, size_t lds, hipStream_t s) {
    static bool lds_raised = false;
    if (!lds_raised && lds > 64 * 1024) {
        // allow the full 160 KiB of gfx950 LDS as dynamic shared memory
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&ehyb_spmv_f64_kernel<L>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
            (void)hipGetLastError();
        lds_raised = true;
    }
    hipLaunchKernelGGL(ehyb_spmv_f64_kernel<L>, dim3(nblocks), dim3(threads), lds, s, a);
}

bool is_aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

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
        {L.slice_meta, P->slice_meta.data(), P->slice_meta.size() * 4},
        {L.ell_val, P->ell_val.data(), P->ell_val.size()},
        {L.ell_col, P->ell_col.data(), P->ell_col.size() * 2},
        {L.er_val, P->er_val.data(), P->er_val.size()},
        {L.er_col, P->er_col.data(), P->er_col.size() * 4},
        {L.perm, P->perm.data(), P->perm.size() * 4},
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
    if (P->value_dtype != EHYB_F64) return fail(EHYB_EUNSUPPORTED, "only FP64 plans have a kernel");
    if (x == y) return fail(EHYB_EINVAL, "x and y must not overlap");
    if (!is_aligned(x, 8) || !is_aligned(y, 8)) return fail(EHYB_EINVAL, "x and y must be 8-byte aligned");
    const size_t vb = (size_t)P->n * 8;
    if ((const char*)x < (const char*)y + vb && (const char*)y < (const char*)x + vb)
        return fail(EHYB_EINVAL, "x and y must not overlap");
    if (P->n == 0) return EHYB_OK;
    hipStream_t s = (hipStream_t)stream;
    const char* blob = (const char*)P->dev_blob;
    const BlobLayout& Ly = P->layout;
    const double* xin = (const double*)x;
    double* yout = (double*)y;
    if (!(flags & EHYB_VEC_PERMUTED)) {
        ehyb_status st = ehyb_permute_x(P, x, (void*)(blob + Ly.xp), stream);
        if (st != EHYB_OK) return st;
        xin = (const double*)(blob + Ly.xp);
        yout = (double*)(blob + Ly.yp);
    }
    SpmvF64Args a;
    a.part_start = (const int32_t*)(blob + Ly.part_start);
    a.slice_start = (const int32_t*)(blob + Ly.slice_start);
    a.slice_meta = (const uint4*)(blob + Ly.slice_meta);
    a.ell_val = (const double*)(blob + Ly.ell_val);
    a.ell_col = (const uint16_t*)(blob + Ly.ell_col);
    a.er_val = (const double*)(blob + Ly.er_val);
    a.er_col = (const int32_t*)(blob + Ly.er_col);
    a.x = xin;
    a.y = yout;
    a.nparts = P->nparts;
    const LaunchShape sh = launch_shape(*P);
    a.wgs_per_part = sh.wgs_per_part;
    const int64_t nblocks = (int64_t)P->nparts * sh.wgs_per_part;
    if (nblocks > INT32_MAX) return fail(EHYB_EUNSUPPORTED, "too many workgroups");
    const size_t lds = (size_t)P->max_part_rows * 8;
    if (lds > 160 * 1024) return fail(EHYB_EUNSUPPORTED, "x-slice larger than LDS");
    const int threads = sh.waves_per_wg * kWave;
    switch (P->L) {
        case 1: launch_spmv_f64<1>(a, (int)nblocks, threads, lds, s); break;
        case 2: launch_spmv_f64<2>(a, (int)nblocks, threads, lds, s); break;
        case 4: launch_spmv_f64<4>(a, (int)nblocks, threads, lds, s); break;
        case 8: launch_spmv_f64<8>(a, (int)nblocks, threads, lds, s); break;
        case 16: launch_spmv_f64<16>(a, (int)nblocks, threads, lds, s); break;
        case 32: launch_spmv_f64<32>(a, (int)nblocks, threads, lds, s); break;
        case 64: launch_spmv_f64<64>(a, (int)nblocks, threads, lds, s); break;
        default: return fail(EHYB_EINVAL, "bad lanes per row");
    }
    ehyb_status st = launch_status("ehyb_spmv");
    if (st != EHYB_OK) return st;
    if (!(flags & EHYB_VEC_PERMUTED)) return ehyb_unpermute_y(P, yout, y, stream);
    return EHYB_OK;
}

ehyb_status ehyb_csr_spmv_f64(int64_t n_rows, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                              const double* val, const double* x, double* y, int32_t lanes_per_row,
                              void* stream) {
    if (n_rows < 0 || nnz < 0) return fail(EHYB_EINVAL, "negative size");
    if (n_rows == 0) return EHYB_OK;
    if (!row_ptr || !x || !y || (nnz > 0 && (!col_idx || !val))) return fail(EHYB_EINVAL, "null argument");
    if (nnz > INT32_MAX) return fail(EHYB_EUNSUPPORTED, "int32 row pointers limit nnz to 2^31-1");
    int L = lanes_per_row;
    if (L == 0) {
        const double mean = (double)nnz / (double)n_rows;
        L = mean <= 4 ? 2 : mean <= 8 ? 4 : mean <= 16 ? 8 : mean <= 32 ? 16 : mean <= 64 ? 32 : 64;
    }
    if (L < 1 || L > 64 || (L & (L - 1))) return fail(EHYB_EINVAL, "lanes_per_row must be a power of two <= 64");
    const int64_t threads = n_rows * L;
    const int64_t nb = (threads + 255) / 256;
    if (nb > INT32_MAX) return fail(EHYB_EUNSUPPORTED, "too many workgroups");
    hipStream_t s = (hipStream_t)stream;
#define EHYB_CSR_CASE(LL)                                                                            \
    case LL:                                                                                         \
        hipLaunchKernelGGL(csr_spmv_f64_kernel<LL>, dim3((unsigned)nb), dim3(256), 0, s, n_rows, row_ptr, \
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

ehyb_status ehyb_probe_read(const void* buf, size_t bytes, void* sink, void* stream) {
    if (!buf || !sink) return fail(EHYB_EINVAL, "null argument");
    if (bytes % 16 || !is_aligned(buf, 16)) return fail(EHYB_EINVAL, "bytes and buf must be 16-byte multiples");
    if (bytes == 0) return EHYB_OK;
    const size_t n16 = bytes / 16;
    const int nb = (int)std::min<size_t>(65536, std::max<size_t>(1, n16 / (256 * 8)));
    hipLaunchKernelGGL(probe_read_kernel, dim3(nb), dim3(256), 0, (hipStream_t)stream, (const u32x4*)buf, n16,
                       (uint64_t*)sink);
    return launch_status("probe_read");
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
