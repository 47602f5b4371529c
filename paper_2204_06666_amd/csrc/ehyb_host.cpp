// Host side of the EHYB library: input validation, graph construction,
// partitioning, reordering (Alg. 1), encoding of the two parts (Alg. 2),
// decoding, plan views and plan files.  No device code lives here.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <stdexcept>

#include "internal.h"

namespace ehyb {

namespace {
thread_local std::string g_last_error;

double now_s() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

int threads_for(const ehyb_params& p) {
    return p.n_threads > 0 ? p.n_threads : omp_get_max_threads();
}

// Sets the OpenMP thread count for the library's own parallel regions and
// restores the caller's setting on exit.
struct ThreadGuard {
    int prev;
    explicit ThreadGuard(int n) : prev(omp_get_max_threads()) { omp_set_num_threads(n); }
    ~ThreadGuard() { omp_set_num_threads(prev); }
};

// Round a binary64 value to the nearest bfloat16 (ties to even) without
// passing through binary32, returning its 16-bit pattern.
uint16_t double_to_bf16(double d) {
    if (std::isnan(d)) return 0x7FC0;
    if (d == 0.0) return std::signbit(d) ? 0x8000 : 0x0000;
    const double a = std::fabs(d);
    int e;
    std::frexp(a, &e);                  // a = m * 2^e, m in [0.5, 1)
    int ulp_exp = (e - 1) - 7;          // 8 significant bits
    if (ulp_exp < -133) ulp_exp = -133;  // subnormal range of bfloat16
    const double q = std::nearbyint(std::ldexp(a, -ulp_exp));  // ties to even
    const double r = std::ldexp(q, ulp_exp);
    float f = (r > 3.3895313892515355e38) ? INFINITY : (float)r;  // exact when finite
    uint32_t bits;
    std::memcpy(&bits, &f, 4);
    uint16_t h = (uint16_t)(bits >> 16);
    if (std::signbit(d)) h |= 0x8000;
    return h;
}

void store_value(unsigned char* dst, int vbytes, int dtype, double v) {
    dtype = storage_dtype(dtype);
    if (dtype == EHYB_F64) {
        std::memcpy(dst, &v, 8);
    } else if (dtype == EHYB_F32) {
        float f = (float)v;
        std::memcpy(dst, &f, 4);
    } else {
        uint16_t h = double_to_bf16(v);
        std::memcpy(dst, &h, 2);
    }
    (void)vbytes;
}

double load_value(const unsigned char* src, int dtype) {
    dtype = storage_dtype(dtype);
    if (dtype == EHYB_F64) {
        double d;
        std::memcpy(&d, src, 8);
        return d;
    }
    if (dtype == EHYB_F32) {
        float f;
        std::memcpy(&f, src, 4);
        return (double)f;
    }
    uint16_t h;
    std::memcpy(&h, src, 2);
    uint32_t bits = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &bits, 4);
    return (double)f;
}

Error validate(const ehyb_csr_host* A) {
    Error e;
    auto bad = [&](ehyb_status st, std::string m) {
        e.status = st;
        e.msg = std::move(m);
        return e;
    };
    if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0) return bad(EHYB_EINVAL, "negative size");
    if (A->n_rows != A->n_cols)
        return bad(EHYB_EUNSUPPORTED, "matrix is not square (rows and columns are one vertex set)");
    if (A->n_rows > (int64_t)INT32_MAX - 1) return bad(EHYB_EUNSUPPORTED, "more than 2^31-2 rows");
    if (A->nnz > 0 && (!A->col_idx || !A->val)) return bad(EHYB_EINVAL, "null col_idx or val");
    if (!A->row_ptr) return bad(EHYB_EINVAL, "null row_ptr");
    const int64_t n = A->n_rows;
    if (A->row_ptr[0] != 0) return bad(EHYB_EINVAL, "row_ptr[0] != 0");
    if (A->row_ptr[n] != A->nnz) return bad(EHYB_EINVAL, "row_ptr[n] != nnz");
    for (int64_t i = 0; i < n; ++i)
        if (A->row_ptr[i + 1] < A->row_ptr[i])
            return bad(EHYB_EINVAL, "row_ptr decreases at row " + std::to_string(i));
    int64_t bad_row = -1;
    int bad_kind = 0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; ++p) {
            const int32_t c = A->col_idx[p];
            int kind = 0;
            if (c < 0 || c >= n) kind = 1;
            else if (p > A->row_ptr[i] && c <= A->col_idx[p - 1]) kind = 2;
            if (kind) {
#pragma omp critical
                {
                    if (bad_row < 0 || i < bad_row) {
                        bad_row = i;
                        bad_kind = kind;
                    }
                }
                break;
            }
        }
    }
    if (bad_row >= 0)
        return bad(EHYB_EINVAL, std::string(bad_kind == 1 ? "column index out of range"
                                                          : "columns not strictly increasing (unsorted or duplicate)") +
                                    " in row " + std::to_string(bad_row));
    return e;
}

// Graph of A + A^T without self loops; edge weight = number of stored entries
// among a_ij, a_ji (Section 3.1: each entry is an edge between its row and
// column vertices).
Graph build_graph(const ehyb_csr_host* A) {
    const int32_t n = (int32_t)A->n_rows;
    const int64_t nnz = A->nnz;
    // transpose pattern (CSC): rows of each column, ascending.  Counts and
    // slots are claimed with atomic adds, then each column is sorted, so the
    // result does not depend on the thread schedule.
    std::vector<int64_t> tptr(n + 1, 0);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < nnz; ++p) __atomic_fetch_add(&tptr[A->col_idx[p] + 1], 1, __ATOMIC_RELAXED);
    for (int32_t j = 0; j < n; ++j) tptr[j + 1] += tptr[j];
    uvec<int32_t> trow(nnz);
    {
        std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
#pragma omp parallel for schedule(dynamic, 4096)
        for (int32_t i = 0; i < n; ++i)
            for (int64_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; ++p)
                trow[__atomic_fetch_add(&fill[A->col_idx[p]], 1, __ATOMIC_RELAXED)] = i;
#pragma omp parallel for schedule(dynamic, 4096)
        for (int32_t j = 0; j < n; ++j) std::sort(trow.begin() + tptr[j], trow.begin() + tptr[j + 1]);
    }
    Graph g;
    g.n = n;
    g.xadj.assign(n + 1, 0);
    g.vw.assign(n, 1);
    // union of row v's columns and column v's rows, self excluded
    auto merge = [&](int32_t v, int32_t* adj, int32_t* ew) -> int64_t {
        int64_t a = A->row_ptr[v], ae = A->row_ptr[v + 1];
        int64_t b = tptr[v], be = tptr[v + 1];
        int64_t k = 0;
        while (a < ae || b < be) {
            int32_t ca = a < ae ? A->col_idx[a] : INT32_MAX;
            int32_t cb = b < be ? trow[b] : INT32_MAX;
            int32_t c;
            int32_t w;
            if (ca == cb) {
                c = ca;
                w = 2;
                ++a;
                ++b;
            } else if (ca < cb) {
                c = ca;
                w = 1;
                ++a;
            } else {
                c = cb;
                w = 1;
                ++b;
            }
            if (c == v) continue;
            if (adj) {
                adj[k] = c;
                ew[k] = w;
            }
            ++k;
        }
        return k;
    };
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; ++v) g.xadj[v + 1] = merge(v, nullptr, nullptr);
    for (int32_t v = 0; v < n; ++v) g.xadj[v + 1] += g.xadj[v];
    g.adj.resize(g.xadj[n]);
    g.ew.resize(g.xadj[n]);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; ++v) merge(v, g.adj.data() + g.xadj[v], g.ew.data() + g.xadj[v]);
    return g;
}

// Work-weighted partition balance.  The paper sizes partitions by rows
// (Eq. 1); on power-law graphs the rows many times longer than the mean fall
// into a few partitions (the partitioner keeps densely linked hubs together),
// whose workgroups then set the time of the launch.  A row of at least twice
// the mean length weighs its ELL-eligible entries (up to the width cap; 0 =
// no cap) in units of the mean length, at most min(64, row_cap / 8); every
// other row weighs 1, so matrices without such rows are partitioned exactly
// as by rows.  The partition count stays Eq. 1's.  The returned weight cap is
// the mean weight per partition plus the allowed imbalance, never below the
// row cap and never above the LDS row limit: a partition's rows, each
// weighing at least 1, always fit its LDS.  Where the LDS limit leaves no room
// for the weights, rows are balanced as without them.
int64_t weigh_long_rows(Graph& g, const ehyb_csr_host* A, int64_t width_cap, int32_t nparts, int64_t row_cap,
                        int64_t max_rows, int32_t imbalance_pct) {
    const int64_t n = g.n;
    if (n == 0 || A->nnz == 0 || nparts < 1) return row_cap;
    const double mean = (double)A->nnz / (double)n;
    const double wmax = (double)std::max<int64_t>(1, std::min<int64_t>(64, row_cap / 8));
    int64_t sumw = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t len = A->row_ptr[v + 1] - A->row_ptr[v];
        int32_t w = 1;
        if ((double)len >= 2.0 * mean) {
            const int64_t e = width_cap > 0 ? std::min<int64_t>(len, width_cap) : len;
            w = (int32_t)std::min(wmax, std::max(1.0, std::floor((double)e / mean)));
        }
        g.vw[v] = w;
        sumw += w;
    }
    const int64_t wcap = std::min<int64_t>(max_rows, std::max<int64_t>(
        row_cap, (sumw + nparts - 1) / nparts * (100 + imbalance_pct) / 100));
    if (wcap * nparts < sumw) {
        // partitions already at the LDS row limit: the weights do not fit,
        // balance rows as before
        std::fill(g.vw.begin(), g.vw.end(), 1);
        return row_cap;
    }
    return wcap;
}

}  // namespace

ehyb_status fail(ehyb_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

ehyb_status ok() { return EHYB_OK; }

int64_t algorithmic_bytes(const ehyb_plan& p) {
    int64_t b = 0;
    b += p.ell_slots * (p.vbytes + 2);                 // ELL values + 16-bit columns
    b += p.er_slots * (p.vbytes + 4);                  // residual values + 32-bit columns
    b += (int64_t)p.nslices * 16;                      // ELL slice metadata
    b += (int64_t)p.ner_slices * (8 + 2 * p.C);        // residual slice metadata + row indices
    b += (int64_t)(p.nparts + 1) * 16 + (int64_t)p.nparts * 4;  // partition, slice and halo bounds
    b += (int64_t)p.halo_idx.size() * 4;                         // halo indices
    b += p.n * p.xbytes;                               // x, each element once (slice staging)
    b += p.n * p.xbytes;                               // y, written once
    if (p.n_pieces > 0)                                // wide slices in pieces: piece list,
        b += (int64_t)(p.ner_slices + 1 + p.nparts) * 4 + (int64_t)p.n_pieces * (12 + 2 * 8);  // partial sums out and in
    return b;
}

BlobLayout compute_layout(const ehyb_plan& p) {
    BlobLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += (bytes + kBlobAlign - 1) / kBlobAlign * kBlobAlign;
        return at;
    };
    L.part_start = take((size_t)(p.nparts + 1) * 4);
    L.slice_start = take((size_t)(p.nparts + 1) * 4);
    L.er_slice_start = take((size_t)(p.nparts + 1) * 4);
    L.ell_free = take((size_t)p.nparts * 4);
    L.halo_start = take((size_t)(p.nparts + 1) * 4);
    L.halo_idx = take(p.halo_idx.size() * 4);
    L.ell_meta = take((size_t)p.nslices * 16);
    L.er_meta = take((size_t)p.ner_slices * 8);
    L.er_row = take((size_t)p.ner_slices * p.C * 2);
    L.ell_val = take((size_t)p.ell_slots * p.vbytes);
    L.ell_col = take((size_t)p.ell_slots * 2);
    L.er_val = take((size_t)p.er_slots * p.vbytes);
    L.er_col = take((size_t)p.er_slots * 4);
    L.perm = take((size_t)p.n * 4);
    L.xp = take((size_t)p.n * p.xbytes);
    L.yp = take((size_t)p.n * p.xbytes);
    if (p.n_pieces > 0) {
        L.piece_start = take((size_t)(p.ner_slices + 1) * 4);
        L.piece_nwide = take((size_t)p.nparts * 4);
        L.pieces = take((size_t)p.n_pieces * 12);
        L.ypart = take((size_t)p.n_pieces * 8);
    }
    L.total = off == 0 ? kBlobAlign : off;
    return L;
}

// LDS of one workgroup: x-slice + halo, then one residual accumulator per
// row when the plan has residual entries, each n_rhs elements wide.
int64_t lds_bytes_used(const ehyb_plan& p, int n_rhs) {
    // x-slice and halo, then (8-byte aligned) one residual accumulator per row
    const int64_t xs = ((int64_t)p.max_part_rows + p.max_halo) * p.xbytes * n_rhs;
    const int64_t ab = acc_bytes(p.value_dtype);
    const int64_t acc = p.ner_slices > 0 ? (int64_t)p.max_part_rows * ab * n_rhs : 0;
    return (acc > 0 ? (xs + ab - 1) / ab * ab : xs) + acc;
}

// Pieces of the wide residual slices: slice e of S steps is cut into
// ceil(S / kPieceSteps) pieces of consecutive steps, in slice order.
void build_pieces(ehyb_plan& P) {
    P.piece_start.assign((size_t)P.ner_slices + 1, 0);
    P.pieces.clear();
    int32_t q = 0;
    for (int32_t e = 0; e < P.ner_slices; ++e) {
        P.piece_start[e] = q;
        const uint32_t m = P.er_meta[2 * (size_t)e + 1];
        if (!(m & kErWide)) continue;
        const int32_t steps = (int32_t)(m & ~kErWide);
        for (int32_t t = 0; t < steps; t += kPieceSteps) {
            P.pieces.push_back(e);
            P.pieces.push_back(t);
            P.pieces.push_back(std::min(steps, t + kPieceSteps));
            ++q;
        }
    }
    P.piece_start[P.ner_slices] = q;
    P.n_pieces = q;
    // wide slices lead each partition's residual slices: count that run
    P.piece_nwide.assign((size_t)P.nparts, 0);
    for (int32_t p = 0; p < P.nparts; ++p) {
        int32_t e = P.er_slice_start[p];
        while (e < P.er_slice_start[p + 1] && (P.er_meta[2 * (size_t)e + 1] & kErWide)) ++e;
        P.piece_nwide[p] = e - P.er_slice_start[p];
    }
    if (q == 0) {
        P.piece_start.clear();
        P.piece_nwide.clear();
    }
}

// Residual position of every permuted row (e*C + r, or -1), from er_row.
void build_er_pos(ehyb_plan& P) {
    P.er_pos.assign((size_t)P.n, -1);
    for (int32_t p = 0; p < P.nparts; ++p)
        for (int32_t e = P.er_slice_start[p]; e < P.er_slice_start[p + 1]; ++e)
            for (int32_t r = 0; r < P.C; ++r) {
                const uint16_t lr = P.er_row[(size_t)e * P.C + r];
                if (lr != 0xFFFF) P.er_pos[P.part_start[p] + lr] = e * P.C + r;
            }
}

}  // namespace ehyb

using namespace ehyb;

namespace {

// ELL slot of entry k of row r in a slice with `full` steps of kc entries
// per lane, followed by single-entry steps.
inline int64_t ell_slot_of(int64_t off, int32_t k, int32_t r, int L, int kc, int32_t full) {
    const int64_t kf = (int64_t)full * L * kc;
    if (k < kf) {
        const int64_t t = k / (L * kc), u = (k / kc) % L, c = k % kc;
        return off + (t * kWave + (int64_t)r * L + u) * kc + c;
    }
    const int64_t k1 = k - kf;
    return off + (int64_t)full * kWave * kc + (k1 / L) * kWave + (int64_t)r * L + k1 % L;
}

// Entries per lane of a slice whose longest row has m ELL entries: whole
// steps of L*kc entries, then single-entry steps of L entries for the rest.
inline int64_t ell_width_of(int64_t m, int L, int kc) {
    const int64_t full = m / (L * kc);
    return full * kc + (m - full * L * kc + L - 1) / L;
}

inline int64_t er_slot_of(int64_t off, int32_t k, int32_t r, int L) {
    const int64_t t = k / L, u = k % L;
    return off + t * kWave + (int64_t)r * L + u;
}

// Alg. 1 (classification and reordering) and Alg. 2 (moving entries into the
// ELL and residual parts), given the partition vector.
ehyb_status build_plan(const ehyb_csr_host* A, const std::vector<int32_t>& part, int32_t nparts,
                       int32_t halo_cap, ehyb_plan* P) {
    const int32_t n = (int32_t)A->n_rows;
    const int cap = P->params.ell_width_cap;
    const int L = P->L, C = P->C, kc = P->kc;
    double t0 = now_s();

    // rows of each partition, in original order
    P->part_start.assign(nparts + 1, 0);
    for (int32_t i = 0; i < n; ++i) P->part_start[part[i] + 1]++;
    for (int32_t p = 0; p < nparts; ++p) P->part_start[p + 1] += P->part_start[p];
    P->perm.resize(n);
    {
        std::vector<int32_t> fill(P->part_start.begin(), P->part_start.end() - 1);
        for (int32_t i = 0; i < n; ++i) P->perm[fill[part[i]]++] = i;
    }

    // Halo of each partition: the out-of-partition columns its rows reference,
    // most referenced first, at most halo_cap of them (original indices here).
    std::vector<std::vector<int32_t>> halo(nparts);
    std::vector<int32_t> ell_cnt(n), er_cnt(n);
    OmpGuard guard;
#pragma omp parallel
    {
        std::vector<int32_t> ext;
        std::vector<std::pair<int32_t, int32_t>> cnt;   // (-count, column)
        std::vector<char> in_halo;
        guard.run([&] { in_halo.assign(halo_cap > 0 ? n : 0, 0); });
#pragma omp for schedule(dynamic, 1)
        for (int32_t p = 0; p < nparts; ++p) guard.run([&] {
            auto& h = halo[p];
            if (halo_cap > 0) {
                ext.clear();
                for (int32_t k = P->part_start[p]; k < P->part_start[p + 1]; ++k) {
                    const int32_t i = P->perm[k];
                    for (int64_t q = A->row_ptr[i]; q < A->row_ptr[i + 1]; ++q)
                        if (part[A->col_idx[q]] != p) ext.push_back(A->col_idx[q]);
                }
                std::sort(ext.begin(), ext.end());
                cnt.clear();
                for (size_t a = 0; a < ext.size();) {
                    size_t b = a;
                    while (b < ext.size() && ext[b] == ext[a]) ++b;
                    cnt.emplace_back(-(int32_t)(b - a), ext[a]);
                    a = b;
                }
                if ((int64_t)cnt.size() > halo_cap) {
                    std::sort(cnt.begin(), cnt.end());
                    cnt.resize(halo_cap);
                }
                h.reserve(cnt.size());
                for (const auto& c : cnt) h.push_back(c.second);
                for (int32_t j : h) in_halo[j] = 1;
            }
            // Alg. 1: entries served by the partition's LDS vector (own x-slice
            // or halo) go to the ELL part, the others to the residual part
            for (int32_t k = P->part_start[p]; k < P->part_start[p + 1]; ++k) {
                const int32_t i = P->perm[k];
                int32_t in = 0;
                for (int64_t q = A->row_ptr[i]; q < A->row_ptr[i + 1]; ++q) {
                    const int32_t j = A->col_idx[q];
                    if (part[j] == p || (halo_cap > 0 && in_halo[j])) ++in;
                }
                const int32_t len = (int32_t)(A->row_ptr[i + 1] - A->row_ptr[i]);
                ell_cnt[i] = (cap > 0 && in > cap) ? cap : in;
                er_cnt[i] = len - ell_cnt[i];
            }
            if (halo_cap > 0)
                for (int32_t j : h) in_halo[j] = 0;
        });
    }
    guard.rethrow();
    // each partition's rows by non-increasing ELL count (stable in the
    // original index)
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t p = 0; p < nparts; ++p)
        std::stable_sort(P->perm.begin() + P->part_start[p], P->perm.begin() + P->part_start[p + 1],
                         [&](int32_t a, int32_t b) { return ell_cnt[a] > ell_cnt[b]; });
    P->iperm.resize(n);
    for (int32_t i = 0; i < n; ++i) P->iperm[P->perm[i]] = i;
    // halos in permuted indices, ascending
    P->halo_start.assign(nparts + 1, 0);
    int32_t maxh = 0;
    for (int32_t p = 0; p < nparts; ++p) {
        for (auto& j : halo[p]) j = P->iperm[j];
        std::sort(halo[p].begin(), halo[p].end());
        P->halo_start[p + 1] = P->halo_start[p] + (int32_t)halo[p].size();
        maxh = std::max(maxh, (int32_t)halo[p].size());
    }
    P->max_halo = maxh;
    P->halo_idx.resize(P->halo_start[nparts]);
    for (int32_t p = 0; p < nparts; ++p)
        std::copy(halo[p].begin(), halo[p].end(), P->halo_idx.begin() + P->halo_start[p]);
    P->row_ell_len.resize(n);
    P->row_er_len.resize(n);
    int32_t maxp = 0;
    for (int32_t p = 0; p < nparts; ++p) maxp = std::max(maxp, P->part_start[p + 1] - P->part_start[p]);
    P->max_part_rows = maxp;
    for (int32_t i = 0; i < n; ++i) {
        P->row_ell_len[i] = ell_cnt[P->perm[i]];
        P->row_er_len[i] = er_cnt[P->perm[i]];
    }
    // residual rows of each partition by non-increasing residual count (the
    // extra-rows arrangement of Alg. 1), ties by local row
    P->er_slice_start.assign(nparts + 1, 0);
    std::vector<std::vector<uint16_t>> er_rows(nparts);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t p = 0; p < nparts; ++p) guard.run([&] {
        auto& v = er_rows[p];
        const int32_t ps = P->part_start[p];
        for (int32_t i = ps; i < P->part_start[p + 1]; ++i)
            if (P->row_er_len[i] > 0) v.push_back((uint16_t)(i - ps));
        std::stable_sort(v.begin(), v.end(), [&](uint16_t a, uint16_t b) {
            return P->row_er_len[ps + a] > P->row_er_len[ps + b];
        });
    });
    guard.rethrow();
    // rows longer than kWideSteps steps on their L lanes (the first ones,
    // counts are non-increasing) get a wide slice each; the rest C per slice
    std::vector<int32_t> er_nwide(nparts, 0);
    for (int32_t p = 0; p < nparts; ++p) {
        const int32_t ps = P->part_start[p];
        if (C > 1)
            while (er_nwide[p] < (int32_t)er_rows[p].size() &&
                   P->row_er_len[ps + er_rows[p][er_nwide[p]]] > kWideSteps * L)
                ++er_nwide[p];
        const int64_t rest = (int64_t)er_rows[p].size() - er_nwide[p];
        P->er_slice_start[p + 1] = P->er_slice_start[p] + er_nwide[p] + (int32_t)((rest + C - 1) / C);
    }
    P->nparts = nparts;
    P->ner_slices = P->er_slice_start[nparts];
    P->er_row.assign((size_t)P->ner_slices * C, 0xFFFF);
    for (int32_t p = 0; p < nparts; ++p) {
        const size_t e0 = (size_t)P->er_slice_start[p];
        const int32_t nw = er_nwide[p];
        for (int32_t j = 0; j < nw; ++j) P->er_row[(e0 + j) * C] = er_rows[p][j];
        for (size_t j = nw; j < er_rows[p].size(); ++j) P->er_row[(e0 + nw) * C + (j - nw)] = er_rows[p][j];
    }
    build_er_pos(*P);
    P->t_reorder = now_s() - t0;
    t0 = now_s();

    // ELL row-slices: C consecutive rows of one partition, stored in the order
    // a workgroup takes them: slices without residual rows first
    P->slice_start.assign(nparts + 1, 0);
    for (int32_t p = 0; p < nparts; ++p)
        P->slice_start[p + 1] = P->slice_start[p] + (P->part_start[p + 1] - P->part_start[p] + C - 1) / C;
    const int32_t ns = P->slice_start[nparts];
    P->nslices = ns;
    if (ns > 0 && (P->part_start[nparts] + C - 1) / C > 0) {
        for (int32_t p = 0; p < nparts; ++p)
            if (P->slice_start[p + 1] - P->slice_start[p] > 65535)
                return fail(EHYB_EUNSUPPORTED, "more than 65535 row-slices in one partition");
    }
    std::vector<int32_t> slice_part(ns), slice_j(ns);
    std::vector<int64_t> ell_steps(ns);  // entries per lane of each slice
    std::vector<uint64_t> er_mask(ns, 0);
    P->ell_free.assign(nparts, 0);
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t p = 0; p < nparts; ++p) guard.run([&] {
        const int32_t ps = P->part_start[p], pe = P->part_start[p + 1];
        const int32_t nsp = P->slice_start[p + 1] - P->slice_start[p];
        std::vector<uint64_t> mk(nsp);
        std::vector<int64_t> st(nsp);
        for (int32_t j = 0; j < nsp; ++j) {
            const int32_t r0 = ps + j * C, r1 = std::min(r0 + C, pe);
            int32_t me = 0;
            uint64_t mask = 0;
            for (int32_t r = r0; r < r1; ++r) {
                me = std::max(me, P->row_ell_len[r]);
                if (P->row_er_len[r] > 0) mask |= 1ull << (r - r0);
            }
            mk[j] = mask;
            st[j] = ell_width_of(me, L, kc);
        }
        int32_t at = P->slice_start[p], nfree = 0;
        for (int pass = 0; pass < 2; ++pass)
            for (int32_t j = 0; j < nsp; ++j)
                if ((mk[j] == 0) == (pass == 0)) {
                    slice_part[at] = p;
                    slice_j[at] = j;
                    ell_steps[at] = st[j];
                    er_mask[at] = mk[j];
                    ++at;
                    nfree += pass == 0;
                }
        P->ell_free[p] = nfree;
    });
    guard.rethrow();
    P->ell_meta.assign((size_t)ns * 4, 0);
    // Slot placement.  The kernel reads every slice's offset from its
    // metadata, so the slices need not sit in partition order: they are laid
    // out round by round, the first kPlaceRound slices (in queue order) of
    // every partition, then the next kPlaceRound, and so on.  The slices that
    // all workgroups read at about the same time then share one window of
    // memory instead of forming one stream per workgroup, which a cold DRAM
    // serves faster.
    constexpr int32_t kPlaceRound = 16;
    std::vector<int32_t> place, active(nparts);
    place.reserve((size_t)ns);
    for (int32_t p = 0; p < nparts; ++p) active[p] = p;
    for (int32_t r = 0; !active.empty(); r += kPlaceRound) {
        size_t keep = 0;
        for (const int32_t p : active) {
            const int32_t s1 = std::min(P->slice_start[p] + r + kPlaceRound, P->slice_start[p + 1]);
            for (int32_t s = P->slice_start[p] + r; s < s1; ++s) place.push_back(s);
            if (s1 < P->slice_start[p + 1]) active[keep++] = p;
        }
        active.resize(keep);
    }
    int64_t eoff = 0;
    for (int32_t s : place) {
        if (eoff > UINT32_MAX) return fail(EHYB_EUNSUPPORTED, "more than 2^32 slots in the ELL part");
        if (ell_steps[s] > 65535) return fail(EHYB_EUNSUPPORTED, "ELL row-slice wider than 65535 entries per lane");
        P->ell_meta[4 * (size_t)s + 0] = (uint32_t)eoff;
        P->ell_meta[4 * (size_t)s + 1] = (uint32_t)ell_steps[s] | ((uint32_t)slice_j[s] << 16);
        P->ell_meta[4 * (size_t)s + 2] = (uint32_t)(er_mask[s] & 0xFFFFFFFFu);
        P->ell_meta[4 * (size_t)s + 3] = (uint32_t)(er_mask[s] >> 32);
        eoff += ell_steps[s] * kWave;
    }
    if (eoff > UINT32_MAX) return fail(EHYB_EUNSUPPORTED, "more than 2^32 slots in the ELL part");
    // residual slices
    const int32_t nes = P->ner_slices;
    P->er_meta.assign((size_t)nes * 2, 0);
    int64_t roff = 0;
    {
        std::vector<int32_t> er_steps(nes, 0);
        std::vector<char> wide(nes, 0);
        for (int32_t p = 0; p < nparts; ++p) {
            const int32_t ps = P->part_start[p];
            for (int32_t e = P->er_slice_start[p]; e < P->er_slice_start[p + 1]; ++e) {
                wide[e] = e - P->er_slice_start[p] < er_nwide[p];
                int32_t mr = 0;
                for (int32_t r = 0; r < C; ++r) {
                    const uint16_t lr = P->er_row[(size_t)e * C + r];
                    if (lr != 0xFFFF) mr = std::max(mr, P->row_er_len[ps + lr]);
                }
                er_steps[e] = wide[e] ? (mr + kWave - 1) / kWave : (mr + L - 1) / L;
            }
        }
        for (int32_t e = 0; e < nes; ++e) {
            if (roff > UINT32_MAX) return fail(EHYB_EUNSUPPORTED, "more than 2^32 slots in the residual part");
            P->er_meta[2 * (size_t)e + 0] = (uint32_t)roff;
            P->er_meta[2 * (size_t)e + 1] = (uint32_t)er_steps[e] | (wide[e] ? kErWide : 0u);
            roff += (int64_t)er_steps[e] * kWave;
            P->n_er_wide += wide[e];
        }
    }
    if (roff > UINT32_MAX) return fail(EHYB_EUNSUPPORTED, "more than 2^32 slots in the residual part");
    P->ell_slots = eoff;
    P->er_slots = roff;
    build_pieces(*P);
    const int vb = P->vbytes, dt = P->value_dtype;
    P->ell_val.assign((size_t)eoff * vb, 0);   // +0.0 padding in every value type
    P->ell_col.assign((size_t)eoff, 0);
    P->er_val.assign((size_t)roff * vb, 0);
    P->er_col.assign((size_t)roff, 0);

    // Alg. 2: move each entry, with its column renumbered by the reorder
    // table, into its slot
    int64_t nnz_ell = 0, nnz_er = 0, n_er_rows = 0, nnz_halo = 0;
#pragma omp parallel reduction(+ : nnz_ell, nnz_er, n_er_rows, nnz_halo)
    {
        std::vector<std::pair<int32_t, int64_t>> ent;  // (new column, source position)
#pragma omp for schedule(dynamic, 64)
        for (int32_t s = 0; s < ns; ++s) guard.run([&] {
            const int32_t p = slice_part[s];
            const int32_t ps = P->part_start[p], pe = P->part_start[p + 1];
            const int32_t r0 = ps + slice_j[s] * C;
            const int32_t r1 = std::min(r0 + C, pe);
            const int64_t eo = P->ell_meta[4 * (size_t)s + 0];
            const int32_t full = (int32_t)(P->ell_meta[4 * (size_t)s + 1] & 0xFFFFu) / kc;
            for (int32_t row = r0; row < r1; ++row) {
                const int32_t r = row - r0;
                const int32_t old = P->perm[row];
                ent.clear();
                for (int64_t q = A->row_ptr[old]; q < A->row_ptr[old + 1]; ++q)
                    ent.emplace_back(P->iperm[A->col_idx[q]], q);
                std::sort(ent.begin(), ent.end());
                int32_t k1 = 0, k2 = 0;
                const int32_t ell_len = P->row_ell_len[row];
                const int32_t ep = P->er_pos[row];
                const int64_t ro = ep >= 0 ? (int64_t)P->er_meta[2 * (size_t)(ep / C)] : 0;
                const bool ew = ep >= 0 && (P->er_meta[2 * (size_t)(ep / C) + 1] & kErWide);
                const int32_t rr = ep >= 0 ? ep % C : 0;
                const int32_t* hb = P->halo_idx.data() + P->halo_start[p];
                const int32_t* he = P->halo_idx.data() + P->halo_start[p + 1];
                for (const auto& pr : ent) {
                    const int32_t nc = pr.first;
                    const double v = A->val[pr.second];
                    int32_t local = -1;
                    if (nc >= ps && nc < pe) {
                        local = nc - ps;
                    } else {
                        const int32_t* f = std::lower_bound(hb, he, nc);
                        if (f != he && *f == nc) local = (pe - ps) + (int32_t)(f - hb);
                    }
                    if (local >= 0 && k1 < ell_len) {
                        const int64_t slot = ell_slot_of(eo, k1++, r, L, kc, full);
                        store_value(&P->ell_val[(size_t)slot * vb], vb, dt, v);
                        P->ell_col[slot] = (uint16_t)local;
                        if (local >= pe - ps) ++nnz_halo;
                    } else {
                        const int64_t slot = ew ? er_slot_of(ro, k2++, 0, kWave) : er_slot_of(ro, k2++, rr, L);
                        store_value(&P->er_val[(size_t)slot * vb], vb, dt, v);
                        P->er_col[slot] = nc;
                    }
                }
                nnz_ell += k1;
                nnz_er += k2;
                n_er_rows += k2 > 0;
            }
        });
    }
    guard.rethrow();
    P->nnz_ell = nnz_ell;
    P->nnz_er = nnz_er;
    P->n_er_rows = n_er_rows;
    P->nnz_halo = nnz_halo;
    P->t_encode = now_s() - t0;
    return EHYB_OK;
}

}  // namespace

extern "C" {

const char* ehyb_last_error(void) { return g_last_error.c_str(); }

const char* ehyb_version(void) { return "0.2.0"; }

}  // extern "C"

namespace {

// Preprocessing with the built-in partitioner (given == nullptr) or with the
// caller's partition vector.
ehyb_status preprocess_impl(const ehyb_csr_host* A, const ehyb_params* params, const int32_t* given,
                            int32_t given_nparts, ehyb_plan** out) {
    try {
        g_last_error.clear();
        if (!A || !out) return fail(EHYB_EINVAL, "null argument");
        *out = nullptr;
        ehyb_params prm{};
        if (params) prm = *params;
        Error e = validate(A);
        if (!e.ok()) return fail(e.status, e.msg);
        if (prm.halo_rows < -1) return fail(EHYB_EINVAL, "halo_rows must be >= -1");
        if (prm.reserved != 0) return fail(EHYB_EINVAL, "reserved parameter field must be 0");
        if (prm.n_rhs == 0) prm.n_rhs = 1;
        if (prm.n_rhs != 1 && prm.n_rhs != 2 && prm.n_rhs != 4 && prm.n_rhs != 8)
            return fail(EHYB_EINVAL, "n_rhs must be 1, 2, 4 or 8");
        if (!valid_dtype(prm.value_dtype)) return fail(EHYB_EINVAL, "unknown value dtype");
        if (prm.rows_per_wave == 0) prm.rows_per_wave = kWave;
        if (prm.rows_per_wave < 1 || prm.rows_per_wave > kWave ||
            (prm.rows_per_wave & (prm.rows_per_wave - 1)))
            return fail(EHYB_EINVAL, "rows_per_wave must be a power of two in [1, 64]");
        if (prm.lds_bytes == 0) prm.lds_bytes = 160 * 1024;
        if (prm.lds_bytes < 64 || prm.lds_bytes > 160 * 1024)
            return fail(EHYB_EINVAL, "lds_bytes must be in [64, 163840]");
        if (prm.num_cus == 0) prm.num_cus = 256;
        if (prm.num_cus < 1) return fail(EHYB_EINVAL, "num_cus must be positive");
        if (prm.imbalance_pct == 0) prm.imbalance_pct = 3;
        if (prm.imbalance_pct < 0 || prm.imbalance_pct > 100)
            return fail(EHYB_EINVAL, "imbalance_pct must be in [0, 100]");
        if (prm.ell_width_cap < -1) return fail(EHYB_EINVAL, "ell_width_cap must be >= -1");
        if (prm.partitioner < 0 || prm.partitioner > 1) return fail(EHYB_EINVAL, "unknown partitioner");
        if (prm.n_threads < 0) return fail(EHYB_EINVAL, "n_threads must be >= 0");

        auto P = std::unique_ptr<ehyb_plan>(new ehyb_plan());
        const int64_t n = A->n_rows;
        P->n = n;
        P->nnz = A->nnz;
        P->value_dtype = prm.value_dtype;
        P->vbytes = value_bytes(prm.value_dtype);
        P->xbytes = x_bytes(prm.value_dtype);
        P->C = prm.rows_per_wave;
        P->L = kWave / prm.rows_per_wave;
        P->kc = kc_for(prm.value_dtype);
        // LDS per partition row: its x elements and its residual accumulators
        P->n_rhs = prm.n_rhs;
        // LDS per partition row: its x element and its residual accumulator
        const int64_t tau = ((int64_t)P->xbytes + acc_bytes(prm.value_dtype)) * prm.n_rhs;
        // (8-byte accumulators after 4-byte x elements may need 4 bytes of alignment)
        const int64_t align_pad = acc_bytes(prm.value_dtype) > P->xbytes ? acc_bytes(prm.value_dtype) - P->xbytes : 0;
        const int64_t max_rows = std::min<int64_t>(65535, (prm.lds_bytes - kStaticLds - align_pad) / tau);
        if (max_rows < 1) return fail(EHYB_EINVAL, "lds_bytes smaller than one partition row");
        // Eq. 1-2: smallest K with n*tau/(K*P) < SHM, VecSize = ceil(n/(K*P))
        int64_t K = 1;
        while (n * tau >= (int64_t)prm.lds_bytes * K * prm.num_cus) ++K;
        P->eq1_K = (int32_t)K;
        const int64_t vec = n > 0 ? (n + K * prm.num_cus - 1) / (K * prm.num_cus) : 0;
        if (prm.slice_rows == 0)
            prm.slice_rows = (int32_t)std::max<int64_t>(
                1, std::min<int64_t>(max_rows, std::max<int64_t>(vec, std::min<int64_t>(n, 512))));
        if (prm.slice_rows < 1) return fail(EHYB_EINVAL, "slice_rows must be >= 1");
        if (prm.slice_rows > max_rows)
            return fail(EHYB_EINVAL, "slice_rows exceeds the LDS budget (x element + accumulator per row) or 65535 rows");
        const int64_t cap = std::min<int64_t>(max_rows, prm.slice_rows + (int64_t)prm.slice_rows * prm.imbalance_pct / 100);
        const int32_t nparts_req = n > 0 ? (int32_t)((n + prm.slice_rows - 1) / prm.slice_rows) : 0;
        // ELL width cap: -1 none (the paper's split), > 0 as given, 0 the
        // automatic cap of kAutoCapSteps load steps per row-slice lane group
        // (only hub rows reach it; their excess goes to wide residual slices)
        if (prm.ell_width_cap == 0) prm.ell_width_cap = kAutoCapSteps * P->L * P->kc;
        else if (prm.ell_width_cap < 0) prm.ell_width_cap = 0;
        P->params = prm;
        ThreadGuard tg(threads_for(prm));

        std::vector<int32_t> part;
        int32_t nparts = nparts_req;
        double t0 = now_s();
        if (given) {
            // caller's partition: ids in [0, given_nparts), every partition
            // within the LDS budget; empty ids are dropped, order kept
            if (given_nparts < 1 && n > 0) return fail(EHYB_EINVAL, "n_parts must be >= 1");
            std::vector<int64_t> cnt(std::max(given_nparts, 0), 0);
            for (int64_t i = 0; i < n; ++i) {
                if (given[i] < 0 || given[i] >= given_nparts)
                    return fail(EHYB_EINVAL, "partition id out of range at row " + std::to_string(i));
                cnt[given[i]]++;
            }
            std::vector<int32_t> remap(cnt.size(), -1);
            nparts = 0;
            int64_t largest = 0;
            for (size_t q = 0; q < cnt.size(); ++q) {
                if (cnt[q] > max_rows)
                    return fail(EHYB_EINVAL, "partition " + std::to_string(q) + " exceeds the LDS budget");
                if (cnt[q] > 0) remap[q] = nparts++;
                largest = std::max(largest, cnt[q]);
            }
            P->params.slice_rows = (int32_t)std::max<int64_t>(1, largest);
            part.resize(n);
            for (int64_t i = 0; i < n; ++i) part[i] = remap[given[i]];
            P->t_graph = 0;
            P->t_partition = now_s() - t0;
        } else if (prm.partitioner == EHYB_PART_NATURAL || nparts_req <= 1) {
            part.resize(n);
            for (int64_t i = 0; i < n; ++i) part[i] = (int32_t)(i / prm.slice_rows);
            P->t_graph = 0;
            P->t_partition = now_s() - t0;
        } else {
            Graph g = build_graph(A);
            P->t_graph = now_s() - t0;
            t0 = now_s();
            const int64_t wcap = weigh_long_rows(g, A, prm.ell_width_cap, nparts_req, cap, max_rows, prm.imbalance_pct);
            Error pe = partition_multilevel(g, nparts_req, wcap, prm.seed, part, nparts);
            if (!pe.ok()) return fail(pe.status, pe.msg);
            P->t_partition = now_s() - t0;
        }
        // halo room: the LDS vector holds x-slice + halo, plus one residual
        // accumulator per row
        int32_t halo_cap = 0;
        if (prm.halo_rows >= 0) {
            int32_t maxp = 0;
            {
                std::vector<int32_t> sizes(nparts, 0);
                for (int64_t i = 0; i < n; ++i) sizes[part[i]]++;
                for (int32_t s2 : sizes) maxp = std::max(maxp, s2);
            }
            const int64_t room =
                acc_bytes(prm.value_dtype) == P->xbytes
                    ? (int64_t)(prm.lds_bytes - kStaticLds) / ((int64_t)P->xbytes * prm.n_rhs) - 2 * (int64_t)maxp
                    : ((int64_t)(prm.lds_bytes - kStaticLds - align_pad) / prm.n_rhs -
                       (int64_t)maxp * (P->xbytes + acc_bytes(prm.value_dtype))) / P->xbytes;
            halo_cap = (int32_t)std::max<int64_t>(0, std::min<int64_t>(room, 65535 - (int64_t)maxp));
            if (prm.halo_rows > 0) halo_cap = std::min(halo_cap, prm.halo_rows);
        }
        ehyb_status st = build_plan(A, part, nparts, halo_cap, P.get());
        if (st != EHYB_OK) return st;
        *out = P.release();
        return EHYB_OK;
    } catch (const std::bad_alloc&) {
        return fail(EHYB_ENOMEM, "host allocation failed during preprocessing");
    } catch (const std::exception& ex) {
        return fail(EHYB_EINVAL, std::string("preprocessing failed: ") + ex.what());
    }
}

}  // namespace

extern "C" {

ehyb_status ehyb_preprocess(const ehyb_csr_host* A, const ehyb_params* params, ehyb_plan** out) {
    return preprocess_impl(A, params, nullptr, 0, out);
}

ehyb_status ehyb_preprocess_partitioned(const ehyb_csr_host* A, const ehyb_params* params,
                                        const int32_t* part, int32_t n_parts, ehyb_plan** out) {
    if (!part && A && A->n_rows > 0) return fail(EHYB_EINVAL, "null partition vector");
    static const int32_t none = 0;
    return preprocess_impl(A, params, part ? part : &none, n_parts, out);
}

ehyb_status ehyb_plan_stats_get(const ehyb_plan* P, ehyb_plan_stats* out) {
    if (!P || !out) return fail(EHYB_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->n = P->n;
    out->nnz = P->nnz;
    out->nnz_ell = P->nnz_ell;
    out->nnz_er = P->nnz_er;
    out->ell_slots = P->ell_slots;
    out->er_slots = P->er_slots;
    out->n_er_rows = P->n_er_rows;
    out->n_er_wide = P->n_er_wide;
    out->n_er_pieces = P->n_pieces;
    out->ell_width_cap = P->params.ell_width_cap;
    out->nnz_halo = P->nnz_halo;
    out->n_halo = (int64_t)P->halo_idx.size();
    out->max_halo = P->max_halo;
    out->lds_bytes_used = (int32_t)lds_bytes_used(*P);
    out->n_rhs = P->n_rhs;
    out->device_bytes = (int64_t)compute_layout(*P).total;
    out->algorithmic_bytes = algorithmic_bytes(*P);
    out->nparts = P->nparts;
    out->nslices = P->nslices;
    out->ner_slices = P->ner_slices;
    out->slice_rows = P->params.slice_rows;
    out->max_part_rows = P->max_part_rows;
    out->rows_per_slice = P->C;
    out->lanes_per_row = P->L;
    out->kc = P->kc;
    out->value_dtype = P->value_dtype;
    out->eq1_K = P->eq1_K;
    out->t_graph_s = P->t_graph;
    out->t_partition_s = P->t_partition;
    out->t_reorder_s = P->t_reorder;
    out->t_encode_s = P->t_encode;
    return EHYB_OK;
}

ehyb_status ehyb_plan_arrays_get(const ehyb_plan* P, ehyb_plan_arrays* out) {
    if (!P || !out) return fail(EHYB_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->n = P->n;
    out->nparts = P->nparts;
    out->nslices = P->nslices;
    out->ner_slices = P->ner_slices;
    out->lanes_per_row = P->L;
    out->kc = P->kc;
    out->value_dtype = P->value_dtype;
    out->ell_slots = P->ell_slots;
    out->er_slots = P->er_slots;
    out->perm = P->perm.data();
    out->part_start = P->part_start.data();
    out->slice_start = P->slice_start.data();
    out->er_slice_start = P->er_slice_start.data();
    out->ell_free = P->ell_free.data();
    out->halo_start = P->halo_start.data();
    out->halo_idx = P->halo_idx.data();
    out->n_halo = (int64_t)P->halo_idx.size();
    out->ell_meta = P->ell_meta.data();
    out->er_meta = P->er_meta.data();
    out->er_row = P->er_row.data();
    out->ell_val = P->ell_val.data();
    out->ell_col = P->ell_col.data();
    out->er_val = P->er_val.data();
    out->er_col = P->er_col.data();
    out->row_ell_len = P->row_ell_len.data();
    out->row_er_len = P->row_er_len.data();
    return EHYB_OK;
}

ehyb_status ehyb_plan_decode_csr(const ehyb_plan* P, int64_t* row_ptr, int32_t* col_idx, double* val) {
    if (!P || !row_ptr || (P->nnz > 0 && (!col_idx || !val))) return fail(EHYB_EINVAL, "null argument");
    const int32_t n = (int32_t)P->n;
    const int L = P->L, C = P->C, kc = P->kc, vb = P->vbytes, dt = P->value_dtype;
    row_ptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + P->row_ell_len[i] + P->row_er_len[i];
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t p = 0; p < P->nparts; ++p) {
        const int32_t ps = P->part_start[p], pe = P->part_start[p + 1];
        for (int32_t s = P->slice_start[p]; s < P->slice_start[p + 1]; ++s) {
            const int64_t eo = P->ell_meta[4 * (size_t)s + 0];
            const int32_t r0 = ps + (int32_t)(P->ell_meta[4 * (size_t)s + 1] >> 16) * C;
            const int32_t full = (int32_t)(P->ell_meta[4 * (size_t)s + 1] & 0xFFFFu) / kc;
            for (int32_t r = 0; r < C && r0 + r < pe; ++r) {
                const int32_t row = r0 + r;
                int64_t out_at = row_ptr[row];
                int32_t a = 0, b = 0;
                const int32_t na = P->row_ell_len[row], nb = P->row_er_len[row];
                const int32_t ep = P->er_pos[row];
                const int64_t ro = ep >= 0 ? (int64_t)P->er_meta[2 * (size_t)(ep / C)] : 0;
                const bool ew = ep >= 0 && (P->er_meta[2 * (size_t)(ep / C) + 1] & kErWide);
                const int32_t rr = ep >= 0 ? ep % C : 0;
                while (a < na || b < nb) {
                    const int64_t sa = a < na ? ell_slot_of(eo, a, r, L, kc, full) : 0;
                    const int64_t sb = b < nb ? (ew ? er_slot_of(ro, b, 0, kWave) : er_slot_of(ro, b, rr, L)) : 0;
                    int32_t ca = INT32_MAX;
                    if (a < na) {
                        const int32_t lc = P->ell_col[sa];
                        ca = lc < pe - ps ? ps + lc : P->halo_idx[P->halo_start[p] + lc - (pe - ps)];
                    }
                    const int32_t cb = b < nb ? P->er_col[sb] : INT32_MAX;
                    if (ca < cb) {
                        col_idx[out_at] = ca;
                        val[out_at] = load_value(&P->ell_val[(size_t)sa * vb], dt);
                        ++a;
                    } else {
                        col_idx[out_at] = cb;
                        val[out_at] = load_value(&P->er_val[(size_t)sb * vb], dt);
                        ++b;
                    }
                    ++out_at;
                }
            }
        }
    }
    return EHYB_OK;
}

ehyb_status ehyb_plan_device_bytes(const ehyb_plan* P, size_t* bytes) {
    if (!P || !bytes) return fail(EHYB_EINVAL, "null argument");
    *bytes = compute_layout(*P).total;
    return EHYB_OK;
}

void ehyb_plan_destroy(ehyb_plan* P) { delete P; }

}  // extern "C"

// ------------------------------------------------------------- plan files
// Layout: magic "EHYBPLN6", u32 version, then fixed header fields and arrays
// (each prefixed by its u64 byte length), then a u64 FNV-1a checksum of all
// preceding bytes.

namespace {
const char kMagic[8] = {'E', 'H', 'Y', 'B', 'P', 'L', 'N', '6'};
const uint32_t kVersion = 6;

uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 1469598103934665603ull) {
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

struct Writer {
    std::vector<unsigned char> buf;
    void raw(const void* p, size_t n) {
        const unsigned char* c = (const unsigned char*)p;
        buf.insert(buf.end(), c, c + n);
    }
    template <class T> void pod(const T& v) { raw(&v, sizeof(T)); }
    template <class T> void vec(const std::vector<T>& v) {
        uint64_t b = v.size() * sizeof(T);
        pod(b);
        raw(v.data(), b);
    }
};

struct Reader {
    const unsigned char* p;
    size_t n, at = 0;
    bool ok = true;
    void raw(void* d, size_t k) {
        if (!ok || at + k > n) {
            ok = false;
            return;
        }
        if (k) std::memcpy(d, p + at, k);  // an empty vector's data() may be null
        at += k;
    }
    template <class T> void pod(T& v) { raw(&v, sizeof(T)); }
    template <class T> void vec(std::vector<T>& v, uint64_t max_elems) {
        uint64_t b = 0;
        pod(b);
        if (!ok || b % sizeof(T) || b / sizeof(T) > max_elems || at + b > n) {
            ok = false;
            return;
        }
        v.resize(b / sizeof(T));
        raw(v.data(), b);
    }
};

// Every bound a kernel relies on, checked on a loaded plan.
const char* validate_loaded(const ehyb_plan& P) {
    const size_t n = (size_t)P.n;
    const int C = P.C;
    if (P.perm.size() != n || P.part_start.size() != (size_t)P.nparts + 1 ||
        P.slice_start.size() != (size_t)P.nparts + 1 || P.er_slice_start.size() != (size_t)P.nparts + 1 ||
        P.ell_free.size() != (size_t)P.nparts || P.halo_start.size() != (size_t)P.nparts + 1 ||
        P.ell_meta.size() != (size_t)P.nslices * 4 || P.er_meta.size() != (size_t)P.ner_slices * 2 ||
        P.er_row.size() != (size_t)P.ner_slices * C ||
        P.ell_val.size() != (size_t)P.ell_slots * P.vbytes || P.ell_col.size() != (size_t)P.ell_slots ||
        P.er_val.size() != (size_t)P.er_slots * P.vbytes || P.er_col.size() != (size_t)P.er_slots ||
        P.row_ell_len.size() != n || P.row_er_len.size() != n)
        return "plan file array sizes are inconsistent";
    if (P.nparts > 0 && (P.part_start[0] != 0 || P.part_start[P.nparts] != (int32_t)n || P.slice_start[0] != 0 ||
                         P.slice_start[P.nparts] != P.nslices || P.er_slice_start[0] != 0 ||
                         P.er_slice_start[P.nparts] != P.ner_slices))
        return "plan file partition bounds are inconsistent";
    if (P.nparts == 0 && n != 0) return "plan file has rows but no partitions";
    if (P.nparts > 0 && (P.halo_start[0] != 0 || (size_t)P.halo_start[P.nparts] != P.halo_idx.size()))
        return "plan file halo bounds are inconsistent";
    int32_t maxh = 0;
    for (int32_t p = 0; p < P.nparts; ++p) {
        const int32_t hs = P.halo_start[p], he = P.halo_start[p + 1];
        if (he < hs) return "plan file halo bounds decrease";
        maxh = std::max(maxh, he - hs);
        for (int32_t k = hs; k < he; ++k) {
            const int32_t j = P.halo_idx[k];
            if (j < 0 || (size_t)j >= n || (j >= P.part_start[p] && j < P.part_start[p + 1]) ||
                (k > hs && j <= P.halo_idx[k - 1]))
                return "plan file halo is invalid";
        }
    }
    if (maxh != P.max_halo) return "plan file largest halo is inconsistent";
    if (lds_bytes_used(P, P.n_rhs) > 160 * 1024 - kStaticLds) return "plan file needs more LDS than a workgroup has";
    const int64_t max_rows = std::min<int64_t>(
        65535, (int64_t)(160 * 1024 - kStaticLds - (acc_bytes(P.value_dtype) > P.xbytes ? 4 : 0)) /
                   (((int64_t)P.xbytes + acc_bytes(P.value_dtype)) * P.n_rhs));
    for (int32_t p = 0; p < P.nparts; ++p) {
        const int64_t sz = (int64_t)P.part_start[p + 1] - P.part_start[p];
        const int64_t sl = (int64_t)P.slice_start[p + 1] - P.slice_start[p];
        const int64_t el = (int64_t)P.er_slice_start[p + 1] - P.er_slice_start[p];
        if (sz <= 0 || sz > max_rows || sl != (sz + C - 1) / C || el < 0 || el > sz)
            return "plan file partition sizes are inconsistent";
        if (P.ell_free[p] < 0 || P.ell_free[p] > sl) return "plan file ELL free-slice count is inconsistent";
        std::vector<char> seen_j((size_t)sl, 0);
        for (int32_t s = P.slice_start[p]; s < P.slice_start[p + 1]; ++s) {
            const uint64_t eo = P.ell_meta[4 * (size_t)s], ew = P.ell_meta[4 * (size_t)s + 1] & 0xFFFFu;
            const int64_t j = P.ell_meta[4 * (size_t)s + 1] >> 16;
            if (j >= sl || seen_j[(size_t)j]) return "plan file ELL slice indices are not a permutation";
            seen_j[(size_t)j] = 1;
            if (eo + ew * kWave > (uint64_t)P.ell_slots) return "plan file ELL slot range out of bounds";
            const int64_t ext = sz + P.halo_start[p + 1] - P.halo_start[p];
            for (uint64_t q = eo; q < eo + ew * kWave; ++q)
                if (P.ell_col[q] >= ext) return "plan file ELL column outside its LDS vector";
            const uint64_t mask = (uint64_t)P.ell_meta[4 * (size_t)s + 2] | ((uint64_t)P.ell_meta[4 * (size_t)s + 3] << 32);
            const int64_t rows = std::min<int64_t>(C, sz - j * C);
            for (int64_t r = 0; r < rows; ++r)
                if (P.row_ell_len[P.part_start[p] + j * C + r] > (int64_t)ew * P.L)
                    return "plan file row has more ELL entries than its slice holds";
            if (rows < 64 && (mask >> rows) != 0) return "plan file residual mask names a missing row";
        }
        for (int32_t e = P.er_slice_start[p]; e < P.er_slice_start[p + 1]; ++e) {
            const uint64_t ro = P.er_meta[2 * (size_t)e], rs = P.er_meta[2 * (size_t)e + 1] & ~kErWide;
            const bool wide = (P.er_meta[2 * (size_t)e + 1] & kErWide) != 0;
            if (ro + rs * kWave > (uint64_t)P.er_slots) return "plan file residual slot range out of bounds";
            if (wide && C == 1) return "plan file has a wide residual slice with one row per slice";
            for (int r = 0; r < C; ++r) {
                const uint16_t lr = P.er_row[(size_t)e * C + r];
                if (lr != 0xFFFF && lr >= sz) return "plan file residual row outside its partition";
                if (lr != 0xFFFF && P.row_er_len[P.part_start[p] + lr] > (int64_t)rs * (wide ? kWave : P.L))
                    return "plan file row has more residual entries than its slice holds";
                if (wide && (r == 0) != (lr != 0xFFFF)) return "plan file wide residual slice must hold one row";
            }
        }
    }
    for (size_t s = 0; s < P.er_col.size(); ++s)
        if (P.er_col[s] < 0 || (size_t)P.er_col[s] >= n) return "plan file residual column out of range";
    std::vector<char> seen(n, 0);
    for (size_t i = 0; i < n; ++i) {
        const int32_t o = P.perm[i];
        if (o < 0 || (size_t)o >= n || seen[o]) return "plan file permutation is invalid";
        seen[o] = 1;
    }
    return nullptr;
}
}  // namespace

extern "C" {

ehyb_status ehyb_plan_save(const ehyb_plan* P, const char* path) {
    try {
        if (!P || !path) return fail(EHYB_EINVAL, "null argument");
        Writer w;
        w.raw(kMagic, 8);
        w.pod(kVersion);
        w.pod(P->n);
        w.pod(P->nnz);
        w.pod(P->params);
        w.pod(P->L);
        w.pod(P->C);
        w.pod(P->kc);
        w.pod(P->nparts);
        w.pod(P->nslices);
        w.pod(P->ner_slices);
        w.pod(P->value_dtype);
        w.pod(P->eq1_K);
        w.pod(P->max_part_rows);
        w.pod(P->ell_slots);
        w.pod(P->er_slots);
        w.pod(P->nnz_ell);
        w.pod(P->nnz_er);
        w.pod(P->n_er_rows);
        w.pod(P->nnz_halo);
        w.pod(P->max_halo);
        w.vec(P->perm);
        w.vec(P->part_start);
        w.vec(P->slice_start);
        w.vec(P->er_slice_start);
        w.vec(P->ell_free);
        w.vec(P->halo_start);
        w.vec(P->halo_idx);
        w.vec(P->ell_meta);
        w.vec(P->er_meta);
        w.vec(P->er_row);
        w.vec(P->ell_val);
        w.vec(P->ell_col);
        w.vec(P->er_val);
        w.vec(P->er_col);
        w.vec(P->row_ell_len);
        w.vec(P->row_er_len);
        uint64_t h = fnv1a(w.buf.data(), w.buf.size());
        w.pod(h);
        FILE* f = std::fopen(path, "wb");
        if (!f) return fail(EHYB_EINVAL, std::string("cannot open ") + path + " for writing");
        size_t wr = std::fwrite(w.buf.data(), 1, w.buf.size(), f);
        int cl = std::fclose(f);
        if (wr != w.buf.size() || cl != 0) return fail(EHYB_EINVAL, "short write to plan file");
        return EHYB_OK;
    } catch (const std::bad_alloc&) {
        return fail(EHYB_ENOMEM, "host allocation failed while saving");
    }
}

ehyb_status ehyb_plan_load(const char* path, ehyb_plan** out) {
    try {
        if (!path || !out) return fail(EHYB_EINVAL, "null argument");
        *out = nullptr;
        FILE* f = std::fopen(path, "rb");
        if (!f) return fail(EHYB_EINVAL, std::string("cannot open ") + path);
        std::vector<unsigned char> buf;
        unsigned char tmp[1 << 16];
        size_t k;
        while ((k = std::fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + k);
        std::fclose(f);
        if (buf.size() < 8 + 4 + 8) return fail(EHYB_EINVAL, "plan file truncated");
        uint64_t h;
        std::memcpy(&h, buf.data() + buf.size() - 8, 8);
        if (fnv1a(buf.data(), buf.size() - 8) != h) return fail(EHYB_EINVAL, "plan file checksum mismatch");
        Reader r{buf.data(), buf.size() - 8};
        char magic[8];
        uint32_t ver = 0;
        r.raw(magic, 8);
        r.pod(ver);
        if (!r.ok || std::memcmp(magic, kMagic, 8) != 0) return fail(EHYB_EINVAL, "not a plan file");
        if (ver != kVersion) return fail(EHYB_EINVAL, "unsupported plan file version");
        auto P = std::unique_ptr<ehyb_plan>(new ehyb_plan());
        r.pod(P->n);
        r.pod(P->nnz);
        r.pod(P->params);
        r.pod(P->L);
        r.pod(P->C);
        r.pod(P->kc);
        r.pod(P->nparts);
        r.pod(P->nslices);
        r.pod(P->ner_slices);
        r.pod(P->value_dtype);
        r.pod(P->eq1_K);
        r.pod(P->max_part_rows);
        r.pod(P->ell_slots);
        r.pod(P->er_slots);
        r.pod(P->nnz_ell);
        r.pod(P->nnz_er);
        r.pod(P->n_er_rows);
        r.pod(P->nnz_halo);
        r.pod(P->max_halo);
        if (!r.ok || P->n < 0 || P->n > INT32_MAX || P->nparts < 0 || P->nslices < 0 || P->ner_slices < 0 ||
            !valid_dtype(P->value_dtype) || P->L < 1 || P->L > kWave || P->C * P->L != kWave ||
            P->kc != kc_for(P->value_dtype) || P->ell_slots < 0 || P->er_slots < 0 || P->max_part_rows < 0)
            return fail(EHYB_EINVAL, "plan file header is inconsistent");
        P->vbytes = value_bytes(P->value_dtype);
        P->xbytes = x_bytes(P->value_dtype);
        P->n_rhs = P->params.n_rhs;
        if (P->n_rhs != 1 && P->n_rhs != 2 && P->n_rhs != 4 && P->n_rhs != 8)
            return fail(EHYB_EINVAL, "plan file right-hand side count is invalid");
        const uint64_t lim = (uint64_t)buf.size();
        r.vec(P->perm, lim);
        r.vec(P->part_start, lim);
        r.vec(P->slice_start, lim);
        r.vec(P->er_slice_start, lim);
        r.vec(P->ell_free, lim);
        r.vec(P->halo_start, lim);
        r.vec(P->halo_idx, lim);
        r.vec(P->ell_meta, lim);
        r.vec(P->er_meta, lim);
        r.vec(P->er_row, lim);
        r.vec(P->ell_val, lim);
        r.vec(P->ell_col, lim);
        r.vec(P->er_val, lim);
        r.vec(P->er_col, lim);
        r.vec(P->row_ell_len, lim);
        r.vec(P->row_er_len, lim);
        if (!r.ok || r.at != r.n) return fail(EHYB_EINVAL, "plan file body is malformed");
        if (const char* why = validate_loaded(*P)) return fail(EHYB_EINVAL, why);
        int32_t maxp = 0;
        for (int32_t p = 0; p < P->nparts; ++p) maxp = std::max(maxp, P->part_start[p + 1] - P->part_start[p]);
        if (maxp != P->max_part_rows) return fail(EHYB_EINVAL, "plan file largest partition is inconsistent");
        P->iperm.resize((size_t)P->n);
        for (size_t i = 0; i < (size_t)P->n; ++i) P->iperm[P->perm[i]] = (int32_t)i;
        build_er_pos(*P);
        build_pieces(*P);
        P->n_er_wide = 0;
        for (int32_t e = 0; e < P->ner_slices; ++e) P->n_er_wide += (P->er_meta[2 * (size_t)e + 1] & kErWide) != 0;
        *out = P.release();
        return EHYB_OK;
    } catch (const std::bad_alloc&) {
        return fail(EHYB_ENOMEM, "host allocation failed while loading");
    }
}

}  // extern "C"
