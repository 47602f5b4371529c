// Sparsity features of a CSR matrix, the input of the learned parameter
// predictor.  The paper chooses the partition size by a fixed rule (Eq. 1)
// and mentions learned format selection only as related work; the predictor
// replaces the rule with a small network evaluated on these 32 numbers.
// Every feature is an O(nnz) (symmetry: O(nnz log d)) pass over the pattern
// as given; values are ignored.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

using namespace ehyb;

namespace {

constexpr int64_t kColBlock = 4096;   // column / row block of the spread features
constexpr int64_t kNearBlock = 512;   // aligned block of the locality feature

// Lower quantile of sorted v: v[floor(q (n-1))].
double quantile(const std::vector<int64_t>& sorted, double q) {
    if (sorted.empty()) return 0.0;
    const size_t k = (size_t)std::floor(q * (double)(sorted.size() - 1));
    return (double)sorted[k];
}

}  // namespace

extern "C" EHYB_API ehyb_status ehyb_features(const ehyb_csr_host* A, int32_t n_threads, float* out) {
    try {
        if (!A || !out) return fail(EHYB_EINVAL, "null argument");
        if (n_threads < 0) return fail(EHYB_EINVAL, "n_threads must be >= 0");
        if (A->n_rows < 1 || A->n_rows != A->n_cols) return fail(EHYB_EINVAL, "matrix must be square with n >= 1");
        if (!A->row_ptr || (A->nnz > 0 && !A->col_idx)) return fail(EHYB_EINVAL, "null row_ptr or col_idx");
        if (A->row_ptr[0] != 0 || A->row_ptr[A->n_rows] != A->nnz) return fail(EHYB_EINVAL, "row_ptr does not span nnz");
        const int64_t n = A->n_rows, nnz = A->nnz;
        const int64_t* rp = A->row_ptr;
        const int32_t* ci = A->col_idx;
        for (int64_t i = 0; i < n; ++i)
            if (rp[i + 1] < rp[i]) return fail(EHYB_EINVAL, "row_ptr decreases");
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                if (ci[p] < 0 || ci[p] >= n) return fail(EHYB_EINVAL, "column index out of range");
                if (p > rp[i] && ci[p] <= ci[p - 1])
                    return fail(EHYB_EINVAL, "columns not strictly increasing (unsorted or duplicate)");
            }
        const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();

        std::vector<int64_t> len(n), bw(n);
        double s_abs = 0, max_abs = 0;
        int64_t near4096 = 0, near512 = 0, diag = 0, blocks = 0, sym = 0, offd = 0;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 2048) \
    reduction(+ : s_abs, near4096, near512, diag, blocks, sym, offd) reduction(max : max_abs)
        for (int64_t i = 0; i < n; ++i) {
            len[i] = rp[i + 1] - rp[i];
            int64_t b = 0, last_blk = -1;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                const int64_t j = ci[p];
                const int64_t d = j > i ? j - i : i - j;
                s_abs += (double)d;
                max_abs = std::max(max_abs, (double)d);
                b = std::max(b, d);
                near4096 += d < kColBlock;
                near512 += (i / kNearBlock) == (j / kNearBlock);
                if (j == i) {
                    ++diag;
                } else {
                    ++offd;
                    // is (j, i) stored?
                    sym += std::binary_search(ci + rp[j], ci + rp[j + 1], (int32_t)i);
                }
                const int64_t blk = j / kColBlock;
                if (blk != last_blk) {
                    // distinct column blocks of the row (columns ascend: count changes)
                    ++blocks;
                    last_blk = blk;
                }
            }
            bw[i] = b;
        }
        const double dn = (double)n, dnnz = (double)nnz;
        const double mu = dnnz / dn;
        double m2 = 0, m3 = 0;
        int64_t empty = 0, heavy = 0;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : m2, m3, empty, heavy)
        for (int64_t i = 0; i < n; ++i) {
            const double d = (double)len[i] - mu;
            m2 += d * d;
            m3 += d * d * d;
            empty += len[i] == 0;
            heavy += (double)len[i] > 2.0 * mu;
        }
        const double sd = std::sqrt(m2 / dn);
        std::vector<int64_t> sl(len);
        std::sort(sl.begin(), sl.end());
        std::vector<int64_t> sbw(bw);
        std::sort(sbw.begin(), sbw.end());
        // Gini coefficient of the row lengths (ascending order, 1-based rank)
        double gnum = 0;
        for (int64_t k = 0; k < n; ++k) gnum += (double)(2 * (k + 1) - n - 1) * (double)sl[k];
        // share of the entries in the longest ceil(n/100) rows
        const int64_t top = (n + 99) / 100;
        double topsum = 0;
        for (int64_t k = n - top; k < n; ++k) topsum += (double)sl[k];
        // column spread of each 4096-row block
        const int64_t nb = (n + kColBlock - 1) / kColBlock;
        std::vector<double> spread(nb);
        OmpGuard guard;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
        for (int64_t rb = 0; rb < nb; ++rb) guard.run([&] {
            std::vector<char> seen(nb, 0);
            int64_t cnt = 0;
            for (int64_t i = rb * kColBlock; i < std::min(n, (rb + 1) * kColBlock); ++i)
                for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                    const int64_t b = ci[p] / kColBlock;
                    if (!seen[b]) {
                        seen[b] = 1;
                        ++cnt;
                    }
                }
            spread[rb] = (double)cnt / (double)nb;
        });
        guard.rethrow();
        double sp_mean = 0, sp_max = 0;
        for (double v : spread) {
            sp_mean += v;
            sp_max = std::max(sp_max, v);
        }
        sp_mean /= (double)nb;
        const double p99 = quantile(sl, 0.99);
        double pad = 0, beyond = 0;
        for (int64_t i = 0; i < n; ++i) {
            pad += p99 - std::min<double>((double)len[i], p99);
            beyond += std::max<double>((double)len[i] - p99, 0.0);
        }
        const double nz1 = std::max(dnnz, 1.0);

        double f[32];
        f[0] = std::log2(dn);
        f[1] = std::log2(dnnz + 1.0);
        f[2] = mu;
        f[3] = sd;
        f[4] = mu > 0 ? sd / mu : 0.0;
        f[5] = (double)sl.front();
        f[6] = (double)sl.back();
        f[7] = std::log2((double)sl.back() + 1.0);
        f[8] = quantile(sl, 0.10);
        f[9] = quantile(sl, 0.25);
        f[10] = quantile(sl, 0.50);
        f[11] = quantile(sl, 0.75);
        f[12] = quantile(sl, 0.90);
        f[13] = p99;
        f[14] = sd > 0 ? (m3 / dn) / (sd * sd * sd) : 0.0;
        f[15] = (double)empty / dn;
        f[16] = (double)heavy / dn;
        f[17] = nnz > 0 ? s_abs / dnnz / dn : 0.0;
        f[18] = max_abs / dn;
        f[19] = quantile(sbw, 0.90) / dn;
        f[20] = (double)near4096 / nz1;
        f[21] = (double)blocks / dn;
        f[22] = sp_mean;
        f[23] = sp_max;
        f[24] = offd > 0 ? (double)sym / (double)offd : 1.0;
        f[25] = (double)diag / dn;
        f[26] = nnz > 0 ? gnum / (dn * dnnz) : 0.0;
        f[27] = topsum / nz1;
        f[28] = mu / 64.0;
        f[29] = pad / nz1;
        f[30] = beyond / nz1;
        f[31] = (double)near512 / nz1;
        for (int k = 0; k < 32; ++k) out[k] = (float)f[k];
        return ok();
    } catch (const std::bad_alloc&) {
        return fail(EHYB_ENOMEM, "host allocation failed");
    }
}
