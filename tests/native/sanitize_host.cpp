// Host-only driver: preprocessing, decode, re-encoding from a given partition,
// save/load and features on random matrices (some with hub rows), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <random>
#include <algorithm>
#include "ehyb.h"
static void csr_random(int n, int deg, unsigned seed, bool hub, std::vector<int64_t>& rp, std::vector<int32_t>& ci, std::vector<double>& v) {
    std::mt19937 g(seed);
    std::vector<std::vector<int32_t>> rows(n);
    for (int i = 0; i < n; ++i) {
        rows[i].push_back(i);
        int d = hub && i < 3 ? n / 3 : (int)(g() % (2 * deg + 1));
        for (int k = 0; k < d; ++k) rows[i].push_back((int32_t)(g() % n));
    }
    // symmetrize a little
    for (int i = 0; i < n; ++i) for (size_t k = 1; k < rows[i].size() && k < 4; ++k) rows[rows[i][k]].push_back(i);
    rp.assign(n + 1, 0); ci.clear(); v.clear();
    for (int i = 0; i < n; ++i) {
        auto& r = rows[i]; std::sort(r.begin(), r.end()); r.erase(std::unique(r.begin(), r.end()), r.end());
        for (int32_t c : r) { ci.push_back(c); v.push_back((double)(g() % 1000) / 997.0 - 0.5); }
        rp[i + 1] = (int64_t)ci.size();
    }
}
int main(int argc, char** argv) {
    const int ntrials = argc > 1 ? atoi(argv[1]) : 6;
    int fails = 0;
    const char* path = argc > 2 ? argv[2] : "sanitize_plan.bin";
    for (int trial = 0; trial < ntrials; ++trial) {
        const int n = 200 + 977 * trial;
        std::vector<int64_t> rp; std::vector<int32_t> ci; std::vector<double> v;
        csr_random(n, 3 + trial % 5, 100 + trial, trial % 3 == 0, rp, ci, v);
        ehyb_csr_host A{n, n, (int64_t)ci.size(), rp.data(), ci.data(), v.data()};
        for (int cfg = 0; cfg < 6; ++cfg) {
            ehyb_params p{};
            p.slice_rows = cfg % 2 ? 128 : 0;
            p.rows_per_wave = (int[]){64, 8, 16, 1, 32, 4}[cfg];
            p.halo_rows = cfg % 3 == 0 ? -1 : 0;
            p.ell_width_cap = cfg == 4 ? 5 : (cfg == 5 ? -1 : 0);
            p.value_dtype = cfg % 3;
            p.n_rhs = (cfg == 2) ? 4 : 0;
            ehyb_plan* P = nullptr;
            if (ehyb_preprocess(&A, &p, &P) != EHYB_OK) { printf("preprocess failed %d %d: %s\n", trial, cfg, ehyb_last_error()); ++fails; continue; }
            std::vector<int64_t> orp(n + 1); std::vector<int32_t> oci(ci.size()); std::vector<double> ov(ci.size());
            if (ehyb_plan_decode_csr(P, orp.data(), oci.data(), ov.data()) != EHYB_OK) { printf("decode failed\n"); ++fails; }
            ehyb_plan_arrays ar; ehyb_plan_arrays_get(P, &ar);
            std::vector<int32_t> part(n);
            for (int q = 0; q < ar.nparts; ++q) for (int i = ar.part_start[q]; i < ar.part_start[q + 1]; ++i) part[ar.perm[i]] = q;
            ehyb_plan* Q = nullptr;
            p.rows_per_wave = 16;
            if (ehyb_preprocess_partitioned(&A, &p, part.data(), ar.nparts, &Q) != EHYB_OK) { printf("partitioned failed: %s\n", ehyb_last_error()); ++fails; }
            if (ehyb_plan_save(P, path) != EHYB_OK) { printf("save failed\n"); ++fails; }
            ehyb_plan* R = nullptr;
            if (ehyb_plan_load(path, &R) != EHYB_OK) { printf("load failed: %s\n", ehyb_last_error()); ++fails; }
            ehyb_plan_destroy(R); ehyb_plan_destroy(Q); ehyb_plan_destroy(P);
        }
        float f[32];
        if (ehyb_features(&A, 0, f) != EHYB_OK) { printf("features failed\n"); ++fails; }
        printf("trial %d n=%d nnz=%zu ok\n", trial, n, ci.size());
    }
    printf("fails=%d\n", fails);
    return fails != 0;
}
