// Host-only driver for allocation failures: the global operator new is
// replaced by one that throws std::bad_alloc at the k-th allocation after a
// countdown is armed.  Each host entry point (preprocessing, re-encoding from a
// partition, features, decode, save, load) runs once to count its
// allocations, then again with the failure placed at allocations spread over
// that count: every run must return EHYB_OK or EHYB_ENOMEM (never abort, never
// another status), leave no plan behind on failure, and leak nothing (the
// test builds this with AddressSanitizer and leak detection).
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "ehyb.h"

static std::atomic<long> g_left{-1};      // allocations until the failure; < 0: disarmed
static std::atomic<long> g_count{0};      // allocations seen while counting
static std::atomic<bool> g_counting{false};

static void* take(std::size_t n) {
    if (g_counting.load(std::memory_order_relaxed)) g_count.fetch_add(1, std::memory_order_relaxed);
    if (g_left.load(std::memory_order_relaxed) >= 0 && g_left.fetch_sub(1) == 0) throw std::bad_alloc();
    void* p = std::malloc(n ? n : 1);
    if (!p) throw std::bad_alloc();
    return p;
}
void* operator new(std::size_t n) { return take(n); }
void* operator new[](std::size_t n) { return take(n); }
void* operator new(std::size_t n, const std::nothrow_t&) noexcept {
    try { return take(n); } catch (...) { return nullptr; }
}
void* operator new[](std::size_t n, const std::nothrow_t&) noexcept {
    try { return take(n); } catch (...) { return nullptr; }
}
void operator delete(void* p) noexcept { std::free(p); }
void operator delete[](void* p) noexcept { std::free(p); }
void operator delete(void* p, std::size_t) noexcept { std::free(p); }
void operator delete[](void* p, std::size_t) noexcept { std::free(p); }

static void csr_random(int n, int deg, unsigned seed, std::vector<int64_t>& rp, std::vector<int32_t>& ci,
                       std::vector<double>& v) {
    std::mt19937 g(seed);
    std::vector<std::vector<int32_t>> rows(n);
    for (int i = 0; i < n; ++i) {
        rows[i].push_back(i);
        const int d = i < 2 ? n / 4 : (int)(g() % (2 * deg + 1));  // two hub rows
        for (int k = 0; k < d; ++k) rows[i].push_back((int32_t)(g() % n));
    }
    for (int i = 0; i < n; ++i)
        for (size_t k = 1; k < rows[i].size() && k < 4; ++k) rows[rows[i][k]].push_back(i);
    rp.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        auto& r = rows[i];
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        for (int32_t c : r) {
            ci.push_back(c);
            v.push_back((double)(g() % 1000) / 997.0 - 0.5);
        }
        rp[i + 1] = (int64_t)ci.size();
    }
}

static int g_bad = 0, g_enomem = 0, g_ok = 0;

// Run `f` (returning a status) with a failure at each of up to `tries`
// allocation indices spread over its allocation count.
template <class F>
static void sweep(const char* what, F f, int tries) {
    g_count = 0;
    g_counting = true;
    ehyb_status st = f();
    g_counting = false;
    const long total = g_count.load();
    if (st != EHYB_OK) {
        std::printf("%s: failed without injection: %s\n", what, ehyb_last_error());
        ++g_bad;
        return;
    }
    int en = 0;
    for (int t = 0; t < tries; ++t) {
        const long k = total <= tries ? t : (long)((double)t * (double)total / tries);
        if (k >= total) break;
        g_left = k;
        st = f();
        g_left = -1;
        if (st == EHYB_ENOMEM) {
            ++g_enomem;
            ++en;
        } else if (st == EHYB_OK) {
            ++g_ok;
        } else {
            std::printf("%s: allocation %ld failed -> status %d (%s)\n", what, k, (int)st, ehyb_last_error());
            ++g_bad;
        }
    }
    std::printf("%s: %ld allocations, %d injected failures reported EHYB_ENOMEM\n", what, total, en);
    if (total > 0 && en == 0) ++g_bad;  // a sweep over allocations must have hit one
}

int main(int argc, char** argv) {
    const int tries = argc > 1 ? std::atoi(argv[1]) : 60;
    const std::string path = argc > 2 ? argv[2] : "alloc_fail_plan.bin";
    const int n = 3000;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
    csr_random(n, 6, 7, rp, ci, v);
    ehyb_csr_host A{n, n, (int64_t)ci.size(), rp.data(), ci.data(), v.data()};
    for (int cfg = 0; cfg < 3; ++cfg) {
        ehyb_params p{};
        p.slice_rows = cfg == 1 ? 256 : 0;
        p.rows_per_wave = cfg == 2 ? 16 : 0;
        p.halo_rows = cfg == 0 ? -1 : 0;
        p.value_dtype = cfg;
        sweep("preprocess", [&] {
            ehyb_plan* P = nullptr;
            const ehyb_status st = ehyb_preprocess(&A, &p, &P);
            if (st != EHYB_OK && P != nullptr) {
                std::printf("preprocess: a plan was returned with status %d\n", (int)st);
                ++g_bad;
            }
            ehyb_plan_destroy(P);
            return st;
        }, tries);
        ehyb_plan* P = nullptr;
        if (ehyb_preprocess(&A, &p, &P) != EHYB_OK) return 2;
        ehyb_plan_arrays ar;
        ehyb_plan_arrays_get(P, &ar);
        std::vector<int32_t> part(n);
        for (int q = 0; q < ar.nparts; ++q)
            for (int i = ar.part_start[q]; i < ar.part_start[q + 1]; ++i) part[ar.perm[i]] = q;
        sweep("preprocess_partitioned", [&] {
            ehyb_plan* Q = nullptr;
            const ehyb_status st = ehyb_preprocess_partitioned(&A, &p, part.data(), ar.nparts, &Q);
            ehyb_plan_destroy(Q);
            return st;
        }, tries);
        std::vector<int64_t> orp(n + 1);
        std::vector<int32_t> oci(ci.size());
        std::vector<double> ov(ci.size());
        sweep("decode", [&] { return ehyb_plan_decode_csr(P, orp.data(), oci.data(), ov.data()); }, tries);
        sweep("save", [&] { return ehyb_plan_save(P, path.c_str()); }, tries);
        sweep("load", [&] {
            ehyb_plan* R = nullptr;
            const ehyb_status st = ehyb_plan_load(path.c_str(), &R);
            ehyb_plan_destroy(R);
            return st;
        }, tries);
        ehyb_plan_destroy(P);
    }
    float f[32];
    sweep("features", [&] { return ehyb_features(&A, 0, f); }, tries);
    std::printf("ok=%d enomem=%d bad=%d\n", g_ok, g_enomem, g_bad);
    return g_bad != 0;
}
