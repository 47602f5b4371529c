// Multilevel k-way graph partitioner with a hard cap on part weight.
//
// Section 3.1 of the paper partitions the graph of A (vertices = row/column
// indices, edges = stored entries) so that most entries join two vertices of
// the same partition; it calls a multi-threaded METIS for this.  No METIS is
// available here, so this file implements the same family of algorithm from
// the published multilevel scheme (coarsen by heavy-edge matching, partition
// the coarsest graph by recursive bisection with greedy graph growing and
// Fiduccia-Mattheyses refinement, then project back level by level with
// greedy k-way boundary refinement).  Unlike METIS's soft imbalance factor,
// the cap here is hard: a partition's x-slice must fit the on-chip budget.
//
// Edge weights count stored entries: an undirected edge {i, j} weighs 1 if
// only one of a_ij, a_ji is stored and 2 if both are, so the weight of the
// cut equals the number of entries that land in the residual part.
//
// The paper's partitioner is multi-threaded and its reordering is named as the
// preprocessing bottleneck (Section 4); here every phase over the whole graph
// runs on all host threads: matching, contraction, k-way refinement, and the
// two halves of every bisection.  Each parallel step is written so that the
// result depends on the seed only, never on the number of threads or their
// timing: matching pairs vertices that choose each other, refinement computes
// moves from a snapshot and accepts them in a fixed order, and every node of
// the bisection tree draws from its own random stream.
#include <omp.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <queue>

#include "internal.h"

namespace ehyb {

int64_t Graph::total_vw() const {
    int64_t s = 0;
    for (int32_t w : vw) s += w;
    return s;
}

namespace {

struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull) {}
    uint64_t next() {  // splitmix64
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    uint32_t below(uint32_t n) { return n ? (uint32_t)(next() % n) : 0; }
    void shuffle(std::vector<int32_t>& v) {
        for (size_t i = v.size(); i > 1; --i) std::swap(v[i - 1], v[below((uint32_t)i)]);
    }
};

// Stateless 64-bit mix (the splitmix64 finaliser) for per-vertex tie-breaks and
// per-task seeds.
inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

std::vector<int32_t> random_order(int32_t n, Rng& rng) {
    std::vector<int32_t> p(n);
    std::iota(p.begin(), p.end(), 0);
    rng.shuffle(p);
    return p;
}

// ---------------------------------------------------------------- coarsening
// Heavy-edge matching in rounds: every unmatched vertex picks the unmatched
// neighbour joined by the heaviest edge (then the lighter one, then a seeded
// per-vertex hash) whose combined weight stays under maxvw; two vertices that
// picked each other are matched.  A final pass in vertex order pairs what is
// left greedily.  Then the matched pairs are contracted; a coarse vertex's
// edges keep the order in which they are first met.
Graph coarsen(const Graph& g, int32_t maxvw, uint64_t key, std::vector<int32_t>& cmap) {
    const int32_t n = g.n;
    std::vector<int32_t> match(n, -1), pref(n, -1);
    auto better = [&](int32_t u, int32_t w, int32_t best, int32_t bestw) {
        if (best < 0 || w > bestw) return true;
        if (w < bestw) return false;
        if (g.vw[u] != g.vw[best]) return g.vw[u] < g.vw[best];
        return mix64(key ^ (uint64_t)u) > mix64(key ^ (uint64_t)best);
    };
    for (int round = 0; round < 4; ++round) {
        int64_t matched = 0;
#pragma omp parallel for schedule(dynamic, 4096)
        for (int32_t v = 0; v < n; ++v) {
            int32_t best = -1, bestw = -1;
            if (match[v] == -1) {
                for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
                    const int32_t u = g.adj[e];
                    if (match[u] != -1 || u == v || g.vw[v] + g.vw[u] > maxvw) continue;
                    if (better(u, g.ew[e], best, bestw)) {
                        best = u;
                        bestw = g.ew[e];
                    }
                }
            }
            pref[v] = best;
        }
#pragma omp parallel for schedule(static) reduction(+ : matched)
        for (int32_t v = 0; v < n; ++v) {
            const int32_t u = pref[v];
            if (u >= 0 && pref[u] == v) {
                match[v] = u;
                ++matched;
            }
        }
        if (matched * 50 < n) break;
    }
    for (int32_t v = 0; v < n; ++v) {
        if (match[v] != -1) continue;
        int32_t best = -1, bestw = -1;
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
            const int32_t u = g.adj[e];
            if (match[u] != -1 || u == v || g.vw[v] + g.vw[u] > maxvw) continue;
            if (better(u, g.ew[e], best, bestw)) {
                best = u;
                bestw = g.ew[e];
            }
        }
        match[v] = best >= 0 ? best : v;
        if (best >= 0) match[best] = v;
    }
    cmap.assign(n, -1);
    std::vector<int32_t> rep;
    rep.reserve(n / 2 + 1);
    int32_t nc = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (v <= match[v]) {
            cmap[v] = nc;
            cmap[match[v]] = nc;
            rep.push_back(v);
            ++nc;
        }
    }
    // contraction: each coarse vertex writes into a slot range sized by the
    // degrees of its two members, then the ranges are packed
    std::vector<int64_t> ub(nc + 1, 0);
    for (int32_t ci = 0; ci < nc; ++ci) {
        const int32_t v = rep[ci], u = match[v];
        ub[ci + 1] = ub[ci] + (g.xadj[v + 1] - g.xadj[v]) + (u != v ? g.xadj[u + 1] - g.xadj[u] : 0);
    }
    uvec<int32_t> tadj(ub[nc]), tew(ub[nc]), cnt(nc);
    Graph c;
    c.n = nc;
    c.vw.assign(nc, 0);
    OmpGuard guard;
#pragma omp parallel
    {
        std::vector<int64_t> marker;
        guard.run([&] { marker.assign(nc, -1); });
#pragma omp for schedule(dynamic, 1024)
        for (int32_t ci = 0; ci < nc; ++ci) {
            if (guard.failed()) continue;
            const int64_t start = ub[ci];
            int64_t end = start;
            const int32_t v = rep[ci], u = match[v];
            c.vw[ci] = g.vw[v] + (u != v ? g.vw[u] : 0);
            for (int k = 0; k < (u != v ? 2 : 1); ++k) {
                const int32_t w = k == 0 ? v : u;
                for (int64_t e = g.xadj[w]; e < g.xadj[w + 1]; ++e) {
                    const int32_t cu = cmap[g.adj[e]];
                    if (cu == ci) continue;
                    if (marker[cu] >= start) {
                        tew[marker[cu]] += g.ew[e];
                    } else {
                        marker[cu] = end;
                        tadj[end] = cu;
                        tew[end] = g.ew[e];
                        ++end;
                    }
                }
            }
            cnt[ci] = (int32_t)(end - start);
        }
    }
    guard.rethrow();
    c.xadj.assign(nc + 1, 0);
    for (int32_t ci = 0; ci < nc; ++ci) c.xadj[ci + 1] = c.xadj[ci] + cnt[ci];
    c.adj.resize(c.xadj[nc]);
    c.ew.resize(c.xadj[nc]);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t ci = 0; ci < nc; ++ci) {
        std::copy(tadj.begin() + ub[ci], tadj.begin() + ub[ci] + cnt[ci], c.adj.begin() + c.xadj[ci]);
        std::copy(tew.begin() + ub[ci], tew.begin() + ub[ci] + cnt[ci], c.ew.begin() + c.xadj[ci]);
    }
    return c;
}

// Induced subgraph on the vertices with keep[v] == side; returns local->global ids.
Graph induced(const Graph& g, const std::vector<int8_t>& side, int8_t which,
              std::vector<int32_t>& ids) {
    std::vector<int32_t> loc(g.n, -1);
    ids.clear();
    for (int32_t v = 0; v < g.n; ++v)
        if (side[v] == which) {
            loc[v] = (int32_t)ids.size();
            ids.push_back(v);
        }
    Graph s;
    s.n = (int32_t)ids.size();
    s.xadj.assign(s.n + 1, 0);
    s.vw.resize(s.n);
    for (int32_t i = 0; i < s.n; ++i) {
        const int32_t v = ids[i];
        s.vw[i] = g.vw[v];
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
            const int32_t u = loc[g.adj[e]];
            if (u >= 0) {
                s.adj.push_back(u);
                s.ew.push_back(g.ew[e]);
            }
        }
        s.xadj[i + 1] = (int64_t)s.adj.size();
    }
    return s;
}

int64_t cut_2way(const Graph& g, const std::vector<int8_t>& side) {
    int64_t cut = 0;
    for (int32_t v = 0; v < g.n; ++v)
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e)
            if (side[g.adj[e]] != side[v]) cut += g.ew[e];
    return cut / 2;
}

struct HeapItem {
    int64_t gain;
    int32_t v;
    bool operator<(const HeapItem& o) const { return gain < o.gain || (gain == o.gain && v > o.v); }
};

// Two-way Fiduccia-Mattheyses refinement with roll-back to the best prefix.
// Side 0 weight w0 must stay within [lo, hi].
void fm_2way(const Graph& g, std::vector<int8_t>& side, int64_t lo, int64_t hi, Rng& rng) {
    const int32_t n = g.n;
    std::vector<int64_t> gain(n);
    std::vector<char> locked(n);
    int64_t w0 = 0;
    for (int32_t v = 0; v < n; ++v)
        if (side[v] == 0) w0 += g.vw[v];
    for (int pass = 0; pass < 10; ++pass) {
        std::fill(locked.begin(), locked.end(), 0);
        std::priority_queue<HeapItem> q[2];
        for (int32_t v = 0; v < n; ++v) {
            int64_t ext = 0, in = 0;
            for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e)
                (side[g.adj[e]] != side[v] ? ext : in) += g.ew[e];
            gain[v] = ext - in;
            if (ext > 0) q[side[v]].push({gain[v], v});
        }
        std::vector<int32_t> moves;
        int64_t cut = cut_2way(g, side), best_cut = cut;
        int64_t best_dev = w0 < lo ? lo - w0 : (w0 > hi ? w0 - hi : 0);
        size_t best_len = 0;
        const size_t patience = (size_t)std::max<int64_t>(64, n / 50);
        while (true) {
            int32_t cand[2] = {-1, -1};
            for (int s = 0; s < 2; ++s) {
                while (!q[s].empty()) {
                    HeapItem it = q[s].top();
                    if (locked[it.v] || side[it.v] != s || it.gain != gain[it.v]) {
                        q[s].pop();
                        continue;
                    }
                    const int64_t nw0 = s == 0 ? w0 - g.vw[it.v] : w0 + g.vw[it.v];
                    const int64_t dev_now = w0 < lo ? lo - w0 : (w0 > hi ? w0 - hi : 0);
                    const int64_t dev_new = nw0 < lo ? lo - nw0 : (nw0 > hi ? nw0 - hi : 0);
                    if (dev_new > 0 && dev_new >= dev_now) {
                        q[s].pop();  // infeasible now; may come back after neighbours move
                        continue;
                    }
                    cand[s] = it.v;
                    break;
                }
            }
            int32_t v;
            if (cand[0] < 0 && cand[1] < 0) break;
            if (cand[0] < 0) v = cand[1];
            else if (cand[1] < 0) v = cand[0];
            else if (gain[cand[0]] != gain[cand[1]]) v = gain[cand[0]] > gain[cand[1]] ? cand[0] : cand[1];
            else v = (w0 > (lo + hi) / 2) ? cand[0] : cand[1];
            const int s = side[v];
            q[s].pop();
            locked[v] = 1;
            side[v] = (int8_t)(1 - s);
            w0 += s == 0 ? -g.vw[v] : g.vw[v];
            cut -= gain[v];
            gain[v] = -gain[v];
            moves.push_back(v);
            for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
                const int32_t u = g.adj[e];
                if (locked[u]) continue;
                // v left side s: edges to u on side s are now external, to u on the other side internal
                gain[u] += (side[u] == s ? 2 : -2) * (int64_t)g.ew[e];
                q[side[u]].push({gain[u], u});
            }
            const int64_t dev = w0 < lo ? lo - w0 : (w0 > hi ? w0 - hi : 0);
            if (dev < best_dev || (dev == best_dev && cut < best_cut)) {
                best_cut = cut;
                best_dev = dev;
                best_len = moves.size();
            } else if (moves.size() - best_len > patience) {
                break;
            }
        }
        for (size_t i = moves.size(); i > best_len; --i) {
            const int32_t v = moves[i - 1];
            w0 += side[v] == 0 ? -g.vw[v] : g.vw[v];
            side[v] = (int8_t)(1 - side[v]);
        }
        if (best_len == 0) break;
    }
    (void)rng;
}

// Greedy graph growing from a random seed, then FM; best of several trials.
// The trials run as separate tasks, each with its own generator drawn from
// `rng`; ties between trials go to the lower trial index.
void grow_and_refine(const Graph& g, int64_t target0, int64_t lo, int64_t hi, Rng& rng,
                     std::vector<int8_t>& side) {
    const int32_t n = g.n;
    side.assign(n, 1);
    std::vector<int64_t> gain(n, 0);
    std::priority_queue<HeapItem> q;
    int64_t w0 = 0;
    int32_t scan = (int32_t)rng.below((uint32_t)n);
    while (w0 < target0) {
        int32_t v = -1;
        while (!q.empty()) {
            HeapItem it = q.top();
            q.pop();
            if (side[it.v] == 1 && it.gain == gain[it.v]) {
                v = it.v;
                break;
            }
        }
        if (v < 0) {  // new component or first seed
            for (int32_t k = 0; k < n; ++k) {
                const int32_t c = (scan + k) % n;
                if (side[c] == 1) {
                    v = c;
                    scan = c;
                    break;
                }
            }
            if (v < 0) break;
        }
        if (w0 + g.vw[v] > hi && w0 >= lo) break;
        side[v] = 0;
        w0 += g.vw[v];
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
            const int32_t u = g.adj[e];
            if (side[u] == 1) {
                gain[u] += 2 * (int64_t)g.ew[e];
                q.push({gain[u], u});
            }
        }
    }
    fm_2way(g, side, lo, hi, rng);
}

void bisect(const Graph& g, int64_t target0, int64_t lo, int64_t hi, Rng& rng,
            std::vector<int8_t>& best_side, OmpGuard& guard) {
    const int32_t n = g.n;
    const int trials = n > 20000 ? 3 : 6;
    std::vector<uint64_t> seeds(trials);
    for (auto& s : seeds) s = rng.next();
    std::vector<std::vector<int8_t>> sides(trials);
    std::vector<int64_t> cut(trials), dev(trials);
    for (int t = 0; t < trials; ++t) {
#pragma omp task default(shared) firstprivate(t) if (g.xadj[n] > 20000)
        guard.run([&] {
            Rng r(seeds[t]);
            grow_and_refine(g, target0, lo, hi, r, sides[t]);
            int64_t wz = 0;
            for (int32_t v = 0; v < n; ++v)
                if (sides[t][v] == 0) wz += g.vw[v];
            dev[t] = wz < lo ? lo - wz : (wz > hi ? wz - hi : 0);
            cut[t] = cut_2way(g, sides[t]);
        });
    }
#pragma omp taskwait
    if (guard.failed()) return;
    int best = 0;
    for (int t = 1; t < trials; ++t)
        if (dev[t] < dev[best] || (dev[t] == dev[best] && cut[t] < cut[best])) best = t;
    best_side.swap(sides[best]);
}

// Recursive bisection of g into parts [p0, p0 + k); writes part[ids[v]].
// Each node of the bisection tree seeds its own generator from (key, p0, k),
// and the two halves run as separate tasks.
void recursive_bisection(const Graph& g, const std::vector<int32_t>& ids, int32_t p0, int32_t k,
                         uint64_t key, std::vector<int32_t>& part, OmpGuard& guard) {
    if (k == 1 || g.n == 0) {
        for (int32_t v = 0; v < g.n; ++v) part[ids[v]] = p0;
        return;
    }
    Rng rng(mix64(key ^ mix64(((uint64_t)(uint32_t)p0 << 32) | (uint32_t)k)));
    const int32_t k1 = k / 2;
    const int64_t W = g.total_vw();
    const int64_t target0 = (W * k1 + k / 2) / k;
    int32_t maxw = 0;
    for (int32_t w : g.vw) maxw = std::max(maxw, w);
    const int64_t delta = std::max<int64_t>(maxw, (int64_t)(0.003 * (double)W));
    std::vector<int8_t> side;
    bisect(g, target0, std::max<int64_t>(0, target0 - delta), target0 + delta, rng, side, guard);
    if (guard.failed()) return;
    for (int8_t s = 0; s < 2; ++s) {
#pragma omp task default(shared) firstprivate(s) if (g.n > 512)
        guard.run([&] {
            std::vector<int32_t> loc_ids;
            Graph sub = induced(g, side, s, loc_ids);
            for (auto& v : loc_ids) v = ids[v];
            recursive_bisection(sub, loc_ids, s == 0 ? p0 : p0 + k1, s == 0 ? k1 : k - k1, key, part, guard);
        });
    }
#pragma omp taskwait
}

// Connectivity of v to the parts around it: returns own-part weight (ID),
// fills touched parts and conn[] (caller clears conn for touched entries).
inline int64_t connectivity(const Graph& g, const std::vector<int32_t>& part, int32_t v,
                            std::vector<int64_t>& conn, std::vector<int32_t>& touched) {
    touched.clear();
    const int32_t own = part[v];
    int64_t id = 0;
    for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
        const int32_t q = part[g.adj[e]];
        if (q == own) {
            id += g.ew[e];
            continue;
        }
        if (conn[q] == 0) touched.push_back(q);
        conn[q] += g.ew[e];
    }
    return id;
}

// Greedy k-way boundary refinement under the hard cap, in parallel.  A pass
// has two half-passes, one that only moves vertices to parts of higher id and
// one to lower id (so two neighbours never swap parts in one step).  In a
// half-pass every vertex computes its best move against a snapshot of the
// partition and part weights; the proposals are then accepted in a fixed
// order (by target part, larger gain first, then vertex id) while the target
// stays within the cap and the source keeps a vertex.
struct Move {
    int32_t v, q;
    int64_t gain;
};

void refine_kway(const Graph& g, std::vector<int32_t>& part, int32_t nparts, int64_t cap,
                 int max_passes) {
    std::vector<int64_t> pw(nparts, 0);
    for (int32_t v = 0; v < g.n; ++v) pw[part[v]] += g.vw[v];
    const int nt = omp_get_max_threads();
    std::vector<std::vector<Move>> local(nt);
    std::vector<Move> props;
    std::vector<int64_t> win(nparts), wout(nparts);
    for (int pass = 0; pass < max_passes; ++pass) {
        int64_t moves = 0;
        for (int dir = 0; dir < 2; ++dir) {
            OmpGuard guard;
#pragma omp parallel num_threads(nt)
            {
                std::vector<int64_t> conn;
                std::vector<int32_t> touched;
                std::vector<Move>& mine = local[omp_get_thread_num()];
                mine.clear();
                guard.run([&] { conn.assign(nparts, 0); });
#pragma omp for schedule(dynamic, 2048)
                for (int32_t v = 0; v < g.n; ++v) guard.run([&] {
                    const int32_t own = part[v];
                    const int64_t id = connectivity(g, part, v, conn, touched);
                    if (touched.empty()) return;
                    int32_t best = -1;
                    int64_t best_ed = -1;
                    for (int32_t q : touched) {
                        if ((dir == 0) != (q > own) || pw[q] + g.vw[v] > cap) continue;
                        if (best < 0 || conn[q] > best_ed ||
                            (conn[q] == best_ed && (pw[q] < pw[best] || (pw[q] == pw[best] && q < best)))) {
                            best = q;
                            best_ed = conn[q];
                        }
                    }
                    for (int32_t q : touched) conn[q] = 0;
                    if (best < 0) return;
                    const int64_t gain = best_ed - id;
                    if (gain > 0 || (gain == 0 && pw[best] + g.vw[v] < pw[own]))
                        mine.push_back({v, best, gain});
                });
            }
            guard.rethrow();
            props.clear();
            for (auto& m : local) props.insert(props.end(), m.begin(), m.end());
            std::sort(props.begin(), props.end(), [](const Move& a, const Move& b) {
                if (a.q != b.q) return a.q < b.q;
                if (a.gain != b.gain) return a.gain > b.gain;
                return a.v < b.v;
            });
            std::fill(win.begin(), win.end(), 0);
            std::fill(wout.begin(), wout.end(), 0);
            for (const Move& m : props) {
                const int32_t own = part[m.v], w = g.vw[m.v];
                if (pw[m.q] + win[m.q] + w > cap || pw[own] - wout[own] - w <= 0) continue;
                // a balancing move (no gain) must still go to the lighter part
                if (m.gain == 0 && pw[m.q] + win[m.q] + w >= pw[own] - wout[own]) continue;
                win[m.q] += w;
                wout[own] += w;
                part[m.v] = m.q;
                ++moves;
            }
            for (int32_t q = 0; q < nparts; ++q) pw[q] += win[q] - wout[q];
        }
        if (moves * 1000 < g.n) break;
    }
}

// Move vertices out of parts above the cap: first to adjacent parts with room
// (least cut increase), then, if still needed, to the lightest part.
// Returns true when every part is within the cap.
bool balance(const Graph& g, std::vector<int32_t>& part, int32_t nparts, int64_t cap, Rng& rng) {
    std::vector<int64_t> pw(nparts, 0), conn(nparts, 0);
    for (int32_t v = 0; v < g.n; ++v) pw[part[v]] += g.vw[v];
    auto over = [&]() {
        for (int32_t p = 0; p < nparts; ++p)
            if (pw[p] > cap) return true;
        return false;
    };
    if (!over()) return true;
    std::vector<int32_t> touched;
    std::vector<int32_t> order = random_order(g.n, rng);
    for (int round = 0; round < 8 && over(); ++round) {
        for (int32_t v : order) {
            const int32_t own = part[v];
            if (pw[own] <= cap) continue;
            const int64_t id = connectivity(g, part, v, conn, touched);
            int32_t best = -1;
            int64_t best_gain = INT64_MIN;
            for (int32_t q : touched) {
                if (pw[q] + g.vw[v] > cap) continue;
                const int64_t gain = conn[q] - id;
                if (gain > best_gain) {
                    best_gain = gain;
                    best = q;
                }
            }
            for (int32_t q : touched) conn[q] = 0;
            if (best >= 0) {
                part[v] = best;
                pw[own] -= g.vw[v];
                pw[best] += g.vw[v];
            }
        }
    }
    // last resort: lightest part anywhere (creates cut, keeps the cap)
    for (int32_t v : order) {
        const int32_t own = part[v];
        if (pw[own] <= cap) continue;
        int32_t light = 0;
        for (int32_t p = 1; p < nparts; ++p)
            if (pw[p] < pw[light]) light = p;
        if (pw[light] + g.vw[v] > cap) continue;
        part[v] = light;
        pw[own] -= g.vw[v];
        pw[light] += g.vw[v];
    }
    return !over();
}

}  // namespace

Error partition_multilevel(const Graph& g0, int32_t nparts, int64_t cap, uint64_t seed,
                           std::vector<int32_t>& part, int32_t& nparts_out) {
    Error err;
    const int32_t n = g0.n;
    part.assign(n, 0);
    nparts_out = n > 0 ? 1 : 0;
    if (n == 0) return err;
    const int64_t W = g0.total_vw();
    if ((int64_t)nparts * cap < W) {
        err.status = EHYB_EINVAL;
        err.msg = "partition cap too small for the requested number of partitions";
        return err;
    }
    if (nparts <= 1) return err;
    Rng rng(seed);
    const uint64_t key = mix64(seed ^ 0x5EEDull);
    const int32_t coarsen_to = std::max<int32_t>(2000, std::min<int64_t>(40LL * nparts, n));
    const int32_t maxvw =
        (int32_t)std::max<int64_t>(1, std::min<int64_t>(cap / 3, (int64_t)(1.5 * (double)W / coarsen_to)));

    std::vector<Graph> levels;
    std::vector<std::vector<int32_t>> cmaps;
    const Graph* cur = &g0;
    while (cur->n > coarsen_to) {
        std::vector<int32_t> cmap;
        Graph c = coarsen(*cur, maxvw, mix64(key + levels.size()), cmap);
        if ((double)c.n > 0.92 * (double)cur->n) break;
        cmaps.push_back(std::move(cmap));
        levels.push_back(std::move(c));
        cur = &levels.back();
    }
    // initial partition of the coarsest graph
    std::vector<int32_t> cpart(cur->n, 0);
    {
        std::vector<int32_t> ids(cur->n);
        std::iota(ids.begin(), ids.end(), 0);
        OmpGuard guard;
#pragma omp parallel
#pragma omp single
        guard.run([&] { recursive_bisection(*cur, ids, 0, nparts, key, cpart, guard); });
        guard.rethrow();
    }
    balance(*cur, cpart, nparts, cap, rng);
    refine_kway(*cur, cpart, nparts, cap, 10);
    // project back, refining at every level
    for (int lv = (int)levels.size() - 1; lv >= 0; --lv) {
        const Graph& fine = lv == 0 ? g0 : levels[lv - 1];
        const std::vector<int32_t>& cmap = cmaps[lv];
        std::vector<int32_t> fpart(fine.n);
#pragma omp parallel for schedule(static)
        for (int32_t v = 0; v < fine.n; ++v) fpart[v] = cpart[cmap[v]];
        cpart.swap(fpart);
        balance(fine, cpart, nparts, cap, rng);
        refine_kway(fine, cpart, nparts, cap, lv == 0 ? 6 : 8);
    }
    if (levels.empty()) {
        // the coarsest graph was the input itself: already refined above
    }
    if (!balance(g0, cpart, nparts, cap, rng)) {
        err.status = EHYB_EINVAL;
        err.msg = "partitioner could not satisfy the partition cap";
        return err;
    }
    // compact ids of non-empty parts, keeping their order
    std::vector<int32_t> remap(nparts, -1);
    std::vector<int64_t> cnt(nparts, 0);
    for (int32_t v = 0; v < n; ++v) cnt[cpart[v]]++;
    int32_t k = 0;
    for (int32_t p = 0; p < nparts; ++p)
        if (cnt[p] > 0) remap[p] = k++;
    for (int32_t v = 0; v < n; ++v) part[v] = remap[cpart[v]];
    nparts_out = k;
    return err;
}

}  // namespace ehyb
