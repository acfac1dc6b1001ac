// Host planner.  See plan.hpp for the three levels.
#include "plan.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <thread>
#include <unordered_map>

namespace svq {

static inline int popc(uint64_t v) { return __builtin_popcountll(v); }
static inline uint64_t bit(int q) { return 1ULL << q; }

// ---------------------------------------------------------------------------
// gate normalisation
// ---------------------------------------------------------------------------

static int arity(int kind) {
    switch (kind) {
    case SVQ_CNOT: case SVQ_CZ: case SVQ_CPHASE: case SVQ_GIVENS: case SVQ_SWAP: case SVQ_U2:
        return 2;
    default:
        return 1;
    }
}

std::string normalize_gates(int n, const svq_gate *gates, int m, int n_theta,
                            std::vector<GateN> &out) {
    out.clear();
    out.reserve(m);
    for (int i = 0; i < m; ++i) {
        const svq_gate &s = gates[i];
        GateN g;
        g.kind = s.kind;
        if (s.kind < SVQ_H || s.kind > SVQ_U2) return "gate " + std::to_string(i) + ": bad kind";
        g.nq = arity(s.kind);
        for (int j = 0; j < g.nq; ++j) {
            if (s.q[j] < 0 || s.q[j] >= n) return "gate " + std::to_string(i) + ": qubit out of range";
            g.q[j] = s.q[j];
        }
        if (g.nq == 2 && g.q[0] == g.q[1]) return "gate " + std::to_string(i) + ": repeated qubit";
        g.param = s.param;
        if (s.param >= n_theta || s.param < -1)
            return "gate " + std::to_string(i) + ": param index out of range";
        bool parametric = s.kind == SVQ_RX || s.kind == SVQ_RY || s.kind == SVQ_RZ ||
                          s.kind == SVQ_CPHASE || s.kind == SVQ_GIVENS;
        if (!parametric && s.param >= 0) return "gate " + std::to_string(i) + ": kind takes no parameter";
        g.offset = s.offset;
        g.scale = s.param >= 0 ? s.scale : 0.0;
        if (!std::isfinite(s.offset) || (s.param >= 0 && !std::isfinite(s.scale)))
            return "gate " + std::to_string(i) + ": non-finite angle offset or scale";
        if (s.kind == SVQ_U1 || s.kind == SVQ_U2) {
            int cnt = s.kind == SVQ_U1 ? 8 : 32;
            for (int j = 0; j < cnt; ++j) {
                if (!std::isfinite(s.mat[j])) return "gate " + std::to_string(i) + ": non-finite matrix";
                g.mat[j] = s.mat[j];
            }
        }
        g.tmask = bit(g.q[0]) | (g.nq == 2 ? bit(g.q[1]) : 0);
        switch (s.kind) {
        case SVQ_Z: case SVQ_S: case SVQ_T: case SVQ_RZ:
            g.diag_q = g.q[0];
            break;
        case SVQ_CZ: case SVQ_CPHASE:
            g.diag_q = g.q[1];
            g.ctrlmask = bit(g.q[0]);
            break;
        case SVQ_CNOT:
            g.ctrlmask = bit(g.q[0]);
            g.mixmask = bit(g.q[1]);
            break;
        case SVQ_GIVENS: case SVQ_SWAP: case SVQ_U2:
            g.mixmask = g.tmask;
            break;
        default:
            g.mixmask = bit(g.q[0]);
        }
        out.push_back(g);
    }
    return "";
}

// ---------------------------------------------------------------------------
// level 1
// ---------------------------------------------------------------------------

std::vector<int> depth_order(const std::vector<uint64_t> &targets) {
    const int m = (int)targets.size();
    std::vector<int> depth(m);
    int last[64];
    for (int q = 0; q < 64; ++q) last[q] = -1;
    for (int i = 0; i < m; ++i) {
        int d = 0;
        for (uint64_t t = targets[i]; t; t &= t - 1) {
            int q = __builtin_ctzll(t);
            d = std::max(d, last[q] + 1);
        }
        depth[i] = d;
        for (uint64_t t = targets[i]; t; t &= t - 1) last[__builtin_ctzll(t)] = d;
    }
    // Bucket by depth (the paper's O(d m) bucket sort), then within a depth
    // order by the ascending target tuple, then by index.
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    auto key_less = [&](int a, int b) {
        if (depth[a] != depth[b]) return depth[a] < depth[b];
        uint64_t ta = targets[a], tb = targets[b];
        while (ta && tb) {   // compare ascending qubit tuples lexicographically
            int qa = __builtin_ctzll(ta), qb = __builtin_ctzll(tb);
            if (qa != qb) return qa < qb;
            ta &= ta - 1;
            tb &= tb - 1;
        }
        if (ta != tb) return ta == 0;   // a shorter tuple that is a prefix sorts first
        return a < b;
    };
    std::stable_sort(order.begin(), order.end(), key_less);
    return order;
}

// Alg. 2: greedy tile under local set QL.
static std::vector<int> tile_construction(uint64_t QL, const std::vector<int> &remain,
                                          const std::vector<uint64_t> &targets) {
    uint64_t avail = QL;
    std::vector<int> tile;
    for (int i : remain) {
        uint64_t T = targets[i];
        if ((T & ~avail) == 0) tile.push_back(i);
        else avail &= ~T;
        if (!avail) break;
    }
    return tile;
}

// Alg. 3: greedy local-set choice from the shallowest remaining operators,
// then the boundary fill with the lowest free qubits of `universe`.
static uint64_t qubit_mapping(uint64_t universe, uint64_t init, const std::vector<int> &remain,
                              const std::vector<uint64_t> &targets, int budget) {
    uint64_t avail = universe;
    uint64_t QL = init;
    for (int i : remain) {
        uint64_t T = targets[i];
        if ((T & ~avail) == 0 && popc(QL | T) <= budget) QL |= T;
        else avail &= ~T;
        if (!avail) break;
    }
    for (uint64_t free = universe & ~QL; popc(QL) < budget && free; free &= free - 1)
        QL |= free & (~free + 1);
    return QL;
}

// Alg. 3 with the boundary fill taking the highest free qubits instead.
static uint64_t qubit_mapping_fill(uint64_t universe, const std::vector<int> &remain,
                                   const std::vector<uint64_t> &targets, int budget, bool highest) {
    uint64_t avail = universe;
    uint64_t QL = 0;
    for (int i : remain) {
        uint64_t T = targets[i];
        if ((T & ~avail) == 0 && popc(QL | T) <= budget) QL |= T;
        else avail &= ~T;
        if (!avail) break;
    }
    if (!QL) return 0;
    if (!highest) {
        for (uint64_t free = universe & ~QL; popc(QL) < budget && free; free &= free - 1)
            QL |= free & (~free + 1);
    } else {
        for (int q = 63; q >= 0 && popc(QL) < budget; --q)
            if (((universe >> q) & 1) && !((QL >> q) & 1)) QL |= bit(q);
    }
    return QL;
}

// Level-2 pass set (our own packing; the paper's tiling has one level).  Two
// greedy candidates: the local-set greedy of Alg. 3, and a set grown from the
// forced bits by repeatedly adding the frontier gate (every earlier gate on
// its qubits already in the pass) that needs the fewest new qubits, which
// keeps light cones compact.
static void pass_candidates(uint64_t universe, uint64_t forced, const std::vector<int> &remain,
                            const std::vector<uint64_t> &targets, int budget, uint64_t &a,
                            uint64_t &b) {
    a = qubit_mapping(universe, forced, remain, targets, budget);
    uint64_t S = forced;
    for (;;) {
        uint64_t avail = S, blocked = 0;
        int pick = -1, pick_new = 99;
        for (int i : remain) {
            const uint64_t T = targets[i];
            if ((T & ~avail) == 0) continue;   // inside the pass
            avail &= ~T;
            // blocked: qubits of every earlier gate outside the pass; a gate
            // on none of them is on the frontier and (as T is not inside
            // S & ~blocked) needs at least one new qubit
            const bool frontier = (T & blocked) == 0;
            blocked |= T;
            if (!frontier) continue;
            const int nw = popc(T & ~S);
            if (nw > 0 && popc(S) + nw <= budget && nw < pick_new) {
                pick = i;
                pick_new = nw;
            }
        }
        if (pick < 0) break;
        S |= targets[pick];
    }
    for (uint64_t free = universe & ~S; popc(S) < budget && free; free &= free - 1)
        S |= free & (~free + 1);
    b = S;
}

static std::vector<int> without(const std::vector<int> &remain, const std::vector<int> &G, int m) {
    std::vector<char> tk(m, 0);
    for (int i : G) tk[i] = 1;
    std::vector<int> rest;
    rest.reserve(remain.size());
    for (int i : remain)
        if (!tk[i]) rest.push_back(i);
    return rest;
}

// The candidate whose pass holds more gates (ties: the Alg. 3 one).
static uint64_t fuller_pass(uint64_t universe, uint64_t forced, const std::vector<int> &remain,
                            const std::vector<uint64_t> &targets, int budget) {
    uint64_t a, b;
    pass_candidates(universe, forced, remain, targets, budget, a, b);
    return tile_construction(b, remain, targets).size() > tile_construction(a, remain, targets).size()
               ? b : a;
}

// Pick between the two candidates by completing each with fuller_pass and
// counting the passes; fewer passes win, then more gates in this pass.
static uint64_t choose_pass_set(uint64_t universe, uint64_t forced, const std::vector<int> &remain,
                                const std::vector<uint64_t> &targets, int budget) {
    uint64_t a, b;
    pass_candidates(universe, forced, remain, targets, budget, a, b);
    const std::vector<int> Ga = tile_construction(a, remain, targets);
    const std::vector<int> Gb = tile_construction(b, remain, targets);
    if (a == b || Gb.empty()) return a;
    if (Ga.empty()) return b;
    const int m = (int)targets.size();
    auto rollout = [&](std::vector<int> rest) {
        int passes = 0;
        while (!rest.empty()) {
            const uint64_t S = fuller_pass(universe, forced, rest, targets, budget);
            const std::vector<int> G = tile_construction(S, rest, targets);
            if (G.empty()) return 1 << 20;
            rest = without(rest, G, m);
            ++passes;
        }
        return passes;
    };
    const int pa = rollout(without(remain, Ga, m)), pb = rollout(without(remain, Gb, m));
    if (pa != pb) return pa < pb ? a : b;
    return Gb.size() > Ga.size() ? b : a;
}

// ---- level 2 with a relabelling store ---------------------------------------
// A pass may store its tile with the tile's bit positions permuted (in place:
// the tile occupies the same addresses).  The previous pass's store therefore
// moves c qubits that the next pass acts on into the c lowest physical
// positions, which every tile must contain for coalescing; the next pass's
// qubit set S (k qubits) then needs at most k - c qubits outside the previous
// pass's set kprev.

static bool rl_fits(uint64_t S, uint64_t kprev, int k, int c) {
    return popc(S) <= k && popc(S & ~kprev) <= k - c;
}

// Complete S to k qubits: first from kprev (free under the k - c budget),
// then from the other local qubits, each in ascending physical position.
static uint64_t rl_fill(uint64_t S, uint64_t universe, uint64_t kprev, int k, int c,
                        const std::vector<int> &lay) {
    std::vector<int> qs;
    for (uint64_t u = universe & ~S; u; u &= u - 1) qs.push_back(__builtin_ctzll(u));
    std::sort(qs.begin(), qs.end(), [&](int a, int b) { return lay[a] < lay[b]; });
    for (int pass = 0; pass < 2; ++pass)
        for (int q : qs) {
            if (popc(S) >= k) return S;
            const bool inprev = (kprev >> q) & 1;
            if ((pass == 0) != inprev || ((S >> q) & 1)) continue;
            if (rl_fits(S | bit(q), kprev, k, c)) S |= bit(q);
        }
    return S;
}

// The two greedy candidates of pass_candidates under the relabelling
// constraint (logical qubit sets).
static void rl_candidates(uint64_t universe, uint64_t kprev, const std::vector<int> &remain,
                          const std::vector<uint64_t> &targets, int k, int c,
                          const std::vector<int> &lay, uint64_t &a, uint64_t &b) {
    uint64_t avail = universe, S = 0;
    for (int i : remain) {
        const uint64_t T = targets[i];
        if ((T & ~avail) == 0 && rl_fits(S | T, kprev, k, c)) S |= T;
        else avail &= ~T;
        if (!avail) break;
    }
    a = rl_fill(S, universe, kprev, k, c, lay);
    S = 0;
    for (;;) {
        uint64_t av = S, blocked = 0;
        int pick = -1, pick_new = 99;
        for (int i : remain) {
            const uint64_t T = targets[i];
            if ((T & ~av) == 0) continue;
            av &= ~T;
            const bool frontier = (T & blocked) == 0;
            blocked |= T;
            if (!frontier) continue;
            const int nw = popc(T & ~S);
            if (nw > 0 && rl_fits(S | T, kprev, k, c) && nw < pick_new) {
                pick = i;
                pick_new = nw;
            }
        }
        if (pick < 0) break;
        S |= targets[pick];
    }
    b = rl_fill(S, universe, kprev, k, c, lay);
}

static uint64_t rl_fuller(uint64_t universe, uint64_t kprev, const std::vector<int> &remain,
                          const std::vector<uint64_t> &targets, int k, int c,
                          const std::vector<int> &lay) {
    uint64_t a, b;
    rl_candidates(universe, kprev, remain, targets, k, c, lay, a, b);
    return tile_construction(b, remain, targets).size() > tile_construction(a, remain, targets).size()
               ? b : a;
}

// Choose between the candidates by completing each greedily (the pass after
// a pass with qubit set S has kprev = S) and counting passes.
static uint64_t rl_choose(uint64_t universe, uint64_t kprev, const std::vector<int> &remain,
                          const std::vector<uint64_t> &targets, int k, int c,
                          const std::vector<int> &lay) {
    uint64_t a, b;
    rl_candidates(universe, kprev, remain, targets, k, c, lay, a, b);
    const std::vector<int> Ga = tile_construction(a, remain, targets);
    const std::vector<int> Gb = tile_construction(b, remain, targets);
    if (a == b || Gb.empty()) return a;
    if (Ga.empty()) return b;
    const int m = (int)targets.size();
    auto rollout = [&](std::vector<int> rest, uint64_t kp) {
        int passes = 0;
        while (!rest.empty()) {
            const uint64_t S = rl_fuller(universe, kp, rest, targets, k, c, lay);
            const std::vector<int> G = tile_construction(S, rest, targets);
            if (G.empty()) return 1 << 20;
            rest = without(rest, G, m);
            kp = S;
            ++passes;
        }
        return passes;
    };
    const int pa = rollout(without(remain, Ga, m), a), pb = rollout(without(remain, Gb, m), b);
    if (pa != pb) return pa < pb ? a : b;
    return Gb.size() > Ga.size() ? b : a;
}

static uint64_t local_set(const std::vector<int> &pos, int nL) {
    uint64_t s = 0;
    for (size_t q = 0; q < pos.size(); ++q)
        if (pos[q] < nL) s |= bit((int)q);
    return s;
}

// Exchange outgoing local qubits with incoming global ones, pairing both in
// ascending physical position; updates pos.
static std::vector<Transposition> remap(std::vector<int> &pos, int nL, uint64_t newQL) {
    const int n = (int)pos.size();
    std::vector<int> out, in;
    for (int q = 0; q < n; ++q) {
        bool loc = pos[q] < nL, want = (newQL >> q) & 1;
        if (loc && !want) out.push_back(q);
        if (!loc && want) in.push_back(q);
    }
    auto by_pos = [&](int a, int b) { return pos[a] < pos[b]; };
    std::sort(out.begin(), out.end(), by_pos);
    std::sort(in.begin(), in.end(), by_pos);
    std::vector<Transposition> tr;
    for (size_t i = 0; i < out.size() && i < in.size(); ++i) {
        tr.push_back({pos[out[i]], pos[in[i]]});
        std::swap(pos[out[i]], pos[in[i]]);
    }
    return tr;
}

std::vector<L1Tile> flat_tiling(int n, int nL, const std::vector<uint64_t> &targets,
                                std::vector<int> &pos) {
    const uint64_t Q = n >= 64 ? ~0ULL : (bit(n) - 1);
    std::vector<int> remain = depth_order(targets);
    uint64_t QL = local_set(pos, nL);
    std::vector<L1Tile> tiles;
    bool first = true;
    while (!remain.empty()) {
        std::vector<Transposition> tr;
        if (!first) {
            QL = qubit_mapping(Q, 0, remain, targets, nL);
            tr = remap(pos, nL, QL);
        }
        first = false;
        std::vector<int> G = tile_construction(QL, remain, targets);
        if (G.empty()) continue;   // (only possible on the first round)
        std::vector<char> taken(targets.size(), 0);
        for (int i : G) taken[i] = 1;
        std::vector<int> rest;
        for (int i : remain)
            if (!taken[i]) rest.push_back(i);
        remain.swap(rest);
        if (!tiles.empty() && tiles.back().local == QL && tr.empty()) {
            tiles.back().ops.insert(tiles.back().ops.end(), G.begin(), G.end());
        } else {
            L1Tile t;
            t.local = QL;
            t.ops = G;
            t.qr = tr;
            tiles.push_back(std::move(t));
        }
    }
    return tiles;
}

std::vector<L1Tile> hierarchical_tiling(int n, int nL, int n_intra,
                                        const std::vector<uint64_t> &targets, bool fill_highest,
                                        std::vector<int> &kinds, std::vector<uint64_t> &intra) {
    const uint64_t Q = n >= 64 ? ~0ULL : (bit(n) - 1);
    std::vector<int> remain = depth_order(targets);
    uint64_t QL = bit(nL) - 1;
    uint64_t QI = (bit(nL + n_intra) - 1) & ~QL;
    std::vector<L1Tile> tiles;
    kinds.clear();
    intra.clear();
    int pending_kind = 0;
    bool first = true;
    while (!remain.empty()) {
        if (!first) {
            // Alg. 5: intra-only pool first; valid only if it admits an operator
            const uint64_t pool = QL | QI;
            uint64_t nl = qubit_mapping_fill(pool, remain, targets, nL, fill_highest);
            if (nl && !tile_construction(nl, remain, targets).empty()) {
                QI = pool & ~nl;
                QL = nl;
                pending_kind = 0;
            } else {
                const uint64_t old_inter = Q & ~QL & ~QI;
                nl = qubit_mapping_fill(Q, remain, targets, nL, fill_highest);
                uint64_t qp = qubit_mapping_fill(Q, remain, targets, nL + n_intra, fill_highest);
                uint64_t qi = qp & ~nl;
                // keep |Q_intra| fixed when the two greedy picks diverge
                if (!fill_highest) {
                    for (int q = 0; q < n && popc(qi) < n_intra; ++q)
                        if (!((nl >> q) & 1) && !((qi >> q) & 1)) qi |= bit(q);
                    while (popc(qi) > n_intra) qi &= ~bit(63 - __builtin_clzll(qi));
                } else {
                    for (int q = n - 1; q >= 0 && popc(qi) < n_intra; --q)
                        if (!((nl >> q) & 1) && !((qi >> q) & 1)) qi |= bit(q);
                    while (popc(qi) > n_intra) qi &= qi - 1;
                }
                QL = nl;
                QI = qi;
                pending_kind = ((Q & ~QL & ~QI) == old_inter) ? 0 : 1;
            }
        }
        first = false;
        std::vector<int> G = tile_construction(QL, remain, targets);
        if (G.empty()) continue;
        std::vector<char> taken(targets.size(), 0);
        for (int i : G) taken[i] = 1;
        std::vector<int> rest;
        for (int i : remain)
            if (!taken[i]) rest.push_back(i);
        remain.swap(rest);
        L1Tile t;
        t.local = QL;
        t.ops = G;
        tiles.push_back(std::move(t));
        kinds.push_back(pending_kind);
        intra.push_back(QI);
    }
    return tiles;
}

std::vector<L1Tile> ad_hoc(int n, int nL, const std::vector<uint64_t> &targets,
                           const std::vector<int> &order, std::vector<int> &pos) {
    std::vector<L1Tile> tiles;
    for (int i : order) {
        uint64_t T = targets[i];
        uint64_t local = local_set(pos, nL);
        std::vector<Transposition> tr;
        if (T & ~local) {
            std::vector<int> in, cand;
            for (int q = 0; q < n; ++q) {
                if (((T >> q) & 1) && !((local >> q) & 1)) in.push_back(q);
                if (((local >> q) & 1) && !((T >> q) & 1)) cand.push_back(q);
            }
            std::sort(in.begin(), in.end(), [&](int a, int b) { return pos[a] < pos[b]; });
            std::sort(cand.begin(), cand.end(), [&](int a, int b) { return pos[a] > pos[b]; });
            cand.resize(in.size());
            std::sort(cand.begin(), cand.end(), [&](int a, int b) { return pos[a] < pos[b]; });
            for (size_t j = 0; j < in.size(); ++j) {
                tr.push_back({pos[cand[j]], pos[in[j]]});
                std::swap(pos[cand[j]], pos[in[j]]);
            }
            local = local_set(pos, nL);
        }
        if (tiles.empty() || !tr.empty() || tiles.back().local != local) {
            L1Tile t;
            t.local = local;
            t.qr = tr;
            tiles.push_back(std::move(t));
        }
        tiles.back().ops.push_back(i);
    }
    return tiles;
}

std::vector<L1Tile> tiling_pauli(int n, int nL, const std::vector<uint64_t> &supports,
                                 const std::vector<int> &weights, std::vector<int> &pos) {
    // All n_L-subsets of {0..n-1} in lexicographic order of sorted tuples.
    std::vector<uint64_t> sets;
    {
        std::vector<int> c(nL);
        for (int i = 0; i < nL; ++i) c[i] = i;
        while (true) {
            uint64_t mk = 0;
            for (int v : c) mk |= bit(v);
            sets.push_back(mk);
            int i = nL - 1;
            while (i >= 0 && c[i] == n - nL + i) --i;
            if (i < 0) break;
            ++c[i];
            for (int j = i + 1; j < nL; ++j) c[j] = c[j - 1] + 1;
        }
    }
    std::vector<int> remain(supports.size());
    for (size_t i = 0; i < supports.size(); ++i) remain[i] = (int)i;
    std::vector<L1Tile> tiles;
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    uint64_t cur = local_set(pos, nL);
    while (!remain.empty()) {
        std::vector<uint64_t> rs(remain.size());
        std::vector<int> rw(remain.size());
        for (size_t i = 0; i < remain.size(); ++i) {
            rs[i] = supports[remain[i]];
            rw[i] = weights[remain[i]];
        }
        auto count = [&](uint64_t mk) {
            long long c = 0;
            for (size_t i = 0; i < rs.size(); ++i)
                if ((rs[i] & ~mk) == 0) c += rw[i];
            return c;
        };
        // Per-thread best over a contiguous slice, strict '<' keeps the first.
        std::vector<long long> bestc(nth, 0);
        std::vector<long long> besti(nth, -1);
        std::vector<std::thread> th;
        const size_t ns = sets.size();
        for (unsigned t = 0; t < nth; ++t) {
            th.emplace_back([&, t]() {
                size_t lo = ns * t / nth, hi = ns * (t + 1) / nth;
                long long bc = 0, bi = -1;
                for (size_t s = lo; s < hi; ++s) {
                    long long c = count(sets[s]);
                    if (bc < c) { bc = c; bi = (long long)s; }
                }
                bestc[t] = bc;
                besti[t] = bi;
            });
        }
        for (auto &x : th) x.join();
        long long bc = count(cur);
        uint64_t best = cur;
        if (bc == 0) best = 0;
        for (unsigned t = 0; t < nth; ++t)
            if (bc < bestc[t]) { bc = bestc[t]; best = sets[besti[t]]; }
        if (bc == 0) break;   // nothing placeable (callers exclude wide supports)
        L1Tile tile;
        tile.local = best;
        tile.qr = remap(pos, nL, best);
        std::vector<int> rest;
        for (int i : remain) {
            if ((supports[i] & ~best) == 0) tile.ops.push_back(i);
            else rest.push_back(i);
        }
        remain.swap(rest);
        cur = best;
        tiles.push_back(std::move(tile));
    }
    return tiles;
}

// ---------------------------------------------------------------------------
// circuit plan: levels 2 and 3
// ---------------------------------------------------------------------------

static uint64_t phys_mask(uint64_t logical, const std::vector<int> &pos) {
    uint64_t m = 0;
    for (uint64_t t = logical; t; t &= t - 1) m |= bit(pos[__builtin_ctzll(t)]);
    return m;
}

// Tile-local index of physical bits in S (sorted ascending).
static uint32_t to_tile(uint64_t phys, uint64_t S) {
    uint32_t out = 0;
    int j = 0;
    for (uint64_t s = S; s; s &= s - 1, ++j)
        if (phys & (s & (~s + 1))) out |= 1u << j;
    return out;
}

static int first_bit(uint64_t v) { return v ? __builtin_ctzll(v) : -1; }

// Choose lane bits for a phase: six non-register tile bits, lowest first,
// with pairwise distinct residues mod 6 where possible (so that the folded
// LDS swizzle keeps the 64 lanes on distinct banks); lane b gets residue b
// when all six residues are present.
static void assign_lanes(int k, uint32_t regs, PhaseDesc &P) {
    int lanes[6];
    int nl = 0;
    bool used_res[6] = {false, false, false, false, false, false};
    uint32_t taken = regs;
    for (int b = 0; b < k && nl < 6; ++b) {
        if ((taken >> b) & 1) continue;
        if (used_res[b % 6]) continue;
        used_res[b % 6] = true;
        lanes[nl++] = b;
        taken |= 1u << b;
    }
    for (int b = 0; b < k && nl < 6; ++b) {   // fall back: any free bit
        if ((taken >> b) & 1) continue;
        lanes[nl++] = b;
        taken |= 1u << b;
    }
    // order by residue so lane bit b has residue b where possible
    std::stable_sort(lanes, lanes + nl, [](int a, int b) { return a % 6 < b % 6; });
    for (int i = 0; i < 8; ++i) P.lane[i] = 0;
    for (int i = 0; i < nl; ++i) P.lane[i] = lanes[i];
    int nw = 0;
    for (int i = 0; i < 8; ++i) P.wave[i] = 0;
    for (int b = 0; b < k; ++b)
        if (!((taken >> b) & 1)) P.wave[nw++] = b;
}

static void set_regs(uint32_t regs, int rb, PhaseDesc &P) {
    int j = 0;
    for (int i = 0; i < 8; ++i) P.reg[i] = 0;
    for (uint32_t r = regs; r && j < rb; r &= r - 1) P.reg[j++] = __builtin_ctz(r);
}

struct L3Gate {
    int gate;
    int kind;
    uint32_t t, mix, ctrl;
    int diag;       // tile-local bit of the diagonal, -1
    int tq0, tq1;   // tile-local bits of the gate's q[0], q[1] (-1 if absent)
};

static int op_type_of(int kind) {
    switch (kind) {
    case SVQ_Z: case SVQ_S: case SVQ_T: case SVQ_RZ:
        return OP_DIAG1;
    case SVQ_CZ: case SVQ_CPHASE:
        return OP_CPHASE;
    case SVQ_X:
        return OP_XSWAP;
    case SVQ_CNOT:
        return OP_CNOT;
    case SVQ_RY:
        return OP_ROTY;
    case SVQ_GIVENS:
        return OP_GIVENS;
    case SVQ_SWAP: case SVQ_U2:
        return OP_MIX2;
    default:
        return OP_MIX1;
    }
}

int op_type_for_kind(int kind) { return op_type_of(kind); }

// Lanes of a load or store phase: the required tile bits (those on the
// lowest physical positions, in position order, so that consecutive lanes
// address consecutive amplitudes), then free bits preferring residue i mod 6
// for lane i (distinct LDS banks under the swizzle).
static void io_lanes(int k, uint32_t regs, const int *req, int nreq, PhaseDesc &D) {
    int lanes[6] = {-1, -1, -1, -1, -1, -1};
    uint32_t taken = regs;
    for (int i = 0; i < nreq && i < 6; ++i) {
        lanes[i] = req[i];
        taken |= 1u << req[i];
    }
    for (int i = std::min(nreq, 6); i < 6; ++i)
        for (int b = 0; b < k; ++b)
            if (!((taken >> b) & 1) && b % 6 == i) {
                lanes[i] = b;
                taken |= 1u << b;
                break;
            }
    for (int i = 0; i < 6; ++i)
        if (lanes[i] < 0)
            for (int b = 0; b < k; ++b)
                if (!((taken >> b) & 1)) {
                    lanes[i] = b;
                    taken |= 1u << b;
                    break;
                }
    for (int i = 0; i < 8; ++i) D.lane[i] = 0;
    for (int i = 0; i < 6; ++i) D.lane[i] = lanes[i];
    int nw = 0;
    for (int i = 0; i < 8; ++i) D.wave[i] = 0;
    for (int b = 0; b < k; ++b)
        if (!((taken >> b) & 1)) D.wave[nw++] = b;
}

// Level 3.  ld/st: the tile bits the load and store phases must have as
// lanes 0.. (in order).  They differ when the pass's store relabels positions.
static void plan_phases(int k, int rb, const std::vector<L3Gate> &gs, CircuitPlan &P,
                        const int *ld, int nld, const int *st, int nst) {
    const uint32_t all = (k >= 32) ? ~0u : ((1u << k) - 1);
    const uint32_t low6 = 63u;
    (void)low6;
    std::vector<int> remain(gs.size());
    for (size_t i = 0; i < gs.size(); ++i) remain[i] = (int)i;
    struct Ph { uint32_t regs; std::vector<int> ops; };
    std::vector<Ph> phs;
    while (!remain.empty()) {
        // mapping: registers from the mixing qubits of the shallowest gates
        uint64_t avail = all, regs = 0;
        for (int i : remain) {
            uint32_t M = gs[i].mix;
            if ((M & ~avail) == 0 && popc(regs | M) <= rb) regs |= M;
            else avail &= ~(uint64_t)gs[i].t;
            if (!avail) break;
        }
        auto fill = [&](uint64_t r) {
            // fill with the highest tile bits outside the coalescing lanes first
            for (int b = k - 1; b >= 6 && popc(r) < rb; --b) r |= 1u << b;
            for (int b = k - 1; b >= 0 && popc(r) < rb; --b) r |= 1u << b;
            return r;
        };
        // tile construction with dependency blocking on all targets
        auto phase_gates = [&](uint64_t r) {
            uint64_t av = all;
            std::vector<int> out;
            for (int i : remain) {
                const L3Gate &g = gs[i];
                if ((g.t & ~av) == 0 && (g.mix & ~r) == 0) out.push_back(i);
                else av &= ~(uint64_t)g.t;
                if (!av) break;
            }
            return out;
        };
        regs = fill(regs);
        std::vector<int> G = phase_gates(regs);
        {
            // second candidate: grow the register set by the frontier gate
            // that needs the fewest new register bits
            uint64_t r2 = 0;
            for (;;) {
                uint64_t av = all, blocked = 0;
                int pick = -1, pick_new = 99;
                for (int i : remain) {
                    const L3Gate &g = gs[i];
                    if ((g.t & ~av) == 0 && (g.mix & ~r2) == 0) continue;   // runs now
                    av &= ~(uint64_t)g.t;
                    const bool frontier = (g.t & blocked) == 0;
                    blocked |= g.t;
                    if (!frontier) continue;
                    const int nw = popc(g.mix & ~r2);
                    if (nw > 0 && popc(r2 | g.mix) <= rb && nw < pick_new) {
                        pick = i;
                        pick_new = nw;
                    }
                }
                if (pick < 0) break;
                r2 |= gs[pick].mix;
            }
            r2 = fill(r2);
            std::vector<int> G2 = phase_gates(r2);
            if (G2.size() > G.size()) {
                regs = r2;
                G.swap(G2);
            }
        }
        std::vector<char> tk(gs.size(), 0);
        for (int i : G) tk[i] = 1;
        std::vector<int> rest;
        for (int i : remain)
            if (!tk[i]) rest.push_back(i);
        remain.swap(rest);
        if (!phs.empty() && phs.back().regs == (uint32_t)regs) {
            phs.back().ops.insert(phs.back().ops.end(), G.begin(), G.end());
        } else {
            phs.push_back({(uint32_t)regs, G});
        }
    }
    // The load phase needs lanes on the tile bits that sit on the lowest
    // physical positions before the pass, the store phase on those that sit
    // there after it; their registers may use any other bits.  A pure
    // transpose phase is added where the first or last gate phase does not
    // allow it (and whenever the two lane sets differ but one phase would do
    // both).
    uint32_t ldm = 0, stm = 0;
    for (int i = 0; i < nld; ++i) ldm |= 1u << ld[i];
    for (int i = 0; i < nst; ++i) stm |= 1u << st[i];
    bool same_io = nld == nst;
    for (int i = 0; same_io && i < nld; ++i) same_io = ld[i] == st[i];
    auto io_regs = [&](uint32_t avoid) {
        uint32_t r = 0;
        for (int b = k - 1; b >= 0 && popc(r) < rb; --b)
            if (!((avoid >> b) & 1)) r |= 1u << b;
        return r;
    };
    if (phs.empty() || (phs.front().regs & ldm)) phs.insert(phs.begin(), Ph{io_regs(ldm), {}});
    if ((phs.back().regs & stm) || (phs.size() == 1 && !same_io)) phs.push_back(Ph{io_regs(stm), {}});
    for (size_t pi = 0; pi < phs.size(); ++pi) {
        auto &ph = phs[pi];
        PhaseDesc D;
        std::memset(&D, 0, sizeof(D));
        set_regs(ph.regs, rb, D);
        if (pi == 0) {
            io_lanes(k, ph.regs, ld, nld, D);
        } else if (pi + 1 == phs.size()) {
            io_lanes(k, ph.regs, st, nst, D);
        } else if ((ph.regs & low6) == 0) {
            // keep lanes on bits 0..5
            for (int i = 0; i < 6; ++i) D.lane[i] = i;
            int nw = 0;
            for (int b = 6; b < k; ++b)
                if (!((ph.regs >> b) & 1)) D.wave[nw++] = b;
        } else {
            assign_lanes(k, ph.regs, D);
        }
        D.op0 = (int)P.ops.size();
        D.nop = (int)ph.ops.size();
        int regpos[32];
        for (int i = 0; i < 32; ++i) regpos[i] = -1;
        for (int j = 0; j < rb; ++j) regpos[(int)D.reg[j]] = j;
        for (int i : ph.ops) {
            const L3Gate &g = gs[i];
            OpDesc o;
            std::memset(&o, 0, sizeof(o));
            o.gslot = -1;
            o.type = op_type_of(g.kind);
            o.spare = 0;
            o.flip = 0;
            o.b0 = regpos[g.tq0];
            o.b1 = g.tq1 >= 0 ? regpos[g.tq1] : 0;
            P.ops.push_back(o);
            P.op_gate.push_back(g.gate);
        }
        P.phases.push_back(D);
    }
    P.n_phases_total += (int)phs.size();
}

// ---- LDS slot map of a gate pass ------------------------------------------
// A transpose between two phases writes the tile to LDS with one phase's
// (lane, wave, register) mapping and reads it back with the next phase's.
// Tile index t lives in slot f(t) = XOR of swz[j] over the set bits j of t;
// f is a bijection of the tile when swz[0..5] are linearly independent six-bit
// values and swz[j] = 2^j ^ (a six-bit value) for j >= 6.
//
// gfx950's LDS serves the 8-byte accesses of a wave in groups of 16 and of 32
// lanes and its 16-byte accesses in groups of 8 lanes; a group runs without
// bank conflicts when its slots are distinct modulo 16, 32 and 8 respectively
// (measured with SQ_LDS_BANK_CONFLICT on single-pattern kernels).  Lane bit b
// adds swz[lane[b]] to the slot, so a phase is conflict-free when the swz
// values of its first three, four and five lanes are linearly independent
// modulo 8, 16 and 32.  The lanes of a phase may be listed in any order, but
// the load and store phases keep the tile bits on the lowest physical
// positions as their first lanes (coalescing).  The planner searches swz
// values, and a lane order per phase, under which every phase of the pass
// meets the condition.

static int gf2_rank(const uint32_t *v, int n, uint32_t mask) {
    uint32_t piv[32] = {0};
    int r = 0;
    for (int i = 0; i < n; ++i) {
        uint32_t x = v[i] & mask;
        while (x) {
            const int hb = 31 - __builtin_clz(x);
            if (!piv[hb]) {
                piv[hb] = x;
                ++r;
                break;
            }
            x ^= piv[hb];
        }
    }
    return r;
}

// An order of the six lane bits L (tile-local) whose first 3/4/5 entries meet
// the bank condition under sv, with the nr required bits req first; false if
// there is none.
static bool lane_chain(const int32_t *L, const int *req, int nr, const uint32_t *sv, int32_t *order) {
    uint32_t rmask = 0;
    for (int i = 0; i < nr; ++i) rmask |= 1u << req[i];
    auto fits = [&](uint32_t S, int p) {
        // the first p lanes are S: S inside the required set while it lasts,
        // and holding all of it after that
        return nr >= p ? (S & ~rmask) == 0 : (rmask & ~S) == 0;
    };
    auto vals = [&](uint32_t S, uint32_t *v) {
        int c = 0;
        for (int i = 0; i < 6; ++i)
            if ((S >> L[i]) & 1) v[c++] = sv[L[i]];
        return c;
    };
    uint32_t all = 0;
    for (int i = 0; i < 6; ++i) all |= 1u << L[i];
    uint32_t v[6];
    for (int ix = 0; ix < 6; ++ix) {
        const uint32_t S5 = all & ~(1u << L[ix]);
        if (!fits(S5, 5) || gf2_rank(v, vals(S5, v), 31u) < 5) continue;
        for (int iy = 0; iy < 6; ++iy) {
            if (!((S5 >> L[iy]) & 1)) continue;
            const uint32_t S4 = S5 & ~(1u << L[iy]);
            if (!fits(S4, 4) || gf2_rank(v, vals(S4, v), 15u) < 4) continue;
            for (int iz = 0; iz < 6; ++iz) {
                if (!((S4 >> L[iz]) & 1)) continue;
                const uint32_t S3 = S4 & ~(1u << L[iz]);
                if (!fits(S3, 3) || gf2_rank(v, vals(S3, v), 7u) < 3) continue;
                int o = 0;
                for (int i = 0; i < nr; ++i)
                    if ((S3 >> req[i]) & 1) order[o++] = req[i];
                for (int i = 0; i < 6; ++i)
                    if (((S3 & ~rmask) >> L[i]) & 1) order[o++] = L[i];
                order[o++] = L[iz];
                order[o++] = L[iy];
                order[o++] = L[ix];
                return true;
            }
        }
    }
    return false;
}

static void choose_swizzle(int k, CircuitPlan &P, PassArgs &pa, const int *ld, int nld, const int *st,
                           int nst) {
    uint32_t sv[16];
    for (int j = 0; j < 16; ++j) sv[j] = j < k ? 1u << (j % 6) : 0u;
    const int np = pa.nphase;
    std::vector<int32_t> order(6 * std::max(np, 1));
    std::vector<char> ok(std::max(np, 1), 0);
    auto req_of = [&](int i, const int *&req) {
        if (i == 0) {
            req = ld;
            return std::min(nld, 6);
        }
        if (i == np - 1) {
            req = st;
            return std::min(nst, 6);
        }
        req = nullptr;
        return 0;
    };
    auto check = [&](int i) {
        const int *req;
        const int nr = req_of(i, req);
        return lane_chain(P.phases[pa.phase0 + i].lane, req, nr, sv, &order[6 * i]);
    };
    if (np >= 2) {
        int score = 0;
        for (int i = 0; i < np; ++i) score += ok[i] = check(i);
        // local search: change one tile bit's value, keep it unless fewer
        // phases meet the condition (deterministic generator)
        uint64_t rs = 0x9E3779B97F4A7C15ull ^ ((uint64_t)pa.phase0 << 17) ^ (uint64_t)k;
        auto rnd = [&]() {
            rs ^= rs << 13;
            rs ^= rs >> 7;
            rs ^= rs << 17;
            return rs;
        };
        for (int it = 0; it < 4000 && score < np; ++it) {
            int bad = (int)(rnd() % (uint64_t)(np - score));
            int fi = 0;
            for (; fi < np; ++fi)
                if (!ok[fi] && bad-- == 0) break;
            const int t = P.phases[pa.phase0 + fi].lane[rnd() % 6];
            const uint32_t old = sv[t];
            sv[t] = t < 6 ? 1u + (uint32_t)(rnd() % 63) : (uint32_t)(rnd() % 64);
            if (t < 6 && gf2_rank(sv, 6, 63u) < 6) {
                sv[t] = old;
                continue;
            }
            std::vector<char> nok(ok);
            int ns = score;
            std::vector<int32_t> keep(order);
            for (int i = 0; i < np; ++i) {
                const int32_t *L = P.phases[pa.phase0 + i].lane;
                bool has = false;
                for (int b = 0; b < 6; ++b) has |= L[b] == t;
                if (!has) continue;
                ns -= nok[i];
                ns += nok[i] = check(i);
            }
            if (ns >= score) {
                score = ns;
                ok.swap(nok);
            } else {
                sv[t] = old;
                order.swap(keep);
            }
        }
        for (int i = 0; i < np; ++i)
            if (ok[i])
                for (int b = 0; b < 6; ++b) P.phases[pa.phase0 + i].lane[b] = order[6 * i + b];
    }
    for (int j = 0; j < 16; ++j) pa.swz[j] = j >= k ? 0 : (int32_t)(j < 6 ? sv[j] : (1u << j) ^ sv[j]);
    for (int i = 0; i < np; ++i) {
        PhaseDesc &D = P.phases[pa.phase0 + i];
        for (int b = 0; b < 8; ++b) {
            D.rsl[b] = pa.swz[D.reg[b] & 15];
            D.lsl[b] = b < 6 ? pa.swz[D.lane[b] & 15] : 0;
            D.wsl[b] = pa.swz[D.wave[b] & 15];
        }
    }
}

std::string plan_empty_pass(int n, int k, int rb, const int *tile_bits, int nphase, CircuitPlan &out) {
    if (k < rb + 6 || k > 16 || k > n || nphase < 1 || nphase > 64) return "bad pass shape";
    for (int j = 0; j < k; ++j)
        if (tile_bits[j] < 0 || tile_bits[j] >= n || (j && tile_bits[j] <= tile_bits[j - 1]))
            return "tile bits must be ascending positions below n";
    out = CircuitPlan();
    out.n = n;
    out.g = 0;
    out.k = k;
    out.rb = rb;
    PassArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    for (int j = 0; j < k; ++j) pa.tphys[j] = pa.tphys_out[j] = tile_bits[j];
    pa.nblocks = 1 << (n - k);
    pa.phase0 = 0;
    pa.nphase = nphase;
    int lows[6];
    for (int i = 0; i < 6; ++i) lows[i] = i;
    const uint32_t top = ((1u << rb) - 1u) << (k - rb);
    const uint32_t mid = ((1u << rb) - 1u) << 6;
    for (int ph = 0; ph < nphase; ++ph) {
        PhaseDesc D;
        std::memset(&D, 0, sizeof(D));
        const uint32_t regs = (ph & 1) ? mid : top;
        set_regs(regs, rb, D);
        if (ph == 0 || ph == nphase - 1) io_lanes(k, regs, lows, std::min(k - rb, 6), D);
        else assign_lanes(k, regs, D);
        D.op0 = 0;
        D.nop = 0;
        out.phases.push_back(D);
    }
    out.n_phases_total = nphase;
    choose_swizzle(k, out, pa, lows, 6, lows, 6);
    out.passes.push_back(pa);
    Step s;
    s.type = 1;
    s.idx = 0;
    out.steps.push_back(s);
    return "";
}

std::string plan_circuit(int n, int g, const std::vector<GateN> &gates, svq_sched sched, int k,
                         int rb, int c, const std::vector<int> &pos0, CircuitPlan &out,
                         bool relayout) {
    out = CircuitPlan();
    out.n = n;
    out.g = g;
    const int nL = n - g;
    const int keff = std::min(k, nL);
    const int ceff = std::min(c, keff);
    out.k = keff;
    out.rb = rb;
    out.c = ceff;
    const int m = (int)gates.size();
    std::vector<uint64_t> targets(m);
    for (int i = 0; i < m; ++i) {
        targets[i] = gates[i].tmask;
        if (popc(targets[i]) > nL) return "gate wider than the local qubit count";
    }
    std::vector<int> pos = pos0;
    out.pos_before = pos;
    std::vector<L1Tile> tiles = (sched == SVQ_LAZY)
                                    ? flat_tiling(n, nL, targets, pos)
                                    : ad_hoc(n, nL, targets, depth_order(targets), pos);
    (void)pos;
    // Replay the layout tile by tile for levels 2/3.  The exchanged qubits of
    // each QR come from level 1; their physical pairing (ascending positions)
    // is taken on the replayed layout, since level 2 may relabel positions
    // inside tiles.
    std::vector<int> lay = pos0;
    const uint64_t localpos = bit(nL) - 1;
    const uint64_t forced = bit(ceff) - 1;
    const int cl = std::min(ceff, 6);   // lowest positions the lanes cover
    int qrtile = 0;
    auto add_positions = [&](const std::vector<int> &G, const L1Tile &T) {
        for (int i : G) {
            out.order.push_back(i);
            out.pos_qrtile.push_back(qrtile);
            out.pos_pass.push_back((int)out.passes.size());
            out.pos_local.push_back(T.local);
        }
    };
    // level 3 of one pass; qin[j] is the logical qubit on tile bit j
    auto level3 = [&](PassArgs &pa, const std::vector<int> &G, const std::vector<int> &qin) {
        std::vector<int> tl(n, -1);
        for (int j = 0; j < keff; ++j) tl[qin[j]] = j;
        std::vector<L3Gate> l3;
        for (int i : G) {
            const GateN &gt = gates[i];
            L3Gate x;
            x.gate = i;
            x.kind = gt.kind;
            x.tq0 = tl[gt.q[0]];
            x.tq1 = gt.nq > 1 ? tl[gt.q[1]] : -1;
            x.t = (1u << x.tq0) | (x.tq1 >= 0 ? 1u << x.tq1 : 0u);
            x.mix = x.t;   // every qubit of the gate is a register bit
            x.ctrl = gt.ctrlmask ? 1u << x.tq0 : 0u;
            x.diag = gt.diag_q >= 0 ? tl[gt.diag_q] : -1;
            l3.push_back(x);
        }
        int ld[6], st[6], nld = 0, nst = 0;
        if (relayout) {
            for (int j = 0; j < keff; ++j)
                if (pa.tphys[j] < cl) ld[nld++] = j;
            for (int ppos = 0; ppos < cl; ++ppos)
                for (int j = 0; j < keff; ++j)
                    if (pa.tphys_out[j] == ppos) st[nst++] = j;
        } else {
            // tile bits 0..3 (16 lanes cover a 128-byte run)
            for (int j = 0; j < 4 && j < keff; ++j) ld[nld++] = st[nst++] = j;
        }
        pa.phase0 = (int)out.phases.size();
        plan_phases(keff, rb, l3, out, ld, nld, st, nst);
        pa.nphase = (int)out.phases.size() - pa.phase0;
        choose_swizzle(keff, out, pa, ld, nld, st, nst);
    };
    for (const L1Tile &T : tiles) {
        if (local_set(lay, nL) != T.local) {
            Step s;
            s.type = 0;
            s.qr = remap(lay, nL, T.local);
            out.steps.push_back(s);
            out.n_qr += 1;
        }
        if (!relayout) {
            std::vector<uint64_t> pt(m, 0);
            for (int i : T.ops) pt[i] = phys_mask(targets[i], lay);
            std::vector<int> remain = T.ops;
            while (!remain.empty()) {
                const uint64_t S = choose_pass_set(localpos, forced, remain, pt, keff);
                std::vector<int> G = tile_construction(S, remain, pt);
                if (G.empty()) return "internal: empty gate pass";
                remain = without(remain, G, m);
                PassArgs pa;
                std::memset(&pa, 0, sizeof(pa));
                std::vector<int> qin(keff);
                int j = 0;
                for (uint64_t u = S; u; u &= u - 1, ++j) {
                    pa.tphys[j] = pa.tphys_out[j] = __builtin_ctzll(u);
                    for (int q = 0; q < n; ++q)
                        if (lay[q] == pa.tphys[j]) qin[j] = q;
                }
                pa.nblocks = 1 << (n - keff);
                level3(pa, G, qin);
                Step s;
                s.type = 1;
                s.idx = (int)out.passes.size();
                out.steps.push_back(s);
                add_positions(G, T);
                out.passes.push_back(pa);
            }
            ++qrtile;
            continue;
        }
        // relabelling passes
        uint64_t kprev = 0;
        for (int q = 0; q < n; ++q)
            if (lay[q] < ceff) kprev |= bit(q);
        const int first = (int)out.passes.size();
        std::vector<std::vector<int>> Gs, qins;
        std::vector<int> remain = T.ops;
        while (!remain.empty()) {
            const uint64_t S = rl_choose(T.local, kprev, remain, targets, keff, ceff, lay);
            std::vector<int> G = tile_construction(S, remain, targets);
            if (G.empty()) return "internal: empty gate pass";
            remain = without(remain, G, m);
            if ((int)out.passes.size() > first) {
                // the previous pass stores its qubits relabelled: those of S
                // on its lowest positions (c of them on the c lowest), the
                // others above
                PassArgs &pp = out.passes.back();
                const std::vector<int> &qp = qins.back();
                std::vector<int> A, B;
                for (int j = 0; j < keff; ++j) ((S >> qp[j]) & 1 ? A : B).push_back(qp[j]);
                if ((int)A.size() < ceff) return "internal: relabelled pass lacks low qubits";
                std::vector<int> order = A;
                order.insert(order.end(), B.begin(), B.end());
                for (int i = 0; i < keff; ++i) lay[order[i]] = pp.tphys[i];   // tphys ascending
                for (int j = 0; j < keff; ++j) pp.tphys_out[j] = lay[qp[j]];
            }
            const uint64_t Tm = phys_mask(S, lay);
            if (popc(Tm) != keff || (Tm & forced) != forced || (Tm & ~localpos))
                return "internal: relabelled tile misses the low positions";
            PassArgs pa;
            std::memset(&pa, 0, sizeof(pa));
            std::vector<int> qin(keff);
            int j = 0;
            for (uint64_t u = Tm; u; u &= u - 1, ++j) {
                pa.tphys[j] = pa.tphys_out[j] = __builtin_ctzll(u);
                for (int q = 0; q < n; ++q)
                    if (lay[q] == pa.tphys[j]) qin[j] = q;
            }
            pa.nblocks = 1 << (n - keff);
            Step s;
            s.type = 1;
            s.idx = (int)out.passes.size();
            out.steps.push_back(s);
            add_positions(G, T);
            out.passes.push_back(pa);
            Gs.push_back(G);
            qins.push_back(qin);
            kprev = S;
        }
        for (size_t i = 0; i < Gs.size(); ++i) level3(out.passes[first + i], Gs[i], qins[i]);
        ++qrtile;
    }
    out.pos_after = lay;
    return "";
}

// ---------------------------------------------------------------------------
// op coefficients
// ---------------------------------------------------------------------------

static void set_c(double *m, int idx, double re, double im) {
    m[2 * idx] = re;
    m[2 * idx + 1] = im;
}

// Shear parameters of the rotation with cosine c and sine s (see OpDesc).
static void set_shear(OpDesc &o, int i, double c, double s) {
    if (c < 0) {
        c = -c;
        s = -s;
        o.flip |= 1 << i;
    }
    o.sh[2 * i] = s / (1.0 + c);
    o.sh[2 * i + 1] = s;
}

static void set_shears(OpDesc &o) {
    o.flip = 0;
    switch (o.type) {
    case OP_GIVENS: case OP_ROTY: set_shear(o, 0, o.m[0], o.m[1]); break;
    case OP_CPHASE: set_shear(o, 0, o.m[2], o.m[3]); break;
    case OP_DIAG1:
        set_shear(o, 0, o.m[0], o.m[1]);
        set_shear(o, 1, o.m[2], o.m[3]);
        break;
    default: break;
    }
}

void fill_ops(const std::vector<GateN> &gates, const double *theta, const std::vector<int> &op_gate,
              std::vector<OpDesc> &ops, bool inverse) {
    const double r2 = 1.0 / std::sqrt(2.0);
    for (size_t i = 0; i < ops.size(); ++i) {
        const GateN &g = gates[op_gate[i]];
        OpDesc &o = ops[i];
        const double t = g.param >= 0 ? g.scale * theta[g.param] + g.offset : g.offset;
        const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
        double *m = o.m;
        std::memset(m, 0, sizeof(o.m));
        std::memset(o.k, 0, sizeof(o.k));
        o.gtype = GEN_NONE;
        switch (g.kind) {
        case SVQ_H: set_c(m, 0, r2, 0); set_c(m, 1, r2, 0); set_c(m, 2, r2, 0); set_c(m, 3, -r2, 0); break;
        case SVQ_Y: set_c(m, 1, 0, -1); set_c(m, 2, 0, 1); break;
        case SVQ_RX:
            set_c(m, 0, c, 0); set_c(m, 1, 0, -s); set_c(m, 2, 0, -s); set_c(m, 3, c, 0);
            o.gtype = GEN_MIX1; set_c(o.k, 1, 0.5, 0); set_c(o.k, 2, 0.5, 0);
            break;
        case SVQ_RY:
            m[0] = c; m[1] = s;
            o.gtype = GEN_MIX1; set_c(o.k, 1, 0, -0.5); set_c(o.k, 2, 0, 0.5);
            break;
        case SVQ_U1:
            for (int j = 0; j < 8; ++j) m[j] = g.mat[j];
            break;
        case SVQ_Z: set_c(m, 0, 1, 0); set_c(m, 1, -1, 0); break;
        case SVQ_S: set_c(m, 0, 1, 0); set_c(m, 1, 0, 1); break;
        case SVQ_T: set_c(m, 0, 1, 0); set_c(m, 1, r2, r2); break;
        case SVQ_RZ:
            set_c(m, 0, c, -s);
            set_c(m, 1, c, s);
            o.gtype = GEN_DIAG1; o.k[0] = 0.5; o.k[1] = -0.5;
            break;
        case SVQ_CZ: set_c(m, 1, -1, 0); break;
        case SVQ_CPHASE:
            set_c(m, 1, std::cos(t), std::sin(t));
            o.gtype = GEN_CPHASE;
            break;
        case SVQ_GIVENS:
            m[0] = c; m[1] = s;
            o.gtype = GEN_GIVENS;
            break;
        case SVQ_SWAP:
            set_c(m, 0, 1, 0); set_c(m, 1 * 4 + 2, 1, 0); set_c(m, 2 * 4 + 1, 1, 0); set_c(m, 15, 1, 0);
            break;
        case SVQ_U2:
            for (int j = 0; j < 32; ++j) m[j] = g.mat[j];
            break;
        default:   // X, CNOT: pure swaps
            break;
        }
        if (g.param < 0) o.gtype = GEN_NONE;
        // Chain rule: the angle is scale * theta + offset, so the derivative
        // by theta is scale * 2 Im <lambda|K|psi>; the scale is folded into
        // the explicit generator entries, or kept in k[0] for the kinds whose
        // generator the kernels hard-code.
        if (o.gtype == GEN_MIX1 || o.gtype == GEN_DIAG1) {
            for (double &kv : o.k) kv *= g.scale;
        } else if (o.gtype == GEN_CPHASE || o.gtype == GEN_GIVENS) {
            o.k[0] = g.scale;
        }
        if (!inverse) {
            set_shears(o);
            continue;
        }
        switch (o.type) {   // U^dagger
        case OP_DIAG1: case OP_CPHASE:
            m[1] = -m[1];
            m[3] = -m[3];
            break;
        case OP_GIVENS: case OP_ROTY:
            m[1] = -m[1];
            break;
        case OP_MIX1: case OP_MIX2: {
            const int d = o.type == OP_MIX1 ? 2 : 4;
            double tmp[32];
            for (int r = 0; r < d; ++r)
                for (int cc = 0; cc < d; ++cc) {
                    tmp[2 * (r * d + cc)] = m[2 * (cc * d + r)];
                    tmp[2 * (r * d + cc) + 1] = -m[2 * (cc * d + r) + 1];
                }
            std::memcpy(m, tmp, sizeof(double) * 2 * d * d);
            break;
        }
        default:
            break;
        }
        set_shears(o);
    }
}

// ---------------------------------------------------------------------------
// Pauli plan
// ---------------------------------------------------------------------------

static uint32_t pext32(uint32_t v, const int32_t *bits, int nb) {
    uint32_t out = 0;
    for (int i = 0; i < nb; ++i)
        if ((v >> bits[i]) & 1) out |= 1u << i;
    return out;
}

// The bits of v at the positions set in m, packed towards bit 0.
static uint64_t pext64(uint64_t v, uint64_t m) {
    uint64_t out = 0;
    int i = 0;
    for (; m; m &= m - 1, ++i)
        if (v & m & (~m + 1)) out |= 1ULL << i;
    return out;
}

std::string plan_paulis(int n, int g, const svq_pauli *terms, int nt, svq_sched sched, int k,
                        int c, bool dbl, const std::vector<int> &pos0, PauliPlan &out) {
    out = PauliPlan();
    out.n = n;
    out.g = g;
    const int nL = n - g;
    const int keff = std::min(k, nL);
    const int ceff = std::min(c, keff);
    out.k = keff;
    out.c = ceff;
    const uint64_t full = n >= 64 ? ~0ULL : (bit(n) - 1);
    // group by flip mask, first appearance order
    std::unordered_map<uint64_t, int> gid;
    out.group_of_term.resize(nt);
    for (int t = 0; t < nt; ++t) {
        if ((terms[t].x & ~full) || (terms[t].z & ~full)) return "pauli mask beyond n qubits";
        if (!std::isfinite(terms[t].coef)) return "non-finite coefficient";
        auto it = gid.find(terms[t].x);
        int id;
        if (it == gid.end()) {
            id = (int)out.group_x.size();
            gid[terms[t].x] = id;
            out.group_x.push_back(terms[t].x);
            out.group_terms.emplace_back();
        } else {
            id = it->second;
        }
        out.group_of_term[t] = id;
        out.group_terms[id].push_back(t);
    }
    const int ng = (int)out.group_x.size();
    // level 1 over groups (lazy) or terms in index order (eager)
    std::vector<int> pos = pos0;
    out.pos_before = pos;
    std::vector<char> wide(ng, 0);
    for (int i = 0; i < ng; ++i)
        if (popc(out.group_x[i]) > nL) wide[i] = 1;
    struct GTile { uint64_t local; std::vector<int> groups; std::vector<Transposition> qr; };
    std::vector<GTile> gtiles;
    if (sched == SVQ_LAZY) {
        std::vector<uint64_t> sup;
        std::vector<int> w, ids;
        for (int i = 0; i < ng; ++i) {
            if (wide[i]) continue;
            sup.push_back(out.group_x[i]);
            w.push_back((int)out.group_terms[i].size());
            ids.push_back(i);
        }
        std::vector<L1Tile> t1 = tiling_pauli(n, nL, sup, w, pos);
        for (auto &t : t1) {
            GTile gt;
            gt.local = t.local;
            gt.qr = t.qr;
            for (int i : t.ops) gt.groups.push_back(ids[i]);
            gtiles.push_back(std::move(gt));
        }
    } else {
        std::vector<uint64_t> tg;
        std::vector<int> ord;
        std::vector<int> term_ids;
        for (int t = 0; t < nt; ++t) {
            if (wide[out.group_of_term[t]]) continue;
            tg.push_back(terms[t].x);
            ord.push_back((int)ord.size());
            term_ids.push_back(t);
        }
        std::vector<L1Tile> t1 = ad_hoc(n, nL, tg, ord, pos);
        for (auto &t : t1) {
            GTile gt;
            gt.local = t.local;
            gt.qr = t.qr;
            std::vector<char> seen(ng, 0);
            for (int i : t.ops) {
                int gi = out.group_of_term[term_ids[i]];
                if (!seen[gi]) {
                    seen[gi] = 1;
                    gt.groups.push_back(gi);
                }
            }
            gtiles.push_back(std::move(gt));
        }
    }
    out.pos_after = pos;
    for (int i = 0; i < ng; ++i)
        if (wide[i]) out.wide_groups.push_back(i);
    // For eager, a group may appear in several QR tiles (its terms were split
    // by intervening reorders); it is evaluated once, in its first tile.
    std::vector<char> done(ng, 0);

    const int TPB = evc_tpb(keff, dbl);   // EVC threads per tile (log2)
    const int Q = keff - 1 - TPB;      // EVC cube bits (half space)
    const int TPBH = hpsi_tpb(keff);   // H|psi> threads per tile (log2)
    const int QH = keff - TPBH;        // H|psi> cube bits (full space)
    if (keff < 8) return "tile too small for the Pauli pass";
    std::vector<int> lay = pos0;
    const uint64_t forced = bit(ceff) - 1;
    const uint64_t localpos = bit(nL) - 1;
    int qrtile = 0;
    for (const GTile &T : gtiles) {
        if (!T.qr.empty()) {
            Step s;
            s.type = 0;
            s.qr = T.qr;
            out.steps.push_back(s);
            out.n_qr += 1;
            for (const Transposition &tr : T.qr)
                for (int q = 0; q < n; ++q) {
                    if (lay[q] == tr.a) lay[q] = tr.b;
                    else if (lay[q] == tr.b) lay[q] = tr.a;
                }
        }
        // physical flip masks of this tile's groups
        std::vector<int> rem;
        std::vector<uint64_t> px(ng, 0);
        for (int gi : T.groups) {
            if (done[gi]) continue;
            done[gi] = 1;
            px[gi] = phys_mask(out.group_x[gi], lay);
            if (popc(px[gi] & ~forced) > keff - ceff) {
                out.wide_groups.push_back(gi);   // fits no tile: direct kernel
                continue;
            }
            rem.push_back(gi);
        }
        // level 2: cover the flip masks by k-bit tiles that contain the forced
        // low bits.  The groups commute, so any cover is valid: a greedy
        // (fewest new bits, then most terms, then a fill with the bits most
        // used by the remaining groups), and the same greedy followed by a
        // local search that swaps single bits while that covers more groups
        // in the pass.  The packing with fewer passes is kept.
        auto cover_pass = [&](const std::vector<int> &rem, bool search) {
            uint64_t S = forced;
            std::vector<char> in(ng, 0);
            while (true) {
                int best = -1, bneed = 99;
                size_t bw = 0;
                for (int gi : rem) {
                    if (in[gi]) continue;
                    int need = popc(px[gi] & ~S);
                    if (popc(S) + need > keff) continue;
                    size_t w = out.group_terms[gi].size();
                    if (need < bneed || (need == bneed && w > bw)) {
                        best = gi;
                        bneed = need;
                        bw = w;
                    }
                }
                if (best < 0) break;
                S |= px[best];
                for (int gi : rem)
                    if (!in[gi] && (px[gi] & ~S) == 0) in[gi] = 1;
            }
            // fill up with the most used free local bits of the remaining groups
            while (popc(S) < keff) {
                int cnt[64] = {0};
                for (int gi : rem)
                    if (!in[gi])
                        for (uint64_t v = px[gi] & ~S; v; v &= v - 1) cnt[__builtin_ctzll(v)]++;
                int bb = -1, bc = -1;
                for (int b = 0; b < nL; ++b)
                    if (!((S >> b) & 1) && ((localpos >> b) & 1) && cnt[b] > bc) {
                        bc = cnt[b];
                        bb = b;
                    }
                if (bb < 0) break;
                S |= bit(bb);
            }
            if (search) {
                auto covered = [&](uint64_t X) {
                    int c = 0;
                    for (int gi : rem) c += (px[gi] & ~X) == 0;
                    return c;
                };
                int cur = covered(S);
                for (int iter = 0; iter < 64; ++iter) {
                    int best = cur;
                    uint64_t bestS = S;
                    for (uint64_t o = S & ~forced; o; o &= o - 1) {
                        const uint64_t bo = o & (~o + 1);
                        for (uint64_t i = localpos & ~S; i; i &= i - 1) {
                            const uint64_t X = (S & ~bo) | (i & (~i + 1));
                            const int c = covered(X);
                            if (c > best) {
                                best = c;
                                bestS = X;
                            }
                        }
                    }
                    if (best <= cur) break;
                    cur = best;
                    S = bestS;
                }
            }
            return S;
        };
        auto pack = [&](bool search) {
            std::vector<uint64_t> seq;
            std::vector<int> r = rem;
            while (!r.empty()) {
                const uint64_t S = cover_pass(r, search);
                std::vector<int> rest;
                for (int gi : r)
                    if (px[gi] & ~S) rest.push_back(gi);
                if (rest.size() == r.size()) break;   // no progress (cannot happen)
                seq.push_back(S);
                r.swap(rest);
            }
            return seq;
        };
        const std::vector<uint64_t> seqA = pack(false), seqB = pack(true);
        const std::vector<uint64_t> &seqS = seqB.size() < seqA.size() ? seqB : seqA;
        size_t pass_i = 0;
        while (!rem.empty() && pass_i < seqS.size()) {
            const uint64_t S = seqS[pass_i++];
            std::vector<char> in(ng, 0);
            for (int gi : rem) in[gi] = (px[gi] & ~S) == 0;
            std::vector<int> pg, rest;
            for (int gi : rem) (in[gi] ? pg : rest).push_back(gi);
            rem.swap(rest);
            // ---- emit EVC pass
            EvcPassArgs ea;
            std::memset(&ea, 0, sizeof(ea));
            int8_t tph[16];
            {
                int j = 0;
                for (uint64_t s = S; s; s &= s - 1) tph[j++] = (int8_t)__builtin_ctzll(s);
            }
            std::memcpy(ea.tphys, tph, 16);
            // the block index's bits are the physical bits outside the tile,
            // in ascending order
            const uint64_t nontile = ~S & ((n >= 64 ? 0 : (1ULL << n)) - 1);
            ea.group0 = (int)out.groups.size();
            ea.ngroups = (int)pg.size();
            ea.nblocks = 1 << (n - keff);
            ea.part0 = out.total_blocks;
            out.total_blocks += ea.nblocks;
            // ---- emit H|psi> pass (fixed cube: top QH tile bits)
            HpsiPassArgs ha;
            std::memset(&ha, 0, sizeof(ha));
            std::memcpy(ha.tphys, tph, 16);
            for (int j = 0; j < TPBH; ++j) ha.tbits[j] = (int8_t)j;
            for (int j = 0; j < QH; ++j) ha.wbits[j] = (int8_t)(TPBH + j);
            ha.group0 = (int)out.hgroups.size();
            ha.ngroups = (int)pg.size();
            ha.accumulate = out.hpasses.empty() ? 0 : 1;
            const uint32_t htmask = (1u << TPBH) - 1;
            for (int gi : pg) {
                const uint32_t xl = to_tile(px[gi], S);
                EvcGroup G;
                std::memset(&G, 0, sizeof(G));
                G.xl = xl;
                G.hbit = xl ? 31 - __builtin_clz(xl) : keff - 1;
                int nb = 0;
                for (int b = 0; b < keff; ++b) {
                    if (b == G.hbit) continue;
                    if (nb < TPB) G.tbits[nb] = b;
                    else G.wbits[nb - TPB] = b;
                    ++nb;
                }
                // The Pauli pass derives a thread's tile index from hbit alone
                // (its thread index with a zero inserted at hbit), so the
                // thread-index bits must be the lowest TPB tile bits other
                // than hbit.
                uint32_t tmask = 0;
                for (int j = 0; j < TPB; ++j) {
                    if (G.tbits[j] != j + (j >= G.hbit ? 1 : 0))
                        return "internal: Pauli group thread bits are not the lowest tile bits";
                    tmask |= 1u << G.tbits[j];
                }
                G.t0 = (int)out.terms.size();
                G.nt = (int)out.group_terms[gi].size();
                HpsiGroup HG;
                std::memset(&HG, 0, sizeof(HG));
                HG.xl = xl;
                HG.xt = xl & htmask;
                HG.xw = xl >> TPBH;
                HG.t0 = (int)out.hterms.size();
                HG.nt = G.nt;
                for (int t : out.group_terms[gi]) {
                    const uint64_t pz = phys_mask(terms[t].z, lay);
                    const uint32_t zl = to_tile(pz, S);
                    const uint64_t zg = pz & ~S;
                    const int nY = popc(terms[t].x & terms[t].z);
                    EvcTerm et;
                    std::memset(&et, 0, sizeof(et));
                    int use_im;
                    if (xl) {
                        // pair (j, j^x) over j with bit h clear:
                        // nY even: 2 (-1)^{nY/2} s_j Re w ; nY odd: 2 (-1)^{(nY+1)/2} s_j Im w
                        if ((nY & 1) == 0) {
                            et.coef = 2.0 * terms[t].coef * (((nY / 2) & 1) ? -1.0 : 1.0);
                            use_im = 0;
                        } else {
                            et.coef = 2.0 * terms[t].coef * ((((nY + 1) / 2) & 1) ? -1.0 : 1.0);
                            use_im = 1;
                        }
                    } else {
                        et.coef = terms[t].coef;
                        use_im = (zl >> G.hbit) & 1;   // difference array
                    }
                    const uint32_t zr = zl & ~(1u << G.hbit);
                    const uint32_t wi = pext32(zr, G.wbits, Q) | (use_im ? 1u << Q : 0u);
                    et.ztw = (zr & tmask) | (wi << kEvcWiShift);
                    et.zb = (uint32_t)pext64(zg, nontile);
                    G.need |= use_im ? 2 : 1;
                    out.terms.push_back(et);
                    HpsiTerm ht;
                    std::memset(&ht, 0, sizeof(ht));
                    const double a = terms[t].coef;
                    switch (nY & 3) {
                    case 0: ht.are = a; ht.aim = 0; break;
                    case 1: ht.are = 0; ht.aim = a; break;
                    case 2: ht.are = -a; ht.aim = 0; break;
                    default: ht.are = 0; ht.aim = -a; break;
                    }
                    // (-1)^(cube z bits . xw): the H|psi> pass reads the
                    // transformed spectrum XOR-shifted by xw
                    if (__builtin_popcount((zl >> TPBH) & HG.xw) & 1) {
                        ht.are = -ht.are;
                        ht.aim = -ht.aim;
                    }
                    ht.are_f = (float)ht.are;
                    ht.aim_f = (float)ht.aim;
                    ht.ztw = (zl & htmask) | ((zl >> TPBH) << kHpsiZwShift);
                    ht.zb = (uint32_t)pext64(zg, nontile);
                    out.hterms.push_back(ht);
                }
                out.groups.push_back(G);
                out.hgroups.push_back(HG);
                out.order.push_back(gi);
                out.pos_qrtile.push_back(qrtile);
                out.pos_pass.push_back((int)out.passes.size());
                out.pos_local.push_back(T.local);
            }
            Step s;
            s.type = 1;
            s.idx = (int)out.passes.size();
            out.steps.push_back(s);
            out.passes.push_back(ea);
            out.hpasses.push_back(ha);
        }
        if (!rem.empty()) return "internal: Pauli packing left groups uncovered";
        ++qrtile;
    }
    // The Pauli and H|psi> passes find a group's first term from the previous
    // group's range and load its first four terms with its descriptor,
    // before they know its term count: the ranges of a pass must be
    // consecutive, and four zero terms at the end keep those loads inside
    // the table.  (groups and hgroups are filled in step: one index.)
    for (const EvcPassArgs &ea : out.passes)
        for (int i = 1; i < ea.ngroups; ++i) {
            const EvcGroup &p = out.groups[ea.group0 + i - 1], &q = out.groups[ea.group0 + i];
            const HpsiGroup &hp = out.hgroups[ea.group0 + i - 1], &hq = out.hgroups[ea.group0 + i];
            if (q.t0 != p.t0 + p.nt || hq.t0 != hp.t0 + hp.nt)
                return "internal: a Pauli pass's term ranges are not consecutive";
        }
    out.terms.resize(out.terms.size() + 4, EvcTerm{});
    out.hterms.resize(out.hterms.size() + 4, HpsiTerm{});
    return "";
}

}  // namespace svq
