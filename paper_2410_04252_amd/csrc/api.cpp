// C ABI of libsvq.so (declared in include/svq.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "svq.h"

using namespace svq;

namespace {

thread_local std::string g_err;

svq_status fail(svq_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

// Largest single device allocation the library makes (SVQ_MAX_ALLOC_BYTES,
// default unlimited); a larger request fails as out of memory, which lets the
// ENOMEM paths be exercised without exhausting the device.
size_t alloc_cap() {
    const char *v = std::getenv("SVQ_MAX_ALLOC_BYTES");
    if (!v || !*v) return SIZE_MAX;
    return (size_t)std::strtoull(v, nullptr, 10);
}

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap) return hipSuccess;
        if (std::max<size_t>(bytes, 256) > alloc_cap()) return hipErrorOutOfMemory;
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            cap = 0;
        }
        size_t want = std::max<size_t>(bytes, 256);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        return e;
    }
};

struct CachedCircuit {
    CircuitPlan plan;
    DevBuf d_phases;
    std::shared_ptr<const std::string> json;   // sv_plan_dump text
};

// Host-only circuit plan (sv_apply_circuit_static keeps its tables in the
// library's static device scratch, not in per-plan device buffers).
struct HostCircuit {
    CircuitPlan plan;
    std::shared_ptr<const std::string> json;
};

struct CachedPaulis {
    PauliPlan plan;
    std::vector<WideTerm> wide;
    DevBuf d_groups, d_terms, d_hgroups, d_hterms, d_off, d_nblk, d_wide;
    std::shared_ptr<const std::string> json;
};

// ---- sv_plan_dump: the executed steps of a plan as JSON ----------------------

void json_qr(std::string &o, const std::vector<Transposition> &tr) {
    o += "{\"type\":\"qr\",\"swaps\":[";
    for (size_t i = 0; i < tr.size(); ++i) {
        if (i) o += ",";
        o += "[" + std::to_string(tr[i].a) + "," + std::to_string(tr[i].b) + "]";
    }
    o += "]}";
}

template <typename T>
void json_bits(std::string &o, const T *bits, int nb) {
    o += "[";
    for (int j = 0; j < nb; ++j) {
        if (j) o += ",";
        o += std::to_string((int)bits[j]);
    }
    o += "]";
}

std::string circuit_json(const CircuitPlan &P, svq_sched sched, bool adj) {
    std::vector<int> gates_in_pass(P.passes.size(), 0);
    for (int p : P.pos_pass) gates_in_pass[p]++;
    std::string o = "{\"kind\":\"circuit\",\"schedule\":\"";
    o += sched == SVQ_LAZY ? "lazy" : "eager";
    o += "\",\"adjoint\":" + std::string(adj ? "true" : "false");
    o += ",\"n\":" + std::to_string(P.n) + ",\"g\":" + std::to_string(P.g);
    o += ",\"tile_k\":" + std::to_string(P.k) + ",\"low_bits\":" + std::to_string(P.c);
    o += ",\"reg_bits\":" + std::to_string(P.rb) + ",\"n_qr\":" + std::to_string(P.n_qr);
    o += ",\"n_passes\":" + std::to_string(P.passes.size());
    o += ",\"order\":[";
    for (size_t i = 0; i < P.order.size(); ++i) o += (i ? "," : "") + std::to_string(P.order[i]);
    o += "],\"steps\":[";
    bool first = true;
    for (const Step &s : P.steps) {
        if (!first) o += ",";
        first = false;
        if (s.type == 0) {
            json_qr(o, s.qr);
            continue;
        }
        const PassArgs &a = P.passes[s.idx];
        o += "{\"type\":\"gate_pass\",\"pass\":" + std::to_string(s.idx) + ",\"tile_bits\":";
        json_bits(o, a.tphys, P.k);
        o += ",\"tile_bits_out\":";
        json_bits(o, a.tphys_out, P.k);
        o += ",\"swz\":";
        json_bits(o, a.swz, P.k);
        o += ",\"gates\":" + std::to_string(gates_in_pass[s.idx]);
        o += ",\"phases\":" + std::to_string(a.nphase) + ",\"lanes\":[";
        for (int ph = 0; ph < a.nphase; ++ph) {
            if (ph) o += ",";
            json_bits(o, P.phases[a.phase0 + ph].lane, 6);
        }
        o += "],\"regs\":[";
        for (int ph = 0; ph < a.nphase; ++ph) {
            if (ph) o += ",";
            json_bits(o, P.phases[a.phase0 + ph].reg, P.rb);
        }
        o += "]}";
    }
    o += "],\"pos_before\":[";
    for (size_t q = 0; q < P.pos_before.size(); ++q) o += (q ? "," : "") + std::to_string(P.pos_before[q]);
    o += "],\"pos_after\":[";
    for (size_t q = 0; q < P.pos_after.size(); ++q) o += (q ? "," : "") + std::to_string(P.pos_after[q]);
    o += "]}";
    return o;
}

std::string pauli_json(const PauliPlan &P, svq_sched sched) {
    std::string o = "{\"kind\":\"paulis\",\"schedule\":\"";
    o += sched == SVQ_LAZY ? "lazy" : "eager";
    o += "\",\"n\":" + std::to_string(P.n) + ",\"g\":" + std::to_string(P.g);
    o += ",\"tile_k\":" + std::to_string(P.k) + ",\"low_bits\":" + std::to_string(P.c);
    o += ",\"n_qr\":" + std::to_string(P.n_qr) + ",\"n_groups\":" + std::to_string(P.group_x.size());
    o += ",\"n_passes\":" + std::to_string(P.passes.size());
    o += ",\"wide_groups\":" + std::to_string(P.wide_groups.size());
    o += ",\"group_order\":[";
    for (size_t i = 0; i < P.order.size(); ++i) o += (i ? "," : "") + std::to_string(P.order[i]);
    o += "],\"steps\":[";
    bool first = true;
    for (const Step &s : P.steps) {
        if (!first) o += ",";
        first = false;
        if (s.type == 0) {
            json_qr(o, s.qr);
            continue;
        }
        const EvcPassArgs &a = P.passes[s.idx];
        o += "{\"type\":\"pauli_pass\",\"pass\":" + std::to_string(s.idx) + ",\"tile_bits\":";
        json_bits(o, a.tphys, P.k);
        o += ",\"groups\":" + std::to_string(a.ngroups) + "}";
    }
    o += "],\"pos_before\":[";
    for (size_t q = 0; q < P.pos_before.size(); ++q) o += (q ? "," : "") + std::to_string(P.pos_before[q]);
    o += "],\"pos_after\":[";
    for (size_t q = 0; q < P.pos_after.size(); ++q) o += (q ? "," : "") + std::to_string(P.pos_after[q]);
    o += "]}";
    return o;
}

int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

// Gate passes relabel their tile's positions on store (PassArgs::tphys_out)
// unless SVQ_RELAYOUT=0.
bool relayout_on() { return env_int("SVQ_RELAYOUT", 1) != 0; }

}  // namespace

struct svq_state_s {
    int n = 0, g = 0;
    svq_dtype dtype = SVQ_C64;
    void *buf = nullptr;
    bool owns = false;
    hipStream_t stream = nullptr;
    std::vector<int> pos;
    bool poisoned = false;
    std::map<std::string, std::unique_ptr<CachedCircuit>> ccache;
    std::map<std::string, std::unique_ptr<CachedPaulis>> pcache;
    std::map<std::string, std::unique_ptr<HostCircuit>> hcache;
    std::shared_ptr<const std::string> last_plan;   // JSON of the last executed plan
    DevBuf d_ops, d_partials, d_chunks, d_extra, d_lam, d_gpart, d_gop, d_ggates, d_pptr, d_pgate,
        d_energy, d_grad;
    int device = 0;
    // per-launch event timing (sv_profile)
    double traffic = 0.0;   // algorithmic HBM bytes of every launch so far
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_rec;

    ~svq_state_s() {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }

    bool dbl() const { return dtype == SVQ_C128; }
    size_t esz() const { return dbl() ? 16 : 8; }
    uint64_t N() const { return 1ULL << n; }
    size_t bytes() const { return (size_t)N() * esz(); }
};

namespace {

hipEvent_t prof_event(svq_state st) {
    if (st->ev_used == st->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        st->ev_pool.push_back(e);
    }
    return st->ev_pool[st->ev_used++];
}

// Bracket one launch of `kind` with events when profiling is on.
struct ProfScope {
    svq_state st;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(svq_state s, int k) : st(s), kind(k) {
        if (!st->prof) return;
        a = prof_event(st);
        b = prof_event(st);
        if (a) (void)hipEventRecord(a, st->stream);
    }
    ~ProfScope() {
        if (!st->prof || !a || !b) return;
        (void)hipEventRecord(b, st->stream);
        st->prof_rec.push_back({kind, {a, b}});
    }
};

// A failed device allocation is ENOMEM and leaves the handle usable: every
// entry point allocates its scratch before its first launch.  Any other HIP
// failure poisons the handle.
svq_status hip_fail(svq_state st, hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory) return fail(SVQ_ENOMEM, std::string(what) + ": out of device memory");
    if (st) st->poisoned = true;
    return fail(SVQ_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(st, expr, what)                       \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hip_fail(st, _e, what); \
    } while (0)

// ---- tuned table: (kind, n, g, dtype) -> (k, c); kind 0 gate pass, 1 Pauli
// pass, 2 batch (k = items per stage, c = low bits; n = g = 0), 3 batch size
// classes (k = smallest instance on 2^12 tiles, c = 0; n = g = 0) -------------
struct TuneKey {
    int kind, n, g, dt;
    bool operator<(const TuneKey &o) const {
        return std::tie(kind, n, g, dt) < std::tie(o.kind, o.n, o.g, o.dt);
    }
};
struct TuneVal {
    int k, c;
    double ms;
};
std::map<TuneKey, TuneVal> &tune_table() {
    static std::map<TuneKey, TuneVal> t;
    return t;
}
std::mutex &tune_mutex() {
    static std::mutex m;
    return m;
}
bool tuned(int kind, int n, int g, int dt, TuneVal &out) {
    std::lock_guard<std::mutex> lk(tune_mutex());
    auto it = tune_table().find({kind, n, g, dt});
    if (it == tune_table().end()) return false;
    out = it->second;
    return true;
}
void set_tuned(int kind, int n, int g, int dt, TuneVal v) {
    std::lock_guard<std::mutex> lk(tune_mutex());
    tune_table()[{kind, n, g, dt}] = v;
}

// Environment overrides win, then a measured value, then the default.
int default_k(const svq_state_s *st) {
    TuneVal tv;
    int k = st->dbl() ? 12 : 12;
    if (tuned(0, st->n, st->g, (int)st->dtype, tv)) k = tv.k;
    k = env_int("SVQ_TILE_K", k);
    return std::max(8, std::min(13, std::min(k, st->n - st->g)));
}

int default_c(const svq_state_s *st) {
    TuneVal tv;
    int c = 4;
    if (tuned(0, st->n, st->g, (int)st->dtype, tv)) c = tv.c;
    return env_int("SVQ_LOW_BITS", c);
}

// Pauli passes are read-only: a wider tile covers more flip masks per read.
int default_evc_k(const svq_state_s *st) {
    TuneVal tv;
    int k = 12;   // the measured best at 28-32 qubits for both precisions
    if (tuned(1, st->n, st->g, (int)st->dtype, tv)) k = tv.k;
    k = env_int("SVQ_EVC_K", k);
    // one staged tile must fit the 128 KiB the EVC pass reserves in LDS
    return std::max(8, std::min(st->dbl() ? 13 : 14, std::min(k, st->n - st->g)));
}

int default_evc_c(const svq_state_s *st) {
    TuneVal tv;
    int c = 4;
    if (tuned(1, st->n, st->g, (int)st->dtype, tv)) c = tv.c;
    return env_int("SVQ_EVC_LOW_BITS", c);
}

// Build the launch arguments of one QR step (disjoint transpositions).
QrArgs make_qr_args(int n, bool dbl, const std::vector<Transposition> &tr) {
    (void)dbl;
    QrArgs a;
    std::memset(&a, 0, sizeof(a));
    int low = 64;
    for (const auto &t : tr) low = std::min(low, std::min(t.a, t.b));
    if (n >= 7 && low >= 6) {
        a.rows_path = 1;
        a.nrows = 1ULL << (n - 6);
        int top = -1, partner_of_top = -1;
        for (const auto &t : tr) {
            a.outer[2 * a.nouter] = (int8_t)t.a;
            a.outer[2 * a.nouter + 1] = (int8_t)t.b;
            a.nouter++;
            if (std::max(t.a, t.b) > top) {
                top = std::max(t.a, t.b);
                partner_of_top = std::min(t.a, t.b);
            }
        }
        a.hbit = top - 6;
        a.lbit = partner_of_top - 6;
        return a;
    }
    int partner[64];
    for (int i = 0; i < 64; ++i) partner[i] = -1;
    for (const auto &t : tr) {
        partner[t.a] = t.b;
        partner[t.b] = t.a;
    }
    const int clow = std::min(n, 5);
    const int target = std::min(n, 10);
    uint64_t T = 0;
    for (int b = 0; b < clow; ++b) {
        T |= 1ULL << b;
        if (partner[b] >= 0) T |= 1ULL << partner[b];
    }
    // grow to `target` bits with unpaired bits or whole pairs, so that the
    // tile stays closed under the involution
    for (int b = 0; b < n && __builtin_popcountll(T) < target; ++b) {
        if ((T >> b) & 1) continue;
        if (partner[b] < 0) {
            T |= 1ULL << b;
        } else if (!((T >> partner[b]) & 1) && __builtin_popcountll(T) + 2 <= target) {
            T |= (1ULL << b) | (1ULL << partner[b]);
        }
    }
    int j = 0;
    int tl[64];
    for (int b = 0; b < 64; ++b) tl[b] = -1;
    for (int b = 0; b < n; ++b)
        if ((T >> b) & 1) {
            tl[b] = j;
            a.tphys[j++] = (int8_t)b;
        }
    a.tbits = j;
    a.ntiles = 1ULL << (n - j);
    for (const auto &t : tr) {
        const bool ia = (T >> t.a) & 1, ib = (T >> t.b) & 1;
        if (ia && ib) {
            a.inner[2 * a.ninner] = (int8_t)tl[t.a];
            a.inner[2 * a.ninner + 1] = (int8_t)tl[t.b];
            a.ninner++;
        } else {
            a.outer[2 * a.nouter] = (int8_t)t.a;
            a.outer[2 * a.nouter + 1] = (int8_t)t.b;
            a.nouter++;
        }
    }
    // tile path with outer pairs: positions, among the non-tile bits (the
    // tile index), of the highest outer bit and its partner
    int top = -1, ptop = -1;
    for (int i = 0; i < a.nouter; ++i) {
        const int x = a.outer[2 * i], y = a.outer[2 * i + 1];
        if (std::max(x, y) > top) {
            top = std::max(x, y);
            ptop = std::min(x, y);
        }
    }
    if (top >= 0) {
        a.hbit = top - __builtin_popcountll(T & ((1ULL << top) - 1));
        a.lbit = ptop - __builtin_popcountll(T & ((1ULL << ptop) - 1));
    }
    return a;
}

void apply_transpositions(std::vector<int> &pos, const std::vector<Transposition> &tr) {
    for (const auto &t : tr)
        for (auto &p : pos) {
            if (p == t.a) p = t.b;
            else if (p == t.b) p = t.a;
        }
}

double qr_bytes(const svq_state_s *st, const std::vector<Transposition> &tr) {
    return 2.0 * (1.0 - std::ldexp(1.0, -(int)tr.size())) * (double)st->bytes();
}

svq_status run_qr(svq_state st, void *buf, const std::vector<Transposition> &tr) {
    if (tr.empty()) return SVQ_OK;
    QrArgs a = make_qr_args(st->n, st->dbl(), tr);
    ProfScope ps(st, 1);
    HIPCHK(st, launch_qr(st->dbl(), buf, a, st->stream), "qr_permute");
    st->traffic += qr_bytes(st, tr);
    return SVQ_OK;
}

// Split an arbitrary relayout (physical p -> sigma[p]) into two involutions.
void split_relayout(const std::vector<int> &sigma, std::vector<Transposition> &t1,
                    std::vector<Transposition> &t2) {
    const int n = (int)sigma.size();
    std::vector<char> seen(n, 0);
    for (int s = 0; s < n; ++s) {
        if (seen[s]) continue;
        std::vector<int> cyc;
        for (int p = s; !seen[p]; p = sigma[p]) {
            seen[p] = 1;
            cyc.push_back(p);
        }
        const int L = (int)cyc.size();
        if (L == 1) continue;
        if (L == 2) {
            t1.push_back({cyc[0], cyc[1]});
            continue;
        }
        // sigma(c_i) = c_{i+1} = tau2(tau1(c_i)) with the involutions
        // tau1: c_i <-> c_{-i} and tau2: c_i <-> c_{1-i} (indices mod L).
        for (int i = 0; i < L; ++i) {
            const int j1 = (L - i) % L;
            if (i < j1) t1.push_back({cyc[i], cyc[j1]});
            const int j2 = ((1 - i) % L + L) % L;
            if (i < j2) t2.push_back({cyc[i], cyc[j2]});
        }
    }
}

svq_status relayout(svq_state st, void *buf, std::vector<int> &pos, const std::vector<int> &newpos) {
    const int n = st->n;
    std::vector<int> sigma(n);
    for (int q = 0; q < n; ++q) sigma[pos[q]] = newpos[q];
    std::vector<Transposition> t1, t2;
    split_relayout(sigma, t1, t2);
    svq_status s = run_qr(st, buf, t1);
    if (s) return s;
    apply_transpositions(pos, t1);
    s = run_qr(st, buf, t2);
    if (s) return s;
    apply_transpositions(pos, t2);
    return SVQ_OK;
}

std::string circuit_key(const std::vector<GateN> &gates, const svq_state_s *st, svq_sched sched,
                        int k, int c, int rb, bool adj) {
    std::string key;
    auto put = [&](const void *p, size_t nb) { key.append((const char *)p, nb); };
    int hdr[8] = {st->n, st->g, (int)sched, k, c, rb, adj ? 1 : 0, relayout_on() ? 1 : 0};
    put(hdr, sizeof(hdr));
    for (int p : st->pos) put(&p, sizeof(p));
    for (const auto &g : gates) {
        int v[4] = {g.kind, g.q[0], g.q[1], g.param >= 0 ? 1 : 0};
        put(v, sizeof(v));
    }
    return key;
}

svq_status get_circuit_plan(svq_state st, const std::vector<GateN> &gates, svq_sched sched,
                            int k, bool adj, CachedCircuit **out, double *ms_plan) {
    const int c = default_c(st);
    const int rb = gate_rb(k, st->dbl(), adj);
    std::string key = circuit_key(gates, st, sched, k, c, rb, adj);
    auto it = st->ccache.find(key);
    if (it != st->ccache.end()) {
        *out = it->second.get();
        *ms_plan = 0.0;
        return SVQ_OK;
    }
    auto t0 = std::chrono::steady_clock::now();
    auto cc = std::make_unique<CachedCircuit>();
    std::string err = plan_circuit(st->n, st->g, gates, sched, k, rb, c, st->pos, cc->plan,
                                   relayout_on());
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    auto t1 = std::chrono::steady_clock::now();
    *ms_plan = std::chrono::duration<double, std::milli>(t1 - t0).count();
    cc->json = std::make_shared<const std::string>(circuit_json(cc->plan, sched, adj));
    HIPCHK(st, cc->d_phases.ensure(sizeof(PhaseDesc) * std::max<size_t>(1, cc->plan.phases.size())),
           "alloc phases");
    HIPCHK(st, hipMemcpyAsync(cc->d_phases.p, cc->plan.phases.data(),
                              sizeof(PhaseDesc) * cc->plan.phases.size(), hipMemcpyHostToDevice,
                              st->stream),
           "upload phases");
    if (st->ccache.size() > 64) st->ccache.clear();
    *out = cc.get();
    st->ccache[key] = std::move(cc);
    return SVQ_OK;
}

svq_status check_state(svq_state st) {
    if (!st) return fail(SVQ_EINVAL, "null handle");
    if (st->poisoned) return fail(SVQ_EPOISONED, "handle poisoned by an earlier HIP failure");
    HIPCHK(st, hipSetDevice(st->device), "hipSetDevice");
    return SVQ_OK;
}

svq_status check_theta(const std::vector<GateN> &gates, const double *theta, int n_theta) {
    bool any = false;
    for (const auto &g : gates) any |= g.param >= 0;
    if (any && !theta) return fail(SVQ_EINVAL, "theta is NULL but gates reference parameters");
    for (int i = 0; i < n_theta && theta; ++i)
        if (!std::isfinite(theta[i])) return fail(SVQ_EINVAL, "non-finite theta");
    return SVQ_OK;
}

// Forward circuit application with an existing plan.
// The QR and gate-pass launches of a circuit plan whose phase and op tables
// are already on the device.
svq_status run_circuit_steps(svq_state st, const CircuitPlan &P, const PhaseDesc *phases_dev,
                             const OpDesc *ops_dev, svq_stats *stats) {
    double bytes = 0.0;
    for (const Step &s : P.steps) {
        if (s.type == 0) {
            svq_status r = run_qr(st, st->buf, s.qr);
            if (r) return r;
            bytes += qr_bytes(st, s.qr);
        } else {
            const PassArgs &a = P.passes[s.idx];
            ProfScope ps(st, 0);
            HIPCHK(st, launch_gate_pass(st->dbl(), P.k, P.rb, false, st->buf, nullptr, a, phases_dev,
                                        ops_dev, nullptr, a.nblocks, st->stream),
                   "gate_pass");
            bytes += 2.0 * (double)st->bytes();
            st->traffic += 2.0 * (double)st->bytes();
        }
    }
    st->pos = P.pos_after;
    if (stats) {
        stats->n_qr += P.n_qr;
        stats->n_gate_passes += (int)P.passes.size();
        stats->n_phases += P.n_phases_total;
        stats->tile_k = P.k;
        stats->bytes += bytes;
    }
    return SVQ_OK;
}

svq_status run_circuit(svq_state st, CachedCircuit *cc, const std::vector<GateN> &gates,
                       const double *theta, svq_stats *stats) {
    CircuitPlan &P = cc->plan;
    st->last_plan = cc->json;
    std::vector<OpDesc> ops = P.ops;
    fill_ops(gates, theta, P.op_gate, ops, false);
    HIPCHK(st, st->d_ops.ensure(sizeof(OpDesc) * std::max<size_t>(1, ops.size())), "alloc ops");
    HIPCHK(st, hipMemcpyAsync(st->d_ops.p, ops.data(), sizeof(OpDesc) * ops.size(),
                              hipMemcpyHostToDevice, st->stream),
           "upload ops");
    return run_circuit_steps(st, P, (const PhaseDesc *)cc->d_phases.p, (const OpDesc *)st->d_ops.p,
                             stats);
}

std::string pauli_key(const svq_pauli *terms, int nt, const svq_state_s *st, svq_sched sched,
                      int k, int c) {
    std::string key;
    int hdr[6] = {st->n, st->g, (int)sched, k, c, st->dbl() ? 1 : 0};
    key.append((const char *)hdr, sizeof(hdr));
    for (int p : st->pos) key.append((const char *)&p, sizeof(p));
    key.append((const char *)terms, sizeof(svq_pauli) * (size_t)nt);
    return key;
}

svq_status get_pauli_plan(svq_state st, const svq_pauli *terms, int nt, svq_sched sched,
                          CachedPaulis **out, double *ms_plan, bool for_hpsi = false) {
    // H|psi> keeps its FP64 accumulators in VGPRs: at most 2^13-wide tiles
    const int k = for_hpsi ? std::min(default_evc_k(st), 13) : default_evc_k(st);
    const int c = default_evc_c(st);
    std::string key = pauli_key(terms, nt, st, sched, k, c);
    auto it = st->pcache.find(key);
    if (it != st->pcache.end()) {
        *out = it->second.get();
        *ms_plan = 0.0;
        return SVQ_OK;
    }
    auto t0 = std::chrono::steady_clock::now();
    auto cp = std::make_unique<CachedPaulis>();
    std::string err = plan_paulis(st->n, st->g, terms, nt, sched, k, c, st->dbl(), st->pos, cp->plan);
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    PauliPlan &P = cp->plan;
    // wide groups are evaluated directly in the final layout
    for (int gi : P.wide_groups)
        for (int t : P.group_terms[gi]) {
            WideTerm w;
            std::memset(&w, 0, sizeof(w));
            uint64_t x = 0, z = 0;
            for (int q = 0; q < st->n; ++q) {
                if ((terms[t].x >> q) & 1) x |= 1ULL << P.pos_after[q];
                if ((terms[t].z >> q) & 1) z |= 1ULL << P.pos_after[q];
            }
            w.x = x;
            w.z = z;
            w.coef = terms[t].coef;
            w.ny = __builtin_popcountll(terms[t].x & terms[t].z);
            cp->wide.push_back(w);
        }
    auto t1 = std::chrono::steady_clock::now();
    *ms_plan = std::chrono::duration<double, std::milli>(t1 - t0).count();
    cp->json = std::make_shared<const std::string>(pauli_json(P, sched));
    auto up = [&](DevBuf &b, const void *src, size_t nb) -> hipError_t {
        hipError_t e = b.ensure(std::max<size_t>(nb, 64));
        if (e != hipSuccess) return e;
        if (nb) e = hipMemcpyAsync(b.p, src, nb, hipMemcpyHostToDevice, st->stream);
        return e;
    };
    std::vector<int> off, nblk;
    for (const auto &pa : P.passes) {
        off.push_back(pa.part0);
        nblk.push_back(pa.nblocks);
    }
    HIPCHK(st, up(cp->d_groups, P.groups.data(), sizeof(EvcGroup) * P.groups.size()), "upload groups");
    HIPCHK(st, up(cp->d_terms, P.terms.data(), sizeof(EvcTerm) * P.terms.size()), "upload terms");
    HIPCHK(st, up(cp->d_hgroups, P.hgroups.data(), sizeof(HpsiGroup) * P.hgroups.size()), "upload hgroups");
    HIPCHK(st, up(cp->d_hterms, P.hterms.data(), sizeof(HpsiTerm) * P.hterms.size()), "upload hterms");
    HIPCHK(st, up(cp->d_off, off.data(), sizeof(int) * off.size()), "upload offsets");
    HIPCHK(st, up(cp->d_nblk, nblk.data(), sizeof(int) * nblk.size()), "upload nblk");
    HIPCHK(st, up(cp->d_wide, cp->wide.data(), sizeof(WideTerm) * cp->wide.size()), "upload wide");
    // keep host copies alive until the async copies ran
    HIPCHK(st, hipStreamSynchronize(st->stream), "sync");
    if (st->pcache.size() > 16) st->pcache.clear();
    *out = cp.get();
    st->pcache[key] = std::move(cp);
    return SVQ_OK;
}

svq_status run_expectation(svq_state st, CachedPaulis *cp, double *energy_dev, double *chunk_dev,
                           svq_stats *stats) {
    PauliPlan &P = cp->plan;
    st->last_plan = cp->json;
    const int nchunk = 1 << st->g;
    HIPCHK(st, st->d_partials.ensure(sizeof(double) * std::max(1, P.total_blocks)), "alloc partials");
    HIPCHK(st, st->d_chunks.ensure(sizeof(double) * (nchunk + reduce_scratch(nchunk))), "alloc chunks");
    const int dgrid = direct_grid(st->N());
    HIPCHK(st, st->d_extra.ensure(sizeof(double) * dgrid), "alloc extra");
    double bytes = 0.0;
    for (const Step &s : P.steps) {
        if (s.type == 0) {
            svq_status r = run_qr(st, st->buf, s.qr);
            if (r) return r;
            bytes += qr_bytes(st, s.qr);
        } else {
            const EvcPassArgs &a = P.passes[s.idx];
            ProfScope ps(st, 2);
            HIPCHK(st, launch_evc_pass(st->dbl(), P.k, st->buf, a, (const EvcGroup *)cp->d_groups.p,
                                       (const EvcTerm *)cp->d_terms.p, (double *)st->d_partials.p,
                                       st->stream),
                   "evc_pass");
            bytes += (double)st->bytes();
        }
    }
    int nextra = 0;
    if (!cp->wide.empty()) {
        HIPCHK(st, launch_evc_direct(st->dbl(), st->buf, st->N(), (const WideTerm *)cp->d_wide.p,
                                     (int)cp->wide.size(), (double *)st->d_extra.p, st->stream),
               "evc_direct");
        nextra = dgrid;
        bytes += 2.0 * (double)st->bytes();
    }
    double *chunks = chunk_dev ? chunk_dev : (double *)st->d_chunks.p;
    HIPCHK(st, launch_reduce_chunks((const double *)st->d_partials.p, (const int *)cp->d_off.p,
                                    (const int *)cp->d_nblk.p, (int)P.passes.size(), nchunk,
                                    (double *)st->d_chunks.p + nchunk, chunks, st->stream),
           "reduce");
    HIPCHK(st, launch_finish_energy(chunks, nchunk, (const double *)st->d_extra.p, nextra, energy_dev,
                                    st->stream),
           "finish");
    st->pos = P.pos_after;
    if (stats) {
        stats->n_qr += P.n_qr;
        stats->n_evc_passes += (int)P.passes.size();
        stats->n_groups += (int)P.group_x.size();
        stats->bytes += bytes;
    }
    return SVQ_OK;
}

}  // namespace

// ---- static device scratch of sv_apply_circuit_static ------------------------
// At most 4 MiB per GPU, held until the process ends.
constexpr size_t kStaticScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// One array per GPU in the library's code object: the phase and op descriptor
// tables of the call.  Host code never passes `scratch` itself to a kernel
// or a copy (on the host the name is only a stand-in); it resolves the array's
// device address once per device with hipGetSymbolAddress and uses that.

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices];

// The device address of this GPU's scratch (the handle's device is current).
svq_status static_scratch(svq_state st, void **out) {
    if (st->device < 0 || st->device >= kMaxDevices) return fail(SVQ_EUNSUP, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch_ptr[st->device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SVQ_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[st->device] = p;
    }
    *out = g_scratch_ptr[st->device];
    return SVQ_OK;
}

}  // namespace

extern "C" {

const char *sv_last_error(void) { return g_err.c_str(); }

svq_status sv_profile(svq_state st, int enable) {
    if (!st) return fail(SVQ_EINVAL, "null handle");
    st->prof = enable != 0;
    st->prof_rec.clear();
    st->ev_used = 0;
    return SVQ_OK;
}

svq_status sv_profile_read(svq_state st, int kind, int *count, double *total_ms) {
    if (!st || !count || !total_ms) return fail(SVQ_EINVAL, "null argument");
    HIPCHK(st, hipStreamSynchronize(st->stream), "sync");
    int c = 0;
    double t = 0.0;
    for (auto &r : st->prof_rec) {
        if (r.first != kind) continue;
        float ms = 0.f;
        HIPCHK(st, hipEventElapsedTime(&ms, r.second.first, r.second.second), "event time");
        t += ms;
        ++c;
    }
    *count = c;
    *total_ms = t;
    return SVQ_OK;
}

svq_status sv_create(int n, int g, svq_dtype dtype, void *dev_buf, size_t buf_bytes, void *stream,
                     svq_state *out) {
    if (!out) return fail(SVQ_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 34) return fail(SVQ_EINVAL, "n must be in [1, 34]");
    if (g < 0 || g >= n) return fail(SVQ_EINVAL, "g must be in [0, n)");
    if (n - g < 8) return fail(SVQ_EINVAL, "need at least 8 chunk-local qubits (n - g >= 8)");
    if (n - g > 32) return fail(SVQ_EINVAL, "at most 32 chunk-local qubits (n - g <= 32)");
    if (dtype != SVQ_C64 && dtype != SVQ_C128) return fail(SVQ_EINVAL, "bad dtype");
    auto st = std::make_unique<svq_state_s>();
    st->n = n;
    st->g = g;
    st->dtype = dtype;
    st->stream = (hipStream_t)stream;
    st->pos.resize(n);
    for (int q = 0; q < n; ++q) st->pos[q] = q;
    hipError_t e = hipGetDevice(&st->device);
    if (e != hipSuccess) return fail(SVQ_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev_buf) {
        if (buf_bytes < st->bytes()) return fail(SVQ_ESHAPE, "buffer smaller than 2^n amplitudes");
        st->buf = dev_buf;
        st->owns = false;
    } else {
        if (st->bytes() > alloc_cap()) return fail(SVQ_ENOMEM, "state larger than SVQ_MAX_ALLOC_BYTES");
        e = hipMalloc(&st->buf, st->bytes());
        if (e != hipSuccess) return fail(SVQ_ENOMEM, std::string("hipMalloc state: ") + hipGetErrorString(e));
        st->owns = true;
    }
    e = launch_fill_basis(st->dbl(), st->buf, st->N(), 0, st->stream);
    if (e != hipSuccess) {
        if (st->owns) (void)hipFree(st->buf);
        return fail(SVQ_EHIP, std::string("init: ") + hipGetErrorString(e));
    }
    *out = st.release();
    return SVQ_OK;
}

svq_status sv_destroy(svq_state st) {
    if (!st) return fail(SVQ_EINVAL, "null handle");
    (void)hipSetDevice(st->device);
    (void)hipStreamSynchronize(st->stream);
    if (st->owns && st->buf) (void)hipFree(st->buf);
    delete st;
    return SVQ_OK;
}

svq_status sv_set_basis(svq_state st, uint64_t index) {
    svq_status s = check_state(st);
    if (s) return s;
    if (index >= st->N()) return fail(SVQ_EINVAL, "basis index >= 2^n");
    HIPCHK(st, launch_fill_basis(st->dbl(), st->buf, st->N(), index, st->stream), "fill_basis");
    for (int q = 0; q < st->n; ++q) st->pos[q] = q;
    return SVQ_OK;
}

svq_status sv_set_amplitudes(svq_state st, const void *host) {
    svq_status s = check_state(st);
    if (s) return s;
    if (!host) return fail(SVQ_EINVAL, "host is NULL");
    HIPCHK(st, hipMemcpyAsync(st->buf, host, st->bytes(), hipMemcpyHostToDevice, st->stream), "H2D");
    HIPCHK(st, hipStreamSynchronize(st->stream), "sync");
    for (int q = 0; q < st->n; ++q) st->pos[q] = q;
    return SVQ_OK;
}

svq_status sv_get_amplitudes(svq_state st, void *host) {
    svq_status s = check_state(st);
    if (s) return s;
    if (!host) return fail(SVQ_EINVAL, "host is NULL");
    std::vector<int> ident(st->n);
    for (int q = 0; q < st->n; ++q) ident[q] = q;
    s = relayout(st, st->buf, st->pos, ident);
    if (s) return s;
    HIPCHK(st, hipMemcpyAsync(host, st->buf, st->bytes(), hipMemcpyDeviceToHost, st->stream), "D2H");
    HIPCHK(st, hipStreamSynchronize(st->stream), "sync");
    return SVQ_OK;
}

svq_status sv_device_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst) return fail(SVQ_EINVAL, "null pointer");
    if (bytes % 16) return fail(SVQ_EINVAL, "bytes must be a multiple of 16");
    hipError_t e = launch_copy(src, dst, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return fail(SVQ_EHIP, std::string("copy: ") + hipGetErrorString(e));
    return SVQ_OK;
}

svq_status sv_pass_ceiling(svq_state st, const int32_t *tile_bits, int k, int nphase, int reps,
                           double *ms_out) {
    if (!st) return fail(SVQ_EINVAL, "null handle");
    if (st->poisoned) return fail(SVQ_EPOISONED, "handle poisoned by an earlier failure");
    if (!tile_bits || !ms_out || reps < 1 || reps > 1000) return fail(SVQ_EINVAL, "bad arguments");
    if (k < 10 || k > 13 || k > st->n - st->g) return fail(SVQ_EINVAL, "k must be in [10, 13] and at most n - g");
    std::vector<int> tb(tile_bits, tile_bits + k);
    for (int j = 0; j < k; ++j)
        if (tb[j] >= st->n - st->g) return fail(SVQ_EINVAL, "tile bits must be local positions");
    CircuitPlan P;
    const std::string err = plan_empty_pass(st->n, k, gate_rb(k), tb.data(), nphase, P);
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    HIPCHK(st, hipSetDevice(st->device), "hipSetDevice");
    DevBuf ph;
    HIPCHK(st, ph.ensure(sizeof(PhaseDesc) * P.phases.size()), "alloc phases");
    HIPCHK(st, hipMemcpyAsync(ph.p, P.phases.data(), sizeof(PhaseDesc) * P.phases.size(),
                              hipMemcpyHostToDevice, st->stream),
           "upload phases");
    const PassArgs &a = P.passes[0];
    const OpDesc *no_ops = (const OpDesc *)ph.p;   // never read: every phase has nop = 0
    hipEvent_t e0, e1;
    HIPCHK(st, hipEventCreate(&e0), "event");
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        HIPCHK(st, he, "event");
    }
    he = launch_gate_pass(st->dbl(), k, P.rb, false, st->buf, nullptr, a, (const PhaseDesc *)ph.p, no_ops,
                          nullptr, a.nblocks, st->stream);   // warm
    if (he == hipSuccess) he = hipEventRecord(e0, st->stream);
    for (int r = 0; r < reps && he == hipSuccess; ++r)
        he = launch_gate_pass(st->dbl(), k, P.rb, false, st->buf, nullptr, a, (const PhaseDesc *)ph.p,
                              no_ops, nullptr, a.nblocks, st->stream);
    if (he == hipSuccess) he = hipEventRecord(e1, st->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(st, he, "pass ceiling");
    *ms_out = (double)ms / reps;
    return SVQ_OK;
}

svq_status sv_plan_dump(svq_state st, char *json_buf, size_t cap, size_t *len_out) {
    if (!st) return fail(SVQ_EINVAL, "null handle");
    const std::string empty = "{}";
    const std::string &j = st->last_plan ? *st->last_plan : empty;
    if (len_out) *len_out = j.size() + 1;
    if (!json_buf) return SVQ_OK;
    if (cap < j.size() + 1) return fail(SVQ_ESHAPE, "json_buf smaller than the plan text");
    std::memcpy(json_buf, j.c_str(), j.size() + 1);
    return SVQ_OK;
}

svq_status sv_get_layout(svq_state st, int32_t *pos_out) {
    if (!st) return fail(SVQ_EINVAL, "null handle");
    if (!pos_out) return fail(SVQ_EINVAL, "pos_out is NULL");
    for (int q = 0; q < st->n; ++q) pos_out[q] = st->pos[q];
    return SVQ_OK;
}

svq_status sv_device_ptr(svq_state st, void **ptr_out) {
    if (!st || !ptr_out) return fail(SVQ_EINVAL, "null argument");
    *ptr_out = st->buf;
    return SVQ_OK;
}

svq_status sv_apply_circuit(svq_state st, const svq_gate *gates, int m, const double *theta,
                            int n_theta, svq_sched sched, int tile_k, svq_stats *stats) {
    svq_status s = check_state(st);
    if (s) return s;
    if (m < 0 || (m > 0 && !gates) || n_theta < 0) return fail(SVQ_EINVAL, "bad gate list");
    if (sched != SVQ_EAGER && sched != SVQ_LAZY) return fail(SVQ_EINVAL, "bad schedule");
    if (tile_k != 0 && (tile_k < 8 || tile_k > 13)) return fail(SVQ_EINVAL, "tile_k must be 0 or in [8, 13]");
    std::vector<GateN> gn;
    std::string err = normalize_gates(st->n, gates, m, n_theta, gn);
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    s = check_theta(gn, theta, n_theta);
    if (s) return s;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (m == 0) return SVQ_OK;
    const int k = tile_k ? std::min(tile_k, st->n - st->g) : default_k(st);
    CachedCircuit *cc = nullptr;
    double ms = 0;
    s = get_circuit_plan(st, gn, sched, k, false, &cc, &ms);
    if (s) return s;
    if (stats) stats->ms_plan = ms;
    return run_circuit(st, cc, gn, theta, stats);
}

svq_status sv_apply_circuit_static(svq_state st, const svq_gate *gates, int m, const double *theta,
                                   int n_theta, svq_sched sched, int tile_k, svq_stats *stats) {
    svq_status s = check_state(st);
    if (s) return s;
    if (m < 0 || (m > 0 && !gates) || n_theta < 0) return fail(SVQ_EINVAL, "bad gate list");
    if (sched != SVQ_EAGER && sched != SVQ_LAZY) return fail(SVQ_EINVAL, "bad schedule");
    if (tile_k != 0 && (tile_k < 8 || tile_k > 13)) return fail(SVQ_EINVAL, "tile_k must be 0 or in [8, 13]");
    std::vector<GateN> gn;
    std::string err = normalize_gates(st->n, gates, m, n_theta, gn);
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    s = check_theta(gn, theta, n_theta);
    if (s) return s;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (m == 0) return SVQ_OK;
    const int k = tile_k ? std::min(tile_k, st->n - st->g) : default_k(st);
    const int c = default_c(st);
    const int rb = gate_rb(k, st->dbl(), false);
    // host plan, cached on the handle (host memory only)
    const std::string key = circuit_key(gn, st, sched, k, c, rb, false);
    auto it = st->hcache.find(key);
    HostCircuit *hc = nullptr;
    if (it != st->hcache.end()) {
        hc = it->second.get();
    } else {
        auto t0 = std::chrono::steady_clock::now();
        auto h = std::make_unique<HostCircuit>();
        err = plan_circuit(st->n, st->g, gn, sched, k, rb, c, st->pos, h->plan, relayout_on());
        if (!err.empty()) return fail(SVQ_EINVAL, err);
        h->json = std::make_shared<const std::string>(circuit_json(h->plan, sched, false));
        if (stats)
            stats->ms_plan = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (st->hcache.size() > 64) st->hcache.clear();
        hc = h.get();
        st->hcache[key] = std::move(h);
    }
    const CircuitPlan &P = hc->plan;
    // tables in the static scratch: phases, then ops at a 256-byte boundary
    const size_t ph_bytes = sizeof(PhaseDesc) * P.phases.size();
    const size_t op_off = (ph_bytes + 255) & ~(size_t)255;
    const size_t need = op_off + sizeof(OpDesc) * P.ops.size();
    if (need > kStaticScratchBytes)
        return fail(SVQ_ESHAPE, "circuit tables need " + std::to_string(need) +
                                    " bytes of static scratch; the limit is " +
                                    std::to_string(kStaticScratchBytes));
    void *scr = nullptr;
    s = static_scratch(st, &scr);
    if (s) return s;
    std::vector<OpDesc> ops = P.ops;
    fill_ops(gn, theta, P.op_gate, ops, false);
    char *base = (char *)scr;
    HIPCHK(st, hipMemcpyAsync(base, P.phases.data(), ph_bytes, hipMemcpyHostToDevice, st->stream),
           "upload phases");
    HIPCHK(st, hipMemcpyAsync(base + op_off, ops.data(), sizeof(OpDesc) * ops.size(),
                              hipMemcpyHostToDevice, st->stream),
           "upload ops");
    st->last_plan = hc->json;
    return run_circuit_steps(st, P, (const PhaseDesc *)base, (const OpDesc *)(base + op_off), stats);
}

svq_status sv_qr_permute(svq_state st, const int32_t *new_pos) {
    svq_status s = check_state(st);
    if (s) return s;
    if (!new_pos) return fail(SVQ_EINVAL, "new_pos is NULL");
    std::vector<int> np(st->n);
    std::vector<char> seen(st->n, 0);
    for (int q = 0; q < st->n; ++q) {
        if (new_pos[q] < 0 || new_pos[q] >= st->n || seen[new_pos[q]])
            return fail(SVQ_EINVAL, "new_pos is not a permutation of 0..n-1");
        seen[new_pos[q]] = 1;
        np[q] = new_pos[q];
    }
    return relayout(st, st->buf, st->pos, np);
}

svq_status sv_expectation(svq_state st, const svq_pauli *terms, int n_terms, svq_sched sched,
                          double *energy_host, double *energy_dev, double *chunk_dev,
                          svq_stats *stats) {
    svq_status s = check_state(st);
    if (s) return s;
    if (n_terms < 0 || (n_terms > 0 && !terms)) return fail(SVQ_EINVAL, "bad term list");
    if (sched != SVQ_EAGER && sched != SVQ_LAZY) return fail(SVQ_EINVAL, "bad schedule");
    if (stats) std::memset(stats, 0, sizeof(*stats));
    CachedPaulis *cp = nullptr;
    double ms = 0;
    s = get_pauli_plan(st, terms, n_terms, sched, &cp, &ms);
    if (s) return s;
    if (stats) stats->ms_plan = ms;
    HIPCHK(st, st->d_energy.ensure(sizeof(double)), "alloc energy");
    double *edev = energy_dev ? energy_dev : (double *)st->d_energy.p;
    s = run_expectation(st, cp, edev, chunk_dev, stats);
    if (s) return s;
    if (stats) stats->tile_k = cp->plan.k;
    if (energy_host) {
        HIPCHK(st, hipMemcpyAsync(energy_host, edev, sizeof(double), hipMemcpyDeviceToHost, st->stream), "D2H");
        HIPCHK(st, hipStreamSynchronize(st->stream), "sync");
    }
    return SVQ_OK;
}

svq_status sv_apply_hamiltonian(svq_state st, const svq_pauli *terms, int n_terms, svq_state out) {
    svq_status s = check_state(st);
    if (s) return s;
    if (!out || out->n != st->n || out->g != st->g || out->dtype != st->dtype)
        return fail(SVQ_ESHAPE, "output handle shape differs");
    if (n_terms < 0 || (n_terms > 0 && !terms)) return fail(SVQ_EINVAL, "bad term list");
    CachedPaulis *cp = nullptr;
    double ms = 0;
    s = get_pauli_plan(st, terms, n_terms, SVQ_LAZY, &cp, &ms, true);
    if (s) return s;
    PauliPlan &P = cp->plan;
    // out follows psi's layout; its old content is overwritten
    const int TPBH = hpsi_tpb(P.k);
    int nblocks = 1 << (st->n - P.k);
    (void)TPBH;
    bool any = false;
    for (const Step &stp : P.steps) {
        if (stp.type == 0) {
            s = run_qr(st, st->buf, stp.qr);
            if (s) return s;
            s = run_qr(st, out->buf, stp.qr);
            if (s) return s;
        } else {
            HpsiPassArgs a = P.hpasses[stp.idx];
            a.accumulate = any ? 1 : 0;
            ProfScope ps(st, 3);
            HIPCHK(st, launch_hpsi_pass(st->dbl(), P.k, nblocks, st->buf, out->buf, a,
                                        (const HpsiGroup *)cp->d_hgroups.p,
                                        (const HpsiTerm *)cp->d_hterms.p, st->stream),
                   "hpsi_pass");
            // read psi, write lambda (and read it first after the first pass)
            st->traffic += (any ? 3.0 : 2.0) * (double)st->bytes();
            any = true;
        }
    }
    if (!cp->wide.empty() || !any) {
        HIPCHK(st, launch_hpsi_direct(st->dbl(), st->buf, out->buf, st->N(),
                                      (const WideTerm *)cp->d_wide.p, (int)cp->wide.size(),
                                      any ? 1 : 0, st->stream),
               "hpsi_direct");
        st->traffic += (any ? 3.0 : 2.0) * (double)st->bytes();
    }
    st->pos = P.pos_after;
    out->pos = P.pos_after;
    return SVQ_OK;
}

svq_status sv_grad(svq_state st, const svq_gate *gates, int m, const double *theta, int n_theta,
                   const svq_pauli *terms, int n_terms, svq_sched sched, double *energy_host,
                   double *energy_dev, double *grad_host, double *grad_dev, svq_stats *stats) {
    svq_status s = check_state(st);
    if (s) return s;
    if (m < 0 || (m > 0 && !gates) || n_theta < 0) return fail(SVQ_EINVAL, "bad gate list");
    if (n_terms < 0 || (n_terms > 0 && !terms)) return fail(SVQ_EINVAL, "bad term list");
    if (sched != SVQ_EAGER && sched != SVQ_LAZY) return fail(SVQ_EINVAL, "bad schedule");
    std::vector<GateN> gn;
    std::string err = normalize_gates(st->n, gates, m, n_theta, gn);
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    s = check_theta(gn, theta, n_theta);
    if (s) return s;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    // two tiles must fit in LDS for the reverse sweep
    int k = default_k(st);
    if (st->dbl()) k = std::min(k, 12);
    const std::vector<int> pos0 = st->pos;
    CachedCircuit *cc = nullptr;
    double ms = 0;
    s = get_circuit_plan(st, gn, sched, k, true, &cc, &ms);
    if (s) return s;
    CircuitPlan &P = cc->plan;
    // Every table and scratch buffer is prepared before the first launch, so
    // that a failed allocation (ENOMEM) leaves the handle as it was.
    // Pauli tables for the layout the forward pass ends in:
    {
        const std::vector<int> keep = st->pos;
        st->pos = P.pos_after;
        CachedPaulis *cph = nullptr;
        double msh = 0;
        s = get_pauli_plan(st, terms, n_terms, SVQ_LAZY, &cph, &msh, true);
        st->pos = keep;
        if (s) return s;
    }
    // inverse ops with generators (chain-rule scale folded in)
    std::vector<OpDesc> inv = P.ops;
    fill_ops(gn, theta, P.op_gate, inv, true);
    for (size_t i = 0; i < inv.size(); ++i) {
        const GateN &g = gn[P.op_gate[i]];
        inv[i].gslot = (g.param >= 0 && inv[i].gtype != GEN_NONE) ? P.op_gate[i] : -1;
        if (inv[i].gslot < 0) inv[i].gtype = GEN_NONE;
    }
    // Gates of the parametric ops of every pass, in the order the reverse pass
    // visits them (phases and ops backwards): slot i of a pass's block
    // partials belongs to gate ggates[goff[pass] + i].
    std::vector<int> ggates, goff(P.passes.size() + 1, 0);
    int gmax = 0;
    for (size_t p = 0; p < P.passes.size(); ++p) {
        const PassArgs &pa = P.passes[p];
        for (int sidx = pa.nphase - 1; sidx >= 0; --sidx) {
            const PhaseDesc &ph = P.phases[pa.phase0 + sidx];
            for (int q = ph.nop - 1; q >= 0; --q)
                if (inv[ph.op0 + q].gtype != GEN_NONE) ggates.push_back(P.op_gate[ph.op0 + q]);
        }
        goff[p + 1] = (int)ggates.size();
        gmax = std::max(gmax, goff[p + 1] - goff[p]);
    }
    // gradient reduction: CSR param -> gates
    std::vector<int> pptr(n_theta + 1, 0), pgate;
    for (int i = 0; i < m; ++i)
        if (gn[i].param >= 0 && (gn[i].kind == SVQ_RX || gn[i].kind == SVQ_RY || gn[i].kind == SVQ_RZ ||
                                 gn[i].kind == SVQ_CPHASE || gn[i].kind == SVQ_GIVENS))
            pptr[gn[i].param + 1]++;
    for (int p = 0; p < n_theta; ++p) pptr[p + 1] += pptr[p];
    pgate.resize(pptr[n_theta]);
    {
        std::vector<int> fillp(pptr.begin(), pptr.end() - 1);
        for (int i = 0; i < m; ++i)
            if (gn[i].param >= 0 && (gn[i].kind == SVQ_RX || gn[i].kind == SVQ_RY || gn[i].kind == SVQ_RZ ||
                                     gn[i].kind == SVQ_CPHASE || gn[i].kind == SVQ_GIVENS))
                pgate[fillp[gn[i].param]++] = i;
    }
    const uint32_t nblocks = 1u << (st->n - P.k);
    const int dg = dot_grid(st->N());
    HIPCHK(st, st->d_lam.ensure(st->bytes()), "alloc lambda");
    HIPCHK(st, st->d_extra.ensure(sizeof(double) * dg), "alloc extra");
    HIPCHK(st, st->d_energy.ensure(sizeof(double)), "alloc energy");
    HIPCHK(st, st->d_ops.ensure(sizeof(OpDesc) * std::max<size_t>(1, inv.size())), "alloc ops");
    HIPCHK(st, st->d_gpart.ensure(sizeof(double) * (size_t)std::max(1, gmax) * nblocks), "alloc gpart");
    HIPCHK(st, st->d_gop.ensure(sizeof(double) * (size_t)std::max(1, m)), "alloc gop");
    HIPCHK(st, st->d_ggates.ensure(sizeof(int) * std::max<size_t>(1, ggates.size())), "alloc ggates");
    HIPCHK(st, st->d_pptr.ensure(sizeof(int) * pptr.size()), "alloc pptr");
    HIPCHK(st, st->d_pgate.ensure(sizeof(int) * std::max<size_t>(1, pgate.size())), "alloc pgate");
    HIPCHK(st, st->d_grad.ensure(sizeof(double) * std::max(1, n_theta)), "alloc grad");
    double *edev = energy_dev ? energy_dev : (double *)st->d_energy.p;
    double *gdev = grad_dev ? grad_dev : (double *)st->d_grad.p;
    const double traffic0 = st->traffic;
    // forward
    s = run_circuit(st, cc, gn, theta, stats);
    if (s) return s;
    // lambda = H psi (lambda buffer follows psi's layout)
    svq_state_s lam_view;
    lam_view.n = st->n;
    lam_view.g = st->g;
    lam_view.dtype = st->dtype;
    lam_view.buf = st->d_lam.p;
    lam_view.stream = st->stream;
    lam_view.pos = st->pos;
    lam_view.device = st->device;
    s = sv_apply_hamiltonian(st, terms, n_terms, &lam_view);
    lam_view.buf = nullptr;   // not owned
    if (s) return s;
    // E = Re <psi|lambda>
    HIPCHK(st, launch_dot_re(st->dbl(), st->buf, st->d_lam.p, st->N(), (double *)st->d_extra.p, st->stream), "dot");
    HIPCHK(st, launch_sum((const double *)st->d_extra.p, dg, edev, st->stream), "sum");
    st->traffic += 2.0 * (double)st->bytes();
    // back to the circuit's final layout (both states)
    {
        std::vector<int> lp = st->pos;
        s = relayout(st, st->d_lam.p, lp, P.pos_after);
        if (s) return s;
        s = relayout(st, st->buf, st->pos, P.pos_after);
        if (s) return s;
    }
    // reverse sweep
    HIPCHK(st, hipMemcpyAsync(st->d_ops.p, inv.data(), sizeof(OpDesc) * inv.size(),
                              hipMemcpyHostToDevice, st->stream),
           "upload inverse ops");
    if (!ggates.empty())
        HIPCHK(st, hipMemcpyAsync(st->d_ggates.p, ggates.data(), sizeof(int) * ggates.size(),
                                  hipMemcpyHostToDevice, st->stream),
               "upload ggates");
    for (auto it = P.steps.rbegin(); it != P.steps.rend(); ++it) {
        if (it->type == 0) {
            s = run_qr(st, st->buf, it->qr);
            if (s) return s;
            s = run_qr(st, st->d_lam.p, it->qr);
            if (s) return s;
        } else {
            const PassArgs &a = P.passes[it->idx];
            {
                ProfScope ps(st, 4);
                HIPCHK(st, launch_gate_pass(st->dbl(), P.k, P.rb, true, st->buf, st->d_lam.p, a,
                                            (const PhaseDesc *)cc->d_phases.p,
                                            (const OpDesc *)st->d_ops.p, (double *)st->d_gpart.p,
                                            (int)nblocks, st->stream),
                       "adjoint_pass");
            }
            st->traffic += 4.0 * (double)st->bytes();   // psi and lambda, read and written
            const int g0 = goff[it->idx], gn_pass = goff[it->idx + 1] - g0;
            HIPCHK(st, launch_grad_tiles((const double *)st->d_gpart.p, nblocks, gn_pass,
                                         (const int *)st->d_ggates.p + g0, (double *)st->d_gop.p,
                                         st->stream),
                   "grad_tiles");
        }
    }
    st->pos = pos0;
    HIPCHK(st, hipMemcpyAsync(st->d_pptr.p, pptr.data(), sizeof(int) * pptr.size(), hipMemcpyHostToDevice, st->stream), "upload pptr");
    if (!pgate.empty())
        HIPCHK(st, hipMemcpyAsync(st->d_pgate.p, pgate.data(), sizeof(int) * pgate.size(), hipMemcpyHostToDevice, st->stream), "upload pgate");
    HIPCHK(st, launch_grad_reduce((const double *)st->d_gop.p, 1, (const int *)st->d_pptr.p,
                                  (const int *)st->d_pgate.p, n_theta, gdev, st->stream),
           "grad_reduce");
    if (stats) {
        // every launch of the call: forward, H|psi>, <psi|lambda>, the
        // relayouts and the reverse sweep (the QRs of both states)
        stats->n_gate_passes += (int)P.passes.size();
        stats->bytes = st->traffic - traffic0;
        stats->ms_plan += ms;
    }
    if (energy_host)
        HIPCHK(st, hipMemcpyAsync(energy_host, edev, sizeof(double), hipMemcpyDeviceToHost, st->stream), "D2H");
    if (grad_host && n_theta)
        HIPCHK(st, hipMemcpyAsync(grad_host, gdev, sizeof(double) * n_theta, hipMemcpyDeviceToHost, st->stream), "D2H");
    // pptr/pgate/ggates host vectors must outlive the async copies
    HIPCHK(st, hipStreamSynchronize(st->stream), "sync");
    return SVQ_OK;
}

svq_status sv_param_shift_grad(svq_state st, const svq_gate *gates, int m, const double *theta,
                               int n_theta, const svq_pauli *terms, int n_terms, svq_sched sched,
                               int rule, double *energy_host, double *grad_host, double *grad_dev,
                               int *n_evals_out, svq_stats *stats) {
    svq_status s = check_state(st);
    if (s) return s;
    if (m < 0 || (m > 0 && !gates) || n_theta < 0) return fail(SVQ_EINVAL, "bad gate list");
    if (n_terms < 0 || (n_terms > 0 && !terms)) return fail(SVQ_EINVAL, "bad term list");
    if (sched != SVQ_EAGER && sched != SVQ_LAZY) return fail(SVQ_EINVAL, "bad schedule");
    if (rule != SVQ_SHIFT_EXACT && rule != SVQ_SHIFT_TWO_TERM) return fail(SVQ_EINVAL, "bad rule");
    std::vector<GateN> gn;
    std::string err = normalize_gates(st->n, gates, m, n_theta, gn);
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    s = check_theta(gn, theta, n_theta);
    if (s) return s;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    // Shifted evaluations: (gate, angle shift, coefficient), grouped by
    // parameter.  One-frequency generators (RX, RY, RZ: spectrum +-1/2;
    // CPHASE: {0, -1}) take f' = [f(a + pi/2) - f(a - pi/2)] / 2.  GIVENS has
    // the spectrum {+-1/2, 0, 0}, i.e. the frequencies 1/2 and 1; its exact
    // rule is the two-frequency equidistant rule with shifts pi/2 and 3pi/2
    // (Wierichs et al., Quantum 6, 677 (2022)).  The two-term rule applies the
    // one-frequency rule to every gate (exact only for one frequency).
    struct Eval { int gate, param; double shift, coef; };
    std::vector<std::vector<Eval>> byp(n_theta);
    const double r2 = std::sqrt(2.0), pi = 3.14159265358979323846;
    const double ga = (r2 + 1.0) / (4.0 * r2), gb = (r2 - 1.0) / (4.0 * r2);
    for (int j = 0; j < m; ++j) {
        const GateN &g = gn[j];
        if (g.param < 0) continue;
        std::vector<std::pair<double, double>> rl;
        if (g.kind == SVQ_GIVENS && rule == SVQ_SHIFT_EXACT)
            rl = {{pi / 2, ga}, {3 * pi / 2, -gb}};
        else
            rl = {{pi / 2, 0.5}};
        for (const auto &r : rl) {
            byp[g.param].push_back({j, g.param, +r.first, +r.second * g.scale});
            byp[g.param].push_back({j, g.param, -r.first, -r.second * g.scale});
        }
    }
    std::vector<Eval> ev;
    std::vector<int> ptr(n_theta + 1, 0);
    std::vector<double> coef;
    for (int p = 0; p < n_theta; ++p) {
        for (const Eval &e : byp[p]) {
            ev.push_back(e);
            coef.push_back(e.coef);
        }
        ptr[p + 1] = (int)ev.size();
    }
    const int ne = (int)ev.size();
    if (n_evals_out) *n_evals_out = ne + (energy_host ? 1 : 0);
    // plans and scratch before the first launch
    const int k = default_k(st);
    const std::vector<int> pos0 = st->pos;
    CachedCircuit *cc = nullptr;
    double ms = 0;
    s = get_circuit_plan(st, gn, sched, k, false, &cc, &ms);
    if (s) return s;
    CachedPaulis *cp = nullptr;
    {
        const std::vector<int> keep = st->pos;
        st->pos = cc->plan.pos_after;
        double msp = 0;
        s = get_pauli_plan(st, terms, n_terms, sched, &cp, &msp);
        st->pos = keep;
        if (s) return s;
    }
    HIPCHK(st, st->d_lam.ensure(st->bytes()), "alloc psi0 copy");
    HIPCHK(st, st->d_gop.ensure(sizeof(double) * (size_t)std::max(1, ne + 1)), "alloc energies");
    HIPCHK(st, st->d_gpart.ensure(sizeof(double) * (size_t)std::max(1, ne)), "alloc coefficients");
    HIPCHK(st, st->d_pptr.ensure(sizeof(int) * ptr.size()), "alloc ptr");
    HIPCHK(st, st->d_grad.ensure(sizeof(double) * std::max(1, n_theta)), "alloc grad");
    HIPCHK(st, st->d_ops.ensure(sizeof(OpDesc) * std::max<size_t>(1, cc->plan.ops.size())), "alloc ops");
    {
        const int nchunk = 1 << st->g;
        HIPCHK(st, st->d_partials.ensure(sizeof(double) * std::max(1, cp->plan.total_blocks)), "alloc partials");
        HIPCHK(st, st->d_chunks.ensure(sizeof(double) * (nchunk + reduce_scratch(nchunk))), "alloc chunks");
        HIPCHK(st, st->d_extra.ensure(sizeof(double) * direct_grid(st->N())), "alloc extra");
    }
    double *evals = (double *)st->d_gop.p;
    double *gdev = grad_dev ? grad_dev : (double *)st->d_grad.p;
    const double traffic0 = st->traffic;
    // psi0 is kept aside and restored before every evaluation
    HIPCHK(st, hipMemcpyAsync(st->d_lam.p, st->buf, st->bytes(), hipMemcpyDeviceToDevice, st->stream),
           "save psi0");
    st->traffic += 2.0 * (double)st->bytes();
    std::vector<GateN> gs = gn;
    svq_stats one;
    for (int e = 0; e <= ne; ++e) {
        if (e == ne && !energy_host) break;
        if (e > 0) {
            HIPCHK(st, hipMemcpyAsync(st->buf, st->d_lam.p, st->bytes(), hipMemcpyDeviceToDevice,
                                      st->stream),
                   "restore psi0");
            st->traffic += 2.0 * (double)st->bytes();
            st->pos = pos0;
        }
        // angle shift of one gate (the plan does not depend on angles)
        if (e < ne) gs[ev[e].gate].offset = gn[ev[e].gate].offset + ev[e].shift;
        std::memset(&one, 0, sizeof(one));
        s = run_circuit(st, cc, gs, theta, &one);
        if (s) return s;
        if (e < ne) gs[ev[e].gate].offset = gn[ev[e].gate].offset;
        s = run_expectation(st, cp, evals + e, nullptr, &one);
        if (s) return s;
        st->traffic += (double)one.n_evc_passes * (double)st->bytes();
        if (stats) {
            stats->n_qr += one.n_qr;
            stats->n_gate_passes += one.n_gate_passes;
            stats->n_evc_passes += one.n_evc_passes;
        }
    }
    HIPCHK(st, hipMemcpyAsync(st->d_gpart.p, coef.data(), sizeof(double) * std::max(1, ne),
                              hipMemcpyHostToDevice, st->stream),
           "upload coefficients");
    HIPCHK(st, hipMemcpyAsync(st->d_pptr.p, ptr.data(), sizeof(int) * ptr.size(),
                              hipMemcpyHostToDevice, st->stream),
           "upload ptr");
    HIPCHK(st, launch_shift_combine(evals, (const double *)st->d_gpart.p, (const int *)st->d_pptr.p,
                                    n_theta, gdev, st->stream),
           "shift_combine");
    // hand psi0 back, as sv_grad does
    HIPCHK(st, hipMemcpyAsync(st->buf, st->d_lam.p, st->bytes(), hipMemcpyDeviceToDevice, st->stream),
           "restore psi0");
    st->traffic += 2.0 * (double)st->bytes();
    st->pos = pos0;
    if (stats) {
        stats->bytes = st->traffic - traffic0;
        stats->ms_plan = ms;
        stats->tile_k = cc->plan.k;
    }
    if (energy_host)
        HIPCHK(st, hipMemcpyAsync(energy_host, evals + ne, sizeof(double), hipMemcpyDeviceToHost, st->stream), "D2H");
    if (grad_host && n_theta)
        HIPCHK(st, hipMemcpyAsync(grad_host, gdev, sizeof(double) * n_theta, hipMemcpyDeviceToHost, st->stream), "D2H");
    HIPCHK(st, hipStreamSynchronize(st->stream), "sync");
    return SVQ_OK;
}

static svq_status plan_common_circuit(int n, int g, const svq_gate *gates, int m, svq_sched sched,
                                      int tile_k, CircuitPlan &P) {
    if (n < 1 || n > 34 || g < 0 || g >= n || n - g < 8) return fail(SVQ_EINVAL, "bad n/g");
    std::vector<GateN> gn;
    std::string err = normalize_gates(n, gates, m, 1 << 30, gn);
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    std::vector<int> pos(n);
    for (int q = 0; q < n; ++q) pos[q] = q;
    int k = tile_k ? tile_k : 12;
    k = std::max(8, std::min(13, std::min(k, n - g)));
    err = plan_circuit(n, g, gn, sched, k, gate_rb(k), env_int("SVQ_LOW_BITS", 4), pos, P,
                       relayout_on());
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    return SVQ_OK;
}

svq_status sv_plan_circuit_json(int n, int g, const svq_gate *gates, int m, svq_sched sched,
                                int tile_k, char *json_buf, size_t cap, size_t *len_out) {
    CircuitPlan P;
    svq_status s = plan_common_circuit(n, g, gates, m, sched, tile_k, P);
    if (s) return s;
    const std::string j = circuit_json(P, sched, false);
    if (len_out) *len_out = j.size() + 1;
    if (!json_buf) return SVQ_OK;
    if (cap < j.size() + 1) return fail(SVQ_ESHAPE, "json_buf smaller than the plan text");
    std::memcpy(json_buf, j.c_str(), j.size() + 1);
    return SVQ_OK;
}

svq_status sv_plan_circuit(int n, int g, const svq_gate *gates, int m, svq_sched sched, int tile_k,
                           int32_t *order_out, int32_t *qr_tile_out, int32_t *pass_out,
                           uint64_t *local_out, int32_t *n_qr_out, int32_t *n_pass_out) {
    CircuitPlan P;
    svq_status s = plan_common_circuit(n, g, gates, m, sched, tile_k, P);
    if (s) return s;
    for (size_t i = 0; i < P.order.size(); ++i) {
        if (order_out) order_out[i] = P.order[i];
        if (qr_tile_out) qr_tile_out[i] = P.pos_qrtile[i];
        if (pass_out) pass_out[i] = P.pos_pass[i];
        if (local_out) local_out[i] = P.pos_local[i];
    }
    if (n_qr_out) *n_qr_out = P.n_qr;
    if (n_pass_out) *n_pass_out = (int)P.passes.size();
    return SVQ_OK;
}

// Level-1 tiles of sv_plan_ops / sv_qr_cost (arguments already checked).
static std::vector<L1Tile> plan_level1(int n, int n_local, const std::vector<uint64_t> &t, int method,
                                       int n_intra, int fill_highest, std::vector<int> &kinds,
                                       std::vector<uint64_t> &intra) {
    const int m = (int)t.size();
    std::vector<int> pos(n);
    for (int q = 0; q < n; ++q) pos[q] = q;
    if (method == 0) return ad_hoc(n, n_local, t, depth_order(t), pos);
    if (method == 1) return flat_tiling(n, n_local, t, pos);
    if (method == 3) {
        std::vector<int> ord(m);
        for (int i = 0; i < m; ++i) ord[i] = i;
        return ad_hoc(n, n_local, t, ord, pos);
    }
    return hierarchical_tiling(n, n_local, n_intra, t, fill_highest != 0, kinds, intra);
}

static svq_status check_ops(int n, int n_local, const uint64_t *targets, int m, int method, int n_intra,
                            std::vector<uint64_t> &t) {
    if (n < 1 || n > 64 || n_local < 1 || n_local > n || m < 0 || (m > 0 && !targets))
        return fail(SVQ_EINVAL, "bad arguments");
    if (method < 0 || method > 3) return fail(SVQ_EINVAL, "method must be 0, 1, 2 or 3");
    if (n_intra < 0 || n_local + n_intra > n) return fail(SVQ_EINVAL, "bad n_intra");
    const uint64_t full = n >= 64 ? ~0ULL : ((1ULL << n) - 1);
    t.assign(targets, targets + m);
    for (uint64_t v : t)
        if ((v & ~full) || __builtin_popcountll(v) > n_local)
            return fail(SVQ_EINVAL, "operator target set out of range or wider than the local set");
    return SVQ_OK;
}

svq_status sv_plan_ops(int n, int n_local, const uint64_t *targets, int m, int method,
                       int n_intra, int fill_highest, int32_t *order_out, uint64_t *local_out,
                       uint64_t *intra_out, int32_t *n_qr_out, int32_t *n_inter_out) {
    std::vector<uint64_t> t;
    if (method != 2) n_intra = 0;
    const svq_status rc = check_ops(n, n_local, targets, m, method, n_intra, t);
    if (rc != SVQ_OK) return rc;
    std::vector<int> kinds;
    std::vector<uint64_t> intra;
    const std::vector<L1Tile> tiles = plan_level1(n, n_local, t, method, n_intra, fill_highest, kinds, intra);
    int x = 0, nqr = 0, ninter = 0;
    uint64_t prev = (1ULL << n_local) - 1;
    for (size_t ti = 0; ti < tiles.size(); ++ti) {
        if (tiles[ti].local != prev) ++nqr;
        if (method == 2 && kinds[ti]) ++ninter;
        prev = tiles[ti].local;
        for (int op : tiles[ti].ops) {
            if (order_out) order_out[x] = op;
            if (local_out) local_out[x] = tiles[ti].local;
            if (intra_out) intra_out[x] = method == 2 ? intra[ti] : 0;
            ++x;
        }
    }
    if (n_qr_out) *n_qr_out = nqr;
    if (n_inter_out) *n_inter_out = ninter;
    return SVQ_OK;
}

svq_status sv_qr_cost(int n, int n_local, int n_intra, const uint64_t *targets, int m, int method,
                      int fill_highest, double w_intra, double w_inter, int32_t *n_intra_out,
                      int32_t *n_inter_out, double *cost_out) {
    std::vector<uint64_t> t;
    const svq_status rc = check_ops(n, n_local, targets, m, method, n_intra, t);
    if (rc != SVQ_OK) return rc;
    if (!std::isfinite(w_intra) || !std::isfinite(w_inter) || w_intra < 0 || w_inter < 0)
        return fail(SVQ_EINVAL, "weights must be finite and non-negative");
    std::vector<int> kinds;
    std::vector<uint64_t> intra;
    const std::vector<L1Tile> tiles = plan_level1(n, n_local, t, method, n_intra, fill_highest, kinds, intra);
    // Positions n_local .. n_local + n_intra - 1 are the intra-node PE bits,
    // those above the inter-node ones.  A flat or ad hoc reorder swaps its
    // incoming qubits with its outgoing ones pairwise in ascending order of
    // position (the ad hoc method's own pairing); it is an inter reorder when
    // an incoming qubit leaves an inter position.  The
    // hierarchical tiling tracks Q_intra itself: its reorder is inter when the
    // set of inter qubits changes.
    std::vector<int> pos(n);
    for (int q = 0; q < n; ++q) pos[q] = q;
    uint64_t prev = (1ULL << n_local) - 1;
    uint64_t prev_intra = ((1ULL << n_intra) - 1) << n_local;
    int ni = 0, ne = 0;
    for (size_t ti = 0; ti < tiles.size(); ++ti) {
        const uint64_t cur = tiles[ti].local;
        bool inter = false;
        if (method == 2) {
            if (cur == prev && intra[ti] == prev_intra) continue;
            inter = kinds[ti] != 0;
            prev_intra = intra[ti];
        } else {
            if (cur == prev) continue;
            std::vector<int> in, out, vac;
            for (int q = 0; q < n; ++q) {
                if (((cur >> q) & 1) && !((prev >> q) & 1)) in.push_back(q);
                if (((prev >> q) & 1) && !((cur >> q) & 1)) out.push_back(q);
            }
            auto by_pos = [&](int a, int b) { return pos[a] < pos[b]; };
            std::sort(in.begin(), in.end(), by_pos);
            std::sort(out.begin(), out.end(), by_pos);
            std::vector<int> loc;
            for (int q : in) vac.push_back(pos[q]);
            for (int q : out) loc.push_back(pos[q]);
            for (int p : vac) inter |= p >= n_local + n_intra;
            for (size_t i = 0; i < out.size(); ++i) pos[out[i]] = vac[i];
            for (size_t i = 0; i < in.size(); ++i) pos[in[i]] = loc[i];
        }
        ++(inter ? ne : ni);
        prev = cur;
    }
    if (n_intra_out) *n_intra_out = ni;
    if (n_inter_out) *n_inter_out = ne;
    if (cost_out) *cost_out = w_intra * ni + w_inter * ne;
    return SVQ_OK;
}

svq_status sv_plan_paulis(int n, int g, const svq_pauli *terms, int n_terms, svq_sched sched,
                          int tile_k, int32_t *order_out, int32_t *qr_tile_out, int32_t *pass_out,
                          uint64_t *local_out, int32_t *n_qr_out, int32_t *n_pass_out) {
    if (n < 1 || n > 34 || g < 0 || g >= n || n - g < 8) return fail(SVQ_EINVAL, "bad n/g");
    std::vector<int> pos(n);
    for (int q = 0; q < n; ++q) pos[q] = q;
    int k = tile_k ? tile_k : env_int("SVQ_EVC_K", 14);
    k = std::max(8, std::min(14, std::min(k, n - g)));
    PauliPlan P;
    std::string err = plan_paulis(n, g, terms, n_terms, sched, k, env_int("SVQ_EVC_LOW_BITS", 4), false, pos, P);
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    for (size_t i = 0; i < P.order.size(); ++i) {
        if (order_out) order_out[i] = P.order[i];
        if (qr_tile_out) qr_tile_out[i] = P.pos_qrtile[i];
        if (pass_out) pass_out[i] = P.pos_pass[i];
        if (local_out) local_out[i] = P.pos_local[i];
    }
    if (n_qr_out) *n_qr_out = P.n_qr;
    if (n_pass_out) *n_pass_out = (int)P.passes.size();
    return SVQ_OK;
}

}  // extern "C"

// ===========================================================================
// batched VQE
// ===========================================================================

struct svq_batch_s {
    int n_inst = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    bool poisoned = false;
    std::vector<std::vector<GateN>> gates;
    std::vector<int> ntheta;
    std::vector<int> theta_off;            // offset of each instance in the grads output
    std::vector<OpDesc> ops_fwd, ops_inv;  // filled per run
    // instances held in LDS: ops in gate order (template), their instance
    std::vector<OpDesc> lops;
    std::vector<int> lop_inst;
    std::vector<BatchLdsInst> linsts;
    int lds_max_n = 0;
    std::vector<int> op_gate, op_inst;     // gate index / instance of every op
    std::vector<BatchInst> insts;
    int nitems = 0, nstages = 0, total_theta = 0;
    double bytes_per_run = 0;              // algorithmic HBM bytes of one run
    bool persistent = false;               // one persistent launch, else level-synchronous
    // level-synchronous launches: type, item0, count, size class (1: the
    // instances whose gate passes use 2^12 tiles)
    std::vector<std::array<int, 4>> groups;
    DevBuf arena, items, stages, dinsts, passes, hpasses, phases, d_ops_fwd, d_ops_inv, hgroups,
        hterms, pptr, pgate, epart, gpart, energies, grads, counters, t_done, t_start;
    OpDesc *h_ops_fwd = nullptr, *h_ops_inv = nullptr;   // pinned staging
    OpDesc *h_lops_fwd = nullptr, *h_lops_inv = nullptr;
    DevBuf d_linst, d_lterms, d_gvals, d_lops_fwd, d_lops_inv;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    BatchArgs args;
    ~svq_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (h_ops_fwd) (void)hipHostFree(h_ops_fwd);
        if (h_ops_inv) (void)hipHostFree(h_ops_inv);
        if (h_lops_fwd) (void)hipHostFree(h_lops_fwd);
        if (h_lops_inv) (void)hipHostFree(h_lops_inv);
    }
};

namespace {

svq_status batch_hip_fail(svq_batch b, hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory) return fail(SVQ_ENOMEM, std::string(what) + ": out of device memory");
    if (b) b->poisoned = true;
    return fail(SVQ_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define BHIPCHK(b, expr, what)                                  \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return batch_hip_fail(b, _e, what); \
    } while (0)

template <typename T>
hipError_t upload(DevBuf &d, const std::vector<T> &h, hipStream_t s) {
    hipError_t e = d.ensure(std::max<size_t>(sizeof(T) * h.size(), 64));
    if (e != hipSuccess || h.empty()) return e;
    return hipMemcpyAsync(d.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s);
}

}  // namespace

extern "C" {

svq_status sv_batch_create(int n_inst, const int32_t *n_qubits, const svq_gate *const *gates,
                           const int32_t *m, const int32_t *n_theta,
                           const svq_pauli *const *terms, const int32_t *n_terms,
                           const uint64_t *psi0, int low_bits, void *stream, svq_batch *out) {
    if (!out) return fail(SVQ_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_inst <= 0 || !n_qubits || !gates || !m || !n_theta || !terms || !n_terms || !psi0)
        return fail(SVQ_EINVAL, "bad batch arguments");
    const int K = kBatchK;
    TuneVal tv{64, 4, 0.0};
    (void)tuned(2, 0, 0, 0, tv);
    const int c = low_bits ? low_bits : env_int("SVQ_BATCH_LOW_BITS", tv.c);
    if (c < 1 || c > 8) return fail(SVQ_EINVAL, "low_bits must be in [1, 8]");
    // items per stage of an instance (each a contiguous tile range)
    const int chunks = std::max(1, env_int("SVQ_BATCH_CHUNKS", tv.k));
    auto b = std::make_unique<svq_batch_s>();
    b->n_inst = n_inst;
    b->stream = (hipStream_t)stream;
    hipError_t he = hipGetDevice(&b->device);
    if (he != hipSuccess) return fail(SVQ_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
    std::vector<BatchStage> stages;
    std::vector<BatchPass> passes;
    std::vector<BatchHPass> hpasses;
    std::vector<PhaseDesc> phases;
    std::vector<HpsiGroup> hgroups;
    std::vector<HpsiTerm> hterms;
    std::vector<int32_t> pptr, pgate;
    int64_t arena_elems = 0;
    int epart_total = 0, gpart_total = 0;
    std::vector<int> inst_stage_count(n_inst);
    std::vector<int> inst_wide(n_inst, 0);
    b->persistent = env_int("SVQ_BATCH_PERSISTENT", 0) != 0;
    // Large instances run their gate passes on 2^12-amplitude tiles with
    // 4-wave blocks (fewer passes, the single-state pass's layout); the
    // persistent form keeps every stage on 2^10 tiles.
    TuneVal tw{kBatchWideN, 0, 0.0};
    (void)tuned(3, 0, 0, 0, tw);
    const int wide_n = env_int("SVQ_BATCH_WIDE_N", tw.k);
    // Small instances keep psi and lambda in one workgroup's LDS for the whole
    // evaluation (level-synchronous form only).
    const int lds_n = b->persistent ? 0 : std::min(kBatchLdsN, env_int("SVQ_BATCH_LDS_N", kBatchLdsN));
    std::vector<WideTerm> lterms;
    int gv_total = 0;
    // CSR parameter -> gates (gate indices local to the instance)
    auto add_csr = [&](int i, const std::vector<GateN> &gn) {
        const int off = (int)pptr.size();
        std::vector<std::vector<int>> byp(n_theta[i]);
        for (int gi = 0; gi < m[i]; ++gi)
            if (gn[gi].param >= 0 && (gn[gi].kind == SVQ_RX || gn[gi].kind == SVQ_RY || gn[gi].kind == SVQ_RZ ||
                                      gn[gi].kind == SVQ_CPHASE || gn[gi].kind == SVQ_GIVENS))
                byp[gn[gi].param].push_back(gi);
        pptr.push_back((int)pgate.size());
        for (int p = 0; p < n_theta[i]; ++p) {
            for (int gi : byp[p]) pgate.push_back(gi);
            pptr.push_back((int)pgate.size());
        }
        return off;
    };
    for (int i = 0; i < n_inst; ++i) {
        const int n = n_qubits[i];
        const bool wide = !b->persistent && n >= wide_n && n >= kBatchKWide;
        const int KG = wide ? kBatchKWide : K;
        inst_wide[i] = wide;
        if (n < K || n > 26) return fail(SVQ_EINVAL, "batch instances need 10 <= n <= 26");
        if (m[i] < 0 || n_theta[i] < 0 || n_terms[i] < 1) return fail(SVQ_EINVAL, "bad instance sizes");
        if (psi0[i] >> n) return fail(SVQ_EINVAL, "psi0 index >= 2^n");
        std::vector<GateN> gn;
        std::string err = normalize_gates(n, gates[i], m[i], n_theta[i], gn);
        if (!err.empty()) return fail(SVQ_EINVAL, "instance " + std::to_string(i) + ": " + err);
        if (n <= lds_n) {
            for (int t = 0; t < n_terms[i]; ++t) {
                const svq_pauli &tp = terms[i][t];
                if (((tp.x | tp.z) >> n) || !std::isfinite(tp.coef))
                    return fail(SVQ_EINVAL, "instance " + std::to_string(i) + ": bad Pauli term");
            }
            BatchLdsInst L;
            std::memset(&L, 0, sizeof(L));
            L.n = n;
            L.m = m[i];
            L.op0 = (int)b->lops.size();
            L.t0 = (int)lterms.size();
            L.nt = n_terms[i];
            L.ntheta = n_theta[i];
            L.grad_off = b->total_theta;
            L.gv_off = gv_total;
            L.inst = i;
            L.psi0_lo = (uint32_t)psi0[i];
            L.psi0_hi = (uint32_t)(psi0[i] >> 32);
            gv_total += std::max(1, m[i]);
            for (int gi = 0; gi < m[i]; ++gi) {
                OpDesc o;
                std::memset(&o, 0, sizeof(o));
                o.type = op_type_for_kind(gn[gi].kind);
                o.b0 = 0;
                o.b1 = gn[gi].nq > 1 ? 1 : 0;
                o.spare = gn[gi].q[0];
                o.pad = gn[gi].nq > 1 ? gn[gi].q[1] : -1;
                o.gslot = -1;
                b->lops.push_back(o);
                b->lop_inst.push_back(i);
            }
            for (int t = 0; t < n_terms[i]; ++t) {
                WideTerm w;
                std::memset(&w, 0, sizeof(w));
                w.x = terms[i][t].x;
                w.z = terms[i][t].z;
                w.coef = terms[i][t].coef;
                w.ny = __builtin_popcountll(terms[i][t].x & terms[i][t].z);
                lterms.push_back(w);
            }
            L.pptr_off = add_csr(i, gn);
            BatchInst I;
            std::memset(&I, 0, sizeof(I));
            I.n = n;
            I.stage0 = (int)stages.size();
            I.nstages = 0;
            I.m = m[i];
            I.ntheta = n_theta[i];
            I.grad_off = b->total_theta;
            inst_stage_count[i] = 0;
            b->theta_off.push_back(b->total_theta);
            b->total_theta += n_theta[i];
            b->linsts.push_back(L);
            b->lds_max_n = std::max(b->lds_max_n, n);
            b->gates.push_back(std::move(gn));
            b->ntheta.push_back(n_theta[i]);
            b->insts.push_back(I);
            continue;
        }
        std::vector<int> pos(n);
        for (int q = 0; q < n; ++q) pos[q] = q;
        CircuitPlan cp;
        err = plan_circuit(n, 0, gn, SVQ_LAZY, KG, gate_rb(KG), c, pos, cp, false);
        if (!err.empty()) return fail(SVQ_EINVAL, err);
        PauliPlan pp;
        err = plan_paulis(n, 0, terms[i], n_terms[i], SVQ_LAZY, KG, c, false, pos, pp);
        if (!err.empty()) return fail(SVQ_EINVAL, err);
        if (cp.n_qr || pp.n_qr || !pp.wide_groups.empty() || cp.k != KG || pp.k != KG)
            return fail(SVQ_EUNSUP, "instance " + std::to_string(i) + " needs a reorder or a wide term");
        BatchInst I;
        std::memset(&I, 0, sizeof(I));
        I.n = n;
        I.ntiles = 1 << (n - K);
        // every stage type splits into the same nchunks items (the gradient
        // and energy partial slots are per chunk)
        I.nchunks = std::min(1 << (n - KG), chunks);
        I.psi_off = arena_elems;
        I.lam_off = arena_elems + (1LL << n);
        arena_elems += 2LL << n;
        I.psi0_lo = (uint32_t)psi0[i];
        I.psi0_hi = (uint32_t)(psi0[i] >> 32);
        I.epart_off = epart_total;
        epart_total += I.nchunks;
        I.m = m[i];
        I.ntheta = n_theta[i];
        I.gpart_off = gpart_total;
        gpart_total += std::max(1, m[i]) * I.nchunks;
        I.grad_off = b->total_theta;
        b->theta_off.push_back(b->total_theta);
        b->total_theta += n_theta[i];
        // ops (fwd and inverse share layout), phases with global op offsets
        const int op_base = (int)b->op_gate.size();
        const int ph_base = (int)phases.size();
        for (size_t o = 0; o < cp.ops.size(); ++o) {
            b->ops_fwd.push_back(cp.ops[o]);
            b->op_gate.push_back(cp.op_gate[o]);
            b->op_inst.push_back(i);
        }
        for (PhaseDesc ph : cp.phases) {
            ph.op0 += op_base;
            phases.push_back(ph);
        }
        const int pass_base = (int)passes.size();
        for (const PassArgs &pa : cp.passes) {
            BatchPass bp;
            std::memset(&bp, 0, sizeof(bp));
            for (int j = 0; j < 16; ++j) {
                bp.tphys[j] = pa.tphys[j];
                bp.swz[j] = pa.swz[j];
            }
            bp.phase0 = pa.phase0 + ph_base;
            bp.nphase = pa.nphase;
            passes.push_back(bp);
        }
        const int hg_base = (int)hgroups.size(), ht_base = (int)hterms.size();
        for (HpsiGroup hg : pp.hgroups) {
            hg.t0 += ht_base;
            hgroups.push_back(hg);
        }
        for (const HpsiTerm &ht : pp.hterms) hterms.push_back(ht);
        const int hp_base = (int)hpasses.size();
        for (const HpsiPassArgs &ha : pp.hpasses) {
            BatchHPass bh;
            std::memset(&bh, 0, sizeof(bh));
            for (int j = 0; j < 16; ++j) bh.tphys[j] = ha.tphys[j];
            bh.group0 = ha.group0 + hg_base;
            bh.ngroups = ha.ngroups;
            hpasses.push_back(bh);
        }
        // stages
        I.stage0 = (int)stages.size();
        auto add = [&](int type, int ntiles, int desc, int acc) {
            BatchStage st;
            st.type = type;
            st.ntiles = ntiles;
            st.desc = desc;
            st.accumulate = acc;
            stages.push_back(st);
        };
        add(IT_INIT, I.ntiles, 0, 0);
        const int gtiles = 1 << (n - KG);
        for (size_t p = 0; p < cp.passes.size(); ++p) add(wide ? IT_FWD_W : IT_FWD, gtiles, pass_base + (int)p, 0);
        for (size_t h = 0; h < pp.hpasses.size(); ++h)
            add(wide ? IT_HPSI_W : IT_HPSI, gtiles, hp_base + (int)h, h > 0);
        add(IT_DOT, I.ntiles, 0, 0);
        for (size_t p = cp.passes.size(); p-- > 0;) add(wide ? IT_ADJ_W : IT_ADJ, gtiles, pass_base + (int)p, 0);
        add(IT_FINAL, n_theta[i] + 1, 0, 0);   // one slot per parameter, one for E
        I.nstages = (int)stages.size() - I.stage0;
        {
            // one write of psi (init); a gate pass reads and writes psi, its
            // reverse psi and lambda; an H pass reads psi and writes lambda
            // (and reads it when accumulating); the dot reads both
            const double S = 8.0 * (double)(1LL << n);
            const double hp = (double)pp.hpasses.size();
            b->bytes_per_run += S * (1.0 + 2.0 * cp.passes.size() + 2.0 * hp + std::max(0.0, hp - 1.0) + 2.0 +
                                     4.0 * cp.passes.size());
        }
        inst_stage_count[i] = I.nstages;
        I.pptr_off = add_csr(i, gn);
        b->gates.push_back(std::move(gn));
        b->ntheta.push_back(n_theta[i]);
        b->insts.push_back(I);
    }
    b->nstages = (int)stages.size();
    // items, stage-major
    std::vector<BatchItem> items;
    int maxst = 0;
    for (int i = 0; i < n_inst; ++i) maxst = std::max(maxst, inst_stage_count[i]);
    // Items are level-major (all first stages, then all second stages, ...),
    // and inside a level grouped by type: the persistent kernel needs every
    // item's predecessor earlier in the queue, the level-synchronous launches
    // one contiguous range per (level, type).
    for (int sidx = 0; sidx < maxst; ++sidx)
      for (int type = IT_INIT; type <= IT_HPSI_W; ++type)
       for (int cls = 0; cls < 2; ++cls) {
        const int item0 = (int)items.size();
        for (int i = 0; i < n_inst; ++i) {
            if (sidx >= inst_stage_count[i] || inst_wide[i] != cls) continue;
            const BatchStage &st = stages[b->insts[i].stage0 + sidx];
            if (st.type != type) continue;
            const int nch = st.type == IT_FINAL ? std::min(st.ntiles, 32) : b->insts[i].nchunks;
            for (int ch = 0; ch < nch; ++ch) {
                const int t0 = (int)((int64_t)st.ntiles * ch / nch);
                const int t1 = (int)((int64_t)st.ntiles * (ch + 1) / nch);
                BatchItem it;
                std::memset(&it, 0, sizeof(it));
                it.inst = i;
                it.stage = sidx;
                it.tile0 = t0;
                it.ntile = t1 - t0;
                it.chunk = ch;
                items.push_back(it);
            }
        }
        if ((int)items.size() > item0) b->groups.push_back({type, item0, (int)items.size() - item0, cls});
       }
    b->nitems = (int)items.size();
    b->ops_inv = b->ops_fwd;
    hipStream_t s = b->stream;
    svq_batch bp = b.get();
    BHIPCHK(bp, b->arena.ensure(sizeof(float2) * (size_t)arena_elems), "alloc arena");
    BHIPCHK(bp, upload(b->items, items, s), "upload items");
    BHIPCHK(bp, upload(b->stages, stages, s), "upload stages");
    BHIPCHK(bp, upload(b->dinsts, b->insts, s), "upload instances");
    BHIPCHK(bp, upload(b->passes, passes, s), "upload passes");
    BHIPCHK(bp, upload(b->hpasses, hpasses, s), "upload H passes");
    BHIPCHK(bp, upload(b->phases, phases, s), "upload phases");
    BHIPCHK(bp, upload(b->hgroups, hgroups, s), "upload H groups");
    BHIPCHK(bp, upload(b->hterms, hterms, s), "upload H terms");
    BHIPCHK(bp, upload(b->pptr, pptr, s), "upload pptr");
    BHIPCHK(bp, upload(b->pgate, pgate, s), "upload pgate");
    BHIPCHK(bp, b->d_ops_fwd.ensure(sizeof(OpDesc) * std::max<size_t>(1, b->ops_fwd.size())), "alloc ops");
    BHIPCHK(bp, b->d_ops_inv.ensure(sizeof(OpDesc) * std::max<size_t>(1, b->ops_fwd.size())), "alloc ops");
    BHIPCHK(bp, b->epart.ensure(sizeof(double) * std::max(1, epart_total)), "alloc epart");
    BHIPCHK(bp, b->gpart.ensure(sizeof(double) * std::max(1, gpart_total)), "alloc gpart");
    BHIPCHK(bp, b->energies.ensure(sizeof(double) * n_inst), "alloc energies");
    BHIPCHK(bp, b->grads.ensure(sizeof(double) * std::max(1, b->total_theta)), "alloc grads");
    BHIPCHK(bp, b->counters.ensure(sizeof(int32_t) * (b->nstages + 2)), "alloc counters");
    BHIPCHK(bp, b->t_done.ensure(sizeof(uint64_t) * n_inst), "alloc times");
    BHIPCHK(bp, b->t_start.ensure(sizeof(uint64_t)), "alloc time");
    BHIPCHK(bp, hipHostMalloc((void **)&b->h_ops_fwd, sizeof(OpDesc) * std::max<size_t>(1, b->ops_fwd.size())), "pinned ops");
    BHIPCHK(bp, hipHostMalloc((void **)&b->h_ops_inv, sizeof(OpDesc) * std::max<size_t>(1, b->ops_fwd.size())), "pinned ops");
    if (!b->linsts.empty()) {
        const size_t nl = std::max<size_t>(1, b->lops.size());
        BHIPCHK(bp, upload(b->d_linst, b->linsts, s), "upload LDS instances");
        BHIPCHK(bp, upload(b->d_lterms, lterms, s), "upload LDS terms");
        BHIPCHK(bp, b->d_gvals.ensure(sizeof(double) * std::max(1, gv_total)), "alloc gradient slots");
        BHIPCHK(bp, b->d_lops_fwd.ensure(sizeof(OpDesc) * nl), "alloc ops");
        BHIPCHK(bp, b->d_lops_inv.ensure(sizeof(OpDesc) * nl), "alloc ops");
        BHIPCHK(bp, hipHostMalloc((void **)&b->h_lops_fwd, sizeof(OpDesc) * nl), "pinned ops");
        BHIPCHK(bp, hipHostMalloc((void **)&b->h_lops_inv, sizeof(OpDesc) * nl), "pinned ops");
        BHIPCHK(bp, prepare_batch_lds(b->lds_max_n), "LDS limit");
    }
    BHIPCHK(bp, hipStreamSynchronize(s), "sync");
    BatchArgs &A = b->args;
    std::memset(&A, 0, sizeof(A));
    A.arena = (float2 *)b->arena.p;
    A.items = (const BatchItem *)b->items.p;
    A.stages = (const BatchStage *)b->stages.p;
    A.insts = (const BatchInst *)b->dinsts.p;
    A.passes = (const BatchPass *)b->passes.p;
    A.hpasses = (const BatchHPass *)b->hpasses.p;
    A.phases = (const PhaseDesc *)b->phases.p;
    A.ops_fwd = (const OpDesc *)b->d_ops_fwd.p;
    A.ops_inv = (const OpDesc *)b->d_ops_inv.p;
    A.hgroups = (const HpsiGroup *)b->hgroups.p;
    A.hterms = (const HpsiTerm *)b->hterms.p;
    A.pptr = (const int32_t *)b->pptr.p;
    A.pgate = (const int32_t *)b->pgate.p;
    A.epart = (double *)b->epart.p;
    A.gpart = (double *)b->gpart.p;
    A.energies = (double *)b->energies.p;
    A.grads = (double *)b->grads.p;
    A.done = (int32_t *)b->counters.p;
    A.head = (int32_t *)b->counters.p + b->nstages;
    A.error = (int32_t *)b->counters.p + b->nstages + 1;
    A.t_done = (uint64_t *)b->t_done.p;
    A.t_start = (uint64_t *)b->t_start.p;
    A.nitems = b->nitems;
    A.spin_limit = env_int("SVQ_BATCH_SPIN_LIMIT", kBatchSpinLimit);
    A.linst = (const BatchLdsInst *)b->d_linst.p;
    A.lops_fwd = (const OpDesc *)b->d_lops_fwd.p;
    A.lops_inv = (const OpDesc *)b->d_lops_inv.p;
    A.lterms = b->d_lterms.p;
    A.gvals = (double *)b->d_gvals.p;
    *out = b.release();
    return SVQ_OK;
}

svq_status sv_batch_run(svq_batch b, const double *const *theta, double *energies_host,
                        double *grads_host, double *latency_ms_host) {
    if (!b) return fail(SVQ_EINVAL, "null batch");
    if (b->poisoned) return fail(SVQ_EPOISONED, "batch poisoned by an earlier failure");
    if (!theta || !energies_host || !grads_host) return fail(SVQ_EINVAL, "null argument");
    BHIPCHK(b, hipSetDevice(b->device), "hipSetDevice");
    for (int i = 0; i < b->n_inst; ++i) {
        if (b->ntheta[i] && !theta[i]) return fail(SVQ_EINVAL, "theta[i] is NULL");
        for (int p = 0; p < b->ntheta[i]; ++p)
            if (!std::isfinite(theta[i][p])) return fail(SVQ_EINVAL, "non-finite theta");
    }
    // op coefficients for these angles, instance by instance
    size_t o = 0;
    for (int i = 0; i < b->n_inst; ++i) {
        size_t o1 = o;
        while (o1 < b->op_inst.size() && b->op_inst[o1] == i) ++o1;
        std::vector<OpDesc> f(b->ops_fwd.begin() + o, b->ops_fwd.begin() + o1);
        std::vector<int> og(b->op_gate.begin() + o, b->op_gate.begin() + o1);
        std::vector<OpDesc> inv = f;
        fill_ops(b->gates[i], theta[i], og, f, false);
        fill_ops(b->gates[i], theta[i], og, inv, true);
        for (size_t j = 0; j < inv.size(); ++j) {
            const GateN &g = b->gates[i][og[j]];
            inv[j].gslot = (g.param >= 0 && inv[j].gtype != GEN_NONE) ? og[j] : -1;
            if (inv[j].gslot < 0) inv[j].gtype = GEN_NONE;
        }
        std::memcpy(b->h_ops_fwd + o, f.data(), sizeof(OpDesc) * f.size());
        std::memcpy(b->h_ops_inv + o, inv.data(), sizeof(OpDesc) * inv.size());
        o = o1;
    }
    // LDS instances: ops in gate order
    for (size_t o = 0; o < b->lops.size();) {
        const int i = b->lop_inst[o];
        size_t o1 = o;
        while (o1 < b->lops.size() && b->lop_inst[o1] == i) ++o1;
        std::vector<OpDesc> f(b->lops.begin() + o, b->lops.begin() + o1);
        std::vector<int> og(f.size());
        for (size_t j = 0; j < og.size(); ++j) og[j] = (int)j;
        std::vector<OpDesc> inv = f;
        fill_ops(b->gates[i], theta[i], og, f, false);
        fill_ops(b->gates[i], theta[i], og, inv, true);
        for (size_t j = 0; j < inv.size(); ++j) {
            const GateN &g = b->gates[i][j];
            if (!(g.param >= 0 && inv[j].gtype != GEN_NONE)) inv[j].gtype = GEN_NONE;
        }
        std::memcpy(b->h_lops_fwd + o, f.data(), sizeof(OpDesc) * f.size());
        std::memcpy(b->h_lops_inv + o, inv.data(), sizeof(OpDesc) * inv.size());
        o = o1;
    }
    if (!b->lops.empty()) {
        BHIPCHK(b, hipMemcpyAsync(b->d_lops_fwd.p, b->h_lops_fwd, sizeof(OpDesc) * b->lops.size(), hipMemcpyHostToDevice, b->stream), "upload ops");
        BHIPCHK(b, hipMemcpyAsync(b->d_lops_inv.p, b->h_lops_inv, sizeof(OpDesc) * b->lops.size(), hipMemcpyHostToDevice, b->stream), "upload ops");
    }
    const size_t nops = b->ops_fwd.size();
    if (nops) {
        BHIPCHK(b, hipMemcpyAsync(b->d_ops_fwd.p, b->h_ops_fwd, sizeof(OpDesc) * nops, hipMemcpyHostToDevice, b->stream), "upload ops");
        BHIPCHK(b, hipMemcpyAsync(b->d_ops_inv.p, b->h_ops_inv, sizeof(OpDesc) * nops, hipMemcpyHostToDevice, b->stream), "upload ops");
    }
    if (!b->exec) {
        // capture the counter reset and the persistent kernel once
        hipStream_t cap;
        BHIPCHK(b, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
        BHIPCHK(b, hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
        int grid = 0;
        // completion times are maxima over an instance's final blocks
        hipError_t le = launch_fill_i32((int32_t *)b->t_done.p, 2 * b->n_inst, 0, cap);
        if (le != hipSuccess) {
        } else if (b->persistent) {
            le = launch_batch(b->args, (int32_t *)b->counters.p, b->nstages + 2, cap, &grid);
        }
        // The two size classes share no data: the small instances' launches
        // go on a branch of their own (forked and joined with events), so
        // they are not queued behind the large instances' launches.
        hipStream_t side = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
        if (le == hipSuccess && !b->persistent) {
            // the error flag stays zero: these launches never wait
            le = launch_fill_i32((int32_t *)b->counters.p, b->nstages + 2, 0, cap);
            if (le == hipSuccess) le = launch_stamp((uint64_t *)b->t_start.p, cap);   // before the fork
            bool cls_used[2] = {!b->linsts.empty(), false};
            for (const auto &gr : b->groups) cls_used[gr[3]] = true;
            const bool branch = cls_used[0] && cls_used[1];
            if (branch && le == hipSuccess) le = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
            if (branch && le == hipSuccess) le = hipEventCreateWithFlags(&join, hipEventDisableTiming);
            if (branch && le == hipSuccess) le = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
            if (branch && le == hipSuccess) le = hipEventRecord(fork, cap);
            if (branch && le == hipSuccess) le = hipStreamWaitEvent(side, fork, 0);
            if (le == hipSuccess)
                le = launch_batch_lds(b->args, (int)b->linsts.size(), b->lds_max_n, branch ? side : cap);
            for (size_t gi = 0; gi < b->groups.size() && le == hipSuccess; ++gi) {
                const auto &gr = b->groups[gi];
                le = launch_batch_stage(b->args, gr[0], gr[1], gr[2], (branch && gr[3] == 0) ? side : cap);
            }
            if (branch && le == hipSuccess) le = hipEventRecord(join, side);
            if (branch && le == hipSuccess) le = hipStreamWaitEvent(cap, join, 0);
        }
        hipError_t ce = hipStreamEndCapture(cap, &b->graph);
        if (side) (void)hipStreamDestroy(side);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        (void)hipStreamDestroy(cap);
        BHIPCHK(b, le, "launch batch");
        BHIPCHK(b, ce, "end capture");
        BHIPCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate graph");
    }
    BHIPCHK(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
    int32_t err = 0;
    BHIPCHK(b, hipMemcpyAsync(&err, (int32_t *)b->counters.p + b->nstages + 1, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream), "D2H");
    BHIPCHK(b, hipMemcpyAsync(energies_host, b->energies.p, sizeof(double) * b->n_inst, hipMemcpyDeviceToHost, b->stream), "D2H");
    if (b->total_theta)
        BHIPCHK(b, hipMemcpyAsync(grads_host, b->grads.p, sizeof(double) * b->total_theta, hipMemcpyDeviceToHost, b->stream), "D2H");
    std::vector<uint64_t> td(b->n_inst);
    uint64_t t0 = 0;
    BHIPCHK(b, hipMemcpyAsync(td.data(), b->t_done.p, sizeof(uint64_t) * b->n_inst, hipMemcpyDeviceToHost, b->stream), "D2H");
    BHIPCHK(b, hipMemcpyAsync(&t0, b->t_start.p, sizeof(uint64_t), hipMemcpyDeviceToHost, b->stream), "D2H");
    BHIPCHK(b, hipStreamSynchronize(b->stream), "sync");
    if (err) {
        b->poisoned = true;
        return fail(SVQ_EHIP, "batch: a dependency wait exceeded its bound");
    }
    if (latency_ms_host) {
        int khz = 100000;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device) != hipSuccess || khz <= 0)
            khz = 100000;
        for (int i = 0; i < b->n_inst; ++i)
            latency_ms_host[i] = (double)(int64_t)(td[i] - t0) / (double)khz;
    }
    return SVQ_OK;
}

svq_status sv_batch_info(svq_batch b, double *bytes_per_run, int32_t *n_stages, int32_t *n_items) {
    if (!b) return fail(SVQ_EINVAL, "null batch");
    if (bytes_per_run) *bytes_per_run = b->bytes_per_run;
    if (n_stages) *n_stages = b->nstages;
    if (n_items) *n_items = b->nitems;
    return SVQ_OK;
}

svq_status sv_batch_destroy(svq_batch b) {
    if (!b) return fail(SVQ_EINVAL, "null batch");
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    delete b;
    return SVQ_OK;
}

}  // extern "C"

// ===========================================================================
// measured tuning
// ===========================================================================

namespace {

// Time one call of fn on the stream (events around the second of two runs).
template <typename F>
svq_status time_twice(hipStream_t s, F fn, double *ms) {
    svq_status r = fn();
    if (r) return r;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return fail(SVQ_EHIP, "event");
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(SVQ_EHIP, "event");
    }
    (void)hipEventRecord(a, s);
    r = fn();
    (void)hipEventRecord(b, s);
    float f = 0.f;
    if (!r && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&f, a, b) != hipSuccess))
        r = fail(SVQ_EHIP, "event timing");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = f;
    return r;
}

}  // namespace

extern "C" {

svq_status sv_expectation_qsu(svq_state st, const svq_pauli *terms, int n_terms,
                              double *energy_host, double *energy_dev, svq_stats *stats) {
    svq_status s = check_state(st);
    if (s) return s;
    if (n_terms < 0 || (n_terms > 0 && !terms)) return fail(SVQ_EINVAL, "bad term list");
    const uint64_t full = st->n == 64 ? ~0ULL : ((1ULL << st->n) - 1);
    for (int t = 0; t < n_terms; ++t) {
        if ((terms[t].x & ~full) || (terms[t].z & ~full)) return fail(SVQ_EINVAL, "pauli mask beyond n qubits");
        if (!std::isfinite(terms[t].coef)) return fail(SVQ_EINVAL, "non-finite coefficient");
    }
    if (stats) std::memset(stats, 0, sizeof(*stats));
    HIPCHK(st, st->d_energy.ensure(sizeof(double)), "alloc energy");
    double *edev = energy_dev ? energy_dev : (double *)st->d_energy.p;
    const int nL = st->n - st->g;
    // ad hoc plan over the full supports, index order
    auto t0 = std::chrono::steady_clock::now();
    std::vector<uint64_t> targets(n_terms);
    std::vector<int> order(n_terms);
    for (int t = 0; t < n_terms; ++t) {
        targets[t] = __builtin_popcountll(terms[t].x) <= nL ? terms[t].x : 0;
        order[t] = t;
    }
    std::vector<int> pos_end = st->pos;
    std::vector<L1Tile> tiles = ad_hoc(st->n, nL, targets, order, pos_end);
    // each term's masks in the layout it runs under
    std::vector<WideTerm> wt(n_terms);
    std::vector<int> cur = st->pos;
    int nqr = 0;
    for (const L1Tile &T : tiles) {
        if (!T.qr.empty()) ++nqr;
        for (const Transposition &tr : T.qr)
            for (int q = 0; q < st->n; ++q) {
                if (cur[q] == tr.a) cur[q] = tr.b;
                else if (cur[q] == tr.b) cur[q] = tr.a;
            }
        for (int t : T.ops) {
            WideTerm &w = wt[t];
            std::memset(&w, 0, sizeof(w));
            for (int q = 0; q < st->n; ++q) {
                if ((terms[t].x >> q) & 1) w.x |= 1ULL << cur[q];
                if ((terms[t].z >> q) & 1) w.z |= 1ULL << cur[q];
            }
            w.coef = terms[t].coef;
            w.ny = __builtin_popcountll(terms[t].x & terms[t].z);
        }
    }
    if (cur != pos_end) return fail(SVQ_EINVAL, "internal: ad hoc layout mismatch");
    auto t1 = std::chrono::steady_clock::now();
    if (n_terms == 0) {
        HIPCHK(st, hipMemsetAsync(edev, 0, sizeof(double), st->stream), "zero energy");
    } else {
        const int dg = dot_grid(st->N());
        HIPCHK(st, st->d_lam.ensure(st->bytes()), "alloc psi'");
        HIPCHK(st, st->d_extra.ensure(sizeof(double) * dg), "alloc extra");
        DevBuf d_wt;
        HIPCHK(st, d_wt.ensure(sizeof(WideTerm) * n_terms), "alloc terms");
        HIPCHK(st, hipMemcpyAsync(d_wt.p, wt.data(), sizeof(WideTerm) * n_terms,
                                  hipMemcpyHostToDevice, st->stream),
               "upload terms");
        double bytes = 0.0;
        bool first = true;
        for (const L1Tile &T : tiles) {
            if (!T.qr.empty()) {
                s = run_qr(st, st->buf, T.qr);
                if (s) return s;
                if (!first) {
                    s = run_qr(st, st->d_lam.p, T.qr);
                    if (s) return s;
                }
                bytes += qr_bytes(st, T.qr) * (first ? 1.0 : 2.0);
            }
            for (int t : T.ops) {
                ProfScope ps(st, 5);
                HIPCHK(st, launch_hpsi_direct(st->dbl(), st->buf, st->d_lam.p, st->N(),
                                              (const WideTerm *)d_wt.p + t, 1, first ? 0 : 1,
                                              st->stream),
                       "pauli gate");
                bytes += (first ? 2.0 : 3.0) * (double)st->bytes();
                first = false;
            }
        }
        HIPCHK(st, launch_dot_re(st->dbl(), st->buf, st->d_lam.p, st->N(), (double *)st->d_extra.p,
                                 st->stream),
               "dot");
        HIPCHK(st, launch_sum((const double *)st->d_extra.p, dg, edev, st->stream), "sum");
        bytes += 2.0 * (double)st->bytes();
        // d_wt is freed when it goes out of scope: finish its readers first
        HIPCHK(st, hipStreamSynchronize(st->stream), "sync");
        if (stats) stats->bytes = bytes;
    }
    st->pos = pos_end;
    if (stats) {
        stats->n_qr = nqr;
        stats->n_evc_passes = n_terms;
        stats->ms_plan = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (energy_host)
        HIPCHK(st, hipMemcpyAsync(energy_host, edev, sizeof(double), hipMemcpyDeviceToHost, st->stream),
               "copy energy");
    if (energy_host) HIPCHK(st, hipStreamSynchronize(st->stream), "sync");
    return SVQ_OK;
}

svq_status sv_tune_circuit(svq_state st, const svq_gate *gates, int m, const double *theta,
                           int n_theta, svq_sched sched, int *k_out, int *c_out, double *ms_out) {
    svq_status s = check_state(st);
    if (s) return s;
    std::vector<GateN> gn;
    std::string err = normalize_gates(st->n, gates, m, n_theta, gn);
    if (!err.empty()) return fail(SVQ_EINVAL, err);
    s = check_theta(gn, theta, n_theta);
    if (s) return s;
    const int nl = st->n - st->g;
    TuneVal best{0, 0, 1e300};
    for (int k = 10; k <= std::min(13, nl); ++k)
        for (int c = 3; c <= 6; ++c) {
            set_tuned(0, st->n, st->g, (int)st->dtype, {k, c, 0.0});
            double ms = 0.0;
            auto fn = [&]() -> svq_status {
                svq_status r = sv_set_basis(st, 0);
                if (r) return r;
                return sv_apply_circuit(st, gates, m, theta, n_theta, sched, 0, nullptr);
            };
            s = time_twice(st->stream, fn, &ms);
            if (s) return s;
            if (ms < best.ms) best = {k, c, ms};
        }
    if (best.k == 0) return fail(SVQ_EUNSUP, "no tile width fits this state");
    set_tuned(0, st->n, st->g, (int)st->dtype, best);
    if (k_out) *k_out = best.k;
    if (c_out) *c_out = best.c;
    if (ms_out) *ms_out = best.ms;
    return SVQ_OK;
}

svq_status sv_tune_paulis(svq_state st, const svq_pauli *terms, int n_terms, int *k_out,
                          int *c_out, double *ms_out) {
    svq_status s = check_state(st);
    if (s) return s;
    const int nl = st->n - st->g;
    TuneVal best{0, 0, 1e300};
    for (int k = 11; k <= std::min(st->dbl() ? 13 : 14, nl); ++k)
        for (int c = 3; c <= 6; ++c) {
            set_tuned(1, st->n, st->g, (int)st->dtype, {k, c, 0.0});
            double ms = 0.0;
            auto fn = [&]() -> svq_status {
                return sv_expectation(st, terms, n_terms, SVQ_LAZY, nullptr, nullptr, nullptr, nullptr);
            };
            s = time_twice(st->stream, fn, &ms);
            if (s) return s;
            if (ms < best.ms) best = {k, c, ms};
        }
    if (best.k == 0) return fail(SVQ_EUNSUP, "no tile width fits this state");
    set_tuned(1, st->n, st->g, (int)st->dtype, best);
    if (k_out) *k_out = best.k;
    if (c_out) *c_out = best.c;
    if (ms_out) *ms_out = best.ms;
    return SVQ_OK;
}

svq_status sv_batch_tune(int n_inst, const int32_t *n_qubits, const svq_gate *const *gates,
                         const int32_t *m, const int32_t *n_theta, const svq_pauli *const *terms,
                         const int32_t *n_terms, const uint64_t *psi0, const double *const *theta,
                         void *stream, int *chunks_out, int *low_bits_out, double *ms_out) {
    if (n_inst <= 0 || !theta) return fail(SVQ_EINVAL, "bad arguments");
    int total = 0;
    for (int i = 0; i < n_inst; ++i) total += n_theta ? n_theta[i] : 0;
    std::vector<double> e(n_inst), g(std::max(1, total));
    TuneVal best{0, 0, 1e300};
    // items per stage, low bits, and the size class from which instances run
    // their gate and H|psi> passes on 2^12 tiles (27: none)
    const int chunk_c[] = {256, 1024};
    const int low_c[] = {3, 4};
    const int wide_c[] = {12, 16, 20, 27};
    TuneVal best_w{kBatchWideN, 0, 1e300};
    for (int ch : chunk_c)
        for (int c : low_c)
          for (int wn : wide_c) {
            set_tuned(2, 0, 0, 0, {ch, c, 0.0});
            set_tuned(3, 0, 0, 0, {wn, 0, 0.0});
            svq_batch b = nullptr;
            svq_status s = sv_batch_create(n_inst, n_qubits, gates, m, n_theta, terms, n_terms, psi0,
                                           0, stream, &b);
            if (s) return s;
            s = sv_batch_run(b, theta, e.data(), g.data(), nullptr);
            auto t0 = std::chrono::steady_clock::now();
            if (!s) s = sv_batch_run(b, theta, e.data(), g.data(), nullptr);
            auto t1 = std::chrono::steady_clock::now();
            (void)sv_batch_destroy(b);
            if (s) return s;
            const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
            if (ms < best.ms) {
                best = {ch, c, ms};
                best_w = {wn, 0, ms};
            }
          }
    set_tuned(2, 0, 0, 0, best);
    set_tuned(3, 0, 0, 0, best_w);
    if (chunks_out) *chunks_out = best.k;
    if (low_bits_out) *low_bits_out = best.c;
    if (ms_out) *ms_out = best.ms;
    return SVQ_OK;
}

svq_status sv_tune_save(const char *path) {
    if (!path) return fail(SVQ_EINVAL, "path is NULL");
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(SVQ_EINVAL, std::string("cannot write ") + path);
    std::lock_guard<std::mutex> lk(tune_mutex());
    for (const auto &kv : tune_table())
        std::fprintf(f, "%d %d %d %d %d %d %.6f\n", kv.first.kind, kv.first.n, kv.first.g,
                     kv.first.dt, kv.second.k, kv.second.c, kv.second.ms);
    std::fclose(f);
    return SVQ_OK;
}

svq_status sv_tune_load(const char *path) {
    if (!path) return fail(SVQ_EINVAL, "path is NULL");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(SVQ_EINVAL, std::string("cannot read ") + path);
    int kind, n, g, dt, k, c;
    double ms;
    int cnt = 0;
    while (std::fscanf(f, "%d %d %d %d %d %d %lf", &kind, &n, &g, &dt, &k, &c, &ms) == 7) {
        // kind 3 (the batch's wide-tile size class) stores no low-bit count
        if (kind < 0 || kind > 3 || k < 1 || c < (kind == 3 ? 0 : 1)) continue;
        set_tuned(kind, n, g, dt, {k, c, ms});
        ++cnt;
    }
    std::fclose(f);
    (void)cnt;
    return SVQ_OK;
}

}  // extern "C"
