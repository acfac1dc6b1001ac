// Host planner: turns a circuit or a Pauli sum into launchable steps.
//
// Level 1 (qubit reordering, the paper's method): which logical qubits are
//   chunk-local for which operators -- flat time-space tiling (Algs. 1-3) or
//   the ad hoc eager baseline for circuits; Alg. 6 with diagonalization or
//   index-order eager for Pauli sums.
// Level 2 (HBM passes): inside one level-1 tile, pack operators into passes
//   over 2^k-amplitude tiles that always contain the c lowest physical bits
//   (coalescing), by the same tile-construction / qubit-mapping greedy.
// Level 3 (register phases): inside one pass, the same greedy with RB
//   register bits, where only mixing qubits must be register bits.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "svq.h"
#include "svq_dev.hpp"

namespace svq {

struct GateN {
    int kind = 0;
    int nq = 1;
    int q[2] = {0, 0};
    int param = -1;
    double scale = 1.0;    // angle = scale * theta[param] + offset (param >= 0)
    double offset = 0.0;   // the whole angle when param < 0
    double mat[32] = {0};
    uint64_t tmask = 0;    // all qubits of the gate
    uint64_t mixmask = 0;  // qubits whose bit value the gate mixes
    uint64_t ctrlmask = 0; // control qubits (must be 1)
    int diag_q = -1;       // diagonal gates: the qubit carrying the phase
};

// Validate and normalise a gate list.  Returns "" or an error message.
std::string normalize_gates(int n, const svq_gate *gates, int m, int n_theta,
                            std::vector<GateN> &out);

// ---- level 1 ---------------------------------------------------------------

struct Transposition { int a, b; };   // physical bit positions

struct L1Tile {
    uint64_t local = 0;                 // logical qubits that are local
    std::vector<int> ops;               // operator indices in schedule order
    std::vector<Transposition> qr;      // physical swaps executed before the tile
};

// Depth of every operator (critical-path length) and the depth order with
// ties broken by ascending target qubits (Section "Flat tiling").
std::vector<int> depth_order(const std::vector<uint64_t> &targets);

// Flat tiling, Algs. 1-3.  targets: logical target masks.  pos: physical bit
// of each logical qubit at the start; it is updated to the final layout.
std::vector<L1Tile> flat_tiling(int n, int nL, const std::vector<uint64_t> &targets,
                                std::vector<int> &pos);

// Ad hoc baseline: breadth-first order; on a wide operator swap the missing
// qubits in, evicting the local qubits at the highest physical positions
// that the operator does not target.
std::vector<L1Tile> ad_hoc(int n, int nL, const std::vector<uint64_t> &targets,
                           const std::vector<int> &order, std::vector<int> &pos);

// Hierarchical tiling, Algs. 4-5: local set plus n_intra intra qubits; a
// remap first tries the intra-only pool Q_L u Q_intra (an intra QR) and
// otherwise chooses from all qubits (an inter QR).  fill_highest selects the
// boundary fill of Alg. 3.  kinds[t] = 1 for an inter QR before tile t.
std::vector<L1Tile> hierarchical_tiling(int n, int nL, int n_intra,
                                        const std::vector<uint64_t> &targets, bool fill_highest,
                                        std::vector<int> &kinds, std::vector<uint64_t> &intra);

// Alg. 6 over weighted supports (bit masks); ties prefer the current local
// set, then the lexicographically first one.
std::vector<L1Tile> tiling_pauli(int n, int nL, const std::vector<uint64_t> &supports,
                                 const std::vector<int> &weights, std::vector<int> &pos);

// ---- full plans -------------------------------------------------------------

struct Step {
    int type = 0;        // 0 = QR (transpositions), 1 = pass
    int idx = 0;         // pass index
    std::vector<Transposition> qr;
};

struct CircuitPlan {
    int n = 0, g = 0, k = 0, rb = 0, c = 0;
    std::vector<int> order;                  // gate index per schedule position
    std::vector<int> pos_qrtile, pos_pass;   // per schedule position
    std::vector<uint64_t> pos_local;         // local logical set per position
    int n_qr = 0;
    std::vector<Step> steps;
    std::vector<PassArgs> passes;
    std::vector<PhaseDesc> phases;
    std::vector<OpDesc> ops;                 // forward ops (coefficients filled per call)
    std::vector<int> op_gate;                // gate index of every op
    std::vector<int> pos_before, pos_after;  // layouts
    int n_phases_total = 0;
};

// relayout: passes may store their tile with its bit positions permuted
// (PassArgs::tphys_out), so that the next pass's qubits sit on the c lowest
// positions; otherwise every tile takes the c lowest positions as they are.
// One gate pass without gates over the tile bits tile_bits[0..k) (ascending
// physical positions): nphase phases whose registers alternate between the
// tile's top rb bits and the rb bits above the six lowest, so that every
// phase change is a full LDS transpose.  The load phase has its lanes on the
// six lowest tile bits.  Used to measure the data movement of a pass alone.
std::string plan_empty_pass(int n, int k, int rb, const int *tile_bits, int nphase, CircuitPlan &out);

std::string plan_circuit(int n, int g, const std::vector<GateN> &gates, svq_sched sched, int k,
                         int rb, int c, const std::vector<int> &pos0, CircuitPlan &out,
                         bool relayout = true);

// The op type that applies gates of this kind (OpType).
int op_type_for_kind(int kind);

// Fill op coefficients for the given angles (forward).  For the adjoint sweep
// `inverse` fills U^dagger and the generator data.
void fill_ops(const std::vector<GateN> &gates, const double *theta, const std::vector<int> &op_gate,
              std::vector<OpDesc> &ops, bool inverse);

struct PauliPlan {
    int n = 0, g = 0, k = 0, c = 0;
    std::vector<int> group_of_term;
    std::vector<uint64_t> group_x;
    std::vector<std::vector<int>> group_terms;
    std::vector<int> order;                  // group index per position
    std::vector<int> pos_qrtile, pos_pass;
    std::vector<uint64_t> pos_local;
    int n_qr = 0;
    std::vector<Step> steps;
    // EVC tables
    std::vector<EvcPassArgs> passes;
    std::vector<EvcGroup> groups;
    std::vector<EvcTerm> terms;
    // H|psi> tables (same passes)
    std::vector<HpsiPassArgs> hpasses;
    std::vector<HpsiGroup> hgroups;
    std::vector<HpsiTerm> hterms;
    std::vector<int> wide_groups;            // groups too wide for any tile (direct kernel)
    std::vector<int> wide_after_step;        // unused placeholder
    std::vector<int> pos_before, pos_after;
    int total_blocks = 0;                    // sum of blocks over passes (partials)
};

// dbl selects the EVC thread geometry of the complex128 kernels.
std::string plan_paulis(int n, int g, const svq_pauli *terms, int nt, svq_sched sched, int k,
                        int c, bool dbl, const std::vector<int> &pos0, PauliPlan &out);

}  // namespace svq
