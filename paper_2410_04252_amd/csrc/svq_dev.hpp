// Descriptor tables shared by the host planner and the HIP kernels.
//
// A plan is a sequence of steps.  A QR step permutes physical bit positions
// (an involution: disjoint transpositions).  A gate pass streams the state
// once: every workgroup owns one tile of 2^k amplitudes whose indices agree
// on all non-tile bits (all tile bits are chunk-local, so a tile never spans
// two chunks -- narrow access, constraint C2), keeps it in registers and LDS,
// and applies a run of gates.  Inside a pass the tile is walked in register
// phases: in a phase every thread holds 2^RB amplitudes that differ in the
// phase's RB "register" tile bits; gates that mix amplitudes act only on
// register bits, diagonal gates and controls act on any tile bit.  Between
// phases the tile is transposed through LDS.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace svq {

constexpr int kMaxTileBits = 14;
constexpr int kLaneBits = 6;      // wave64

// Register bits per thread of a gate pass over 2^k amplitudes (at least one
// wave per tile).  A fifth bit cuts the phases (LDS transposes) of the
// 30-qubit fabric plan by a fifth but doubles the amplitude registers, and
// measured no faster; the streaming forward pass also holds the next tile.
constexpr int gate_rb(int k, bool dbl = false, bool adj = false) {
    (void)dbl;
    (void)adj;
    return k - 6 < 4 ? k - 6 : 4;
}
// Threads (log2) of a Pauli pass: every thread owns a 2^(k-1-tpb) cube of
// the half space (EVC) or a 2^(k-tpb) cube of outputs (H|psi>).  Eight pairs
// per thread keep twice as many waves resident per staged tile as sixteen
// would (the tile, not the registers, limits residency).
constexpr int evc_tpb(int k, bool dbl = false) {
    (void)dbl;
    return k - 4 > 6 ? k - 4 : 6;
}
constexpr int hpsi_tpb(int k) { return k - 4 > 6 ? k - 4 : 6; }

// Gate-pass operations.  Every qubit of a gate is a register bit in the
// phase that applies it, so b0/b1 (register-bit positions; b0 = the gate
// matrix's local bit 0, for controlled gates the control) are compile-time
// values after dispatch and no per-amplitude index test is needed.
enum OpType : int32_t {
    OP_DIAG1 = 0,   // amp *= (bit b0 ? d1 : d0);               m = {d0.re, d0.im, d1.re, d1.im}
    OP_MIX1 = 1,    // 2x2 dense on b0;                          m = row-major complex 2x2
    OP_XSWAP = 2,   // swap along b0 (X)
    OP_GIVENS = 3,  // real rotation of (|b0=1,b1=0>, |b0=0,b1=1>); m = {c, s}
    OP_MIX2 = 4,    // 4x4 dense on (b0, b1);                    m = row-major complex 4x4
    OP_CPHASE = 5,  // amp *= d1 where both bits are set;        m = {-, -, d1.re, d1.im}
    OP_CNOT = 6,    // swap along b1 where b0 is set
    OP_ROTY = 7,    // real 2x2 [[c, -s], [s, c]] on b0;         m = {c, s}
};

// Generator K of a parametric op (U = exp(-i t K)), for the adjoint sweep,
// times the gate's angle scale d t / d theta (chain rule).
enum GenType : int32_t {
    GEN_NONE = 0,
    GEN_DIAG1 = 1,   // diag(k0, k1) on b0 (real)
    GEN_MIX1 = 2,    // 2x2 Hermitian on b0: k = row-major complex 2x2
    GEN_GIVENS = 3,  // k0 (X_b0 Y_b1 - Y_b0 X_b1)/4
    GEN_CPHASE = 4,  // -k0 |11><11| on (b0, b1)
};

// Unit-modulus ops (ROTY, GIVENS: a real rotation of an amplitude pair;
// CPHASE, DIAG1: a phase, i.e. a rotation of (re, im)) run in place as three
// shears, x += -t y; y += s x; x += -t y with t = tan(a/2), s = sin(a), which
// needs no temporaries.  The angle is first reduced to |a| <= pi/2 (then
// |t| <= 1) by writing R(a) = -R(a - pi); bit i of `flip` marks rotation i as
// negated afterwards.  m[16 + 2i] = t_i, m[17 + 2i] = s_i.
struct OpDesc {
    int32_t type;
    int32_t b0, b1;
    int32_t flip;
    int32_t spare;
    int32_t gslot;   // adjoint: slot of this gate in the gradient partials (-1: none)
    int32_t gtype;   // GenType
    int32_t pad;
    // shear parameters (t, s) of one or two rotations, next to the header so
    // that one scalar load brings an op's code and its parameters
    double sh[4];
    double m[32];
    double k[8];
};

// Device-resident descriptors use 32-bit fields only: gfx9 scalar loads are
// dword-granular, and a sub-dword field would be fetched by a vector load
// whose vmcnt wait also stalls on the tile's outstanding global loads.
struct PhaseDesc {
    int32_t reg[8];   // tile-local bit of register bit b
    int32_t lane[8];  // tile-local bit of lane bit b (6 used)
    int32_t wave[8];  // tile-local bit of wave bit b
    int32_t op0, nop;
    // LDS slot contribution of register, lane and wave bit b under the pass's
    // slot map (PassArgs::swz of the tile bit), stored here so that a
    // transpose reads them with the phase instead of through a second,
    // dependent lookup
    int32_t rsl[8], lsl[8], wsl[8];
};

struct PassArgs {
    int32_t nphase;
    int32_t phase0;
    int32_t spare;
    int32_t nblocks;
    // 32-bit entries: the kernels index them with phase-table values, which
    // must stay scalar loads (a byte would be a vector load whose wait also
    // waits for the tile's amplitude loads in flight).
    int32_t tphys[16];     // physical bit of tile-local bit j when loaded (ascending)
    int32_t tphys_out[16]; // physical bit of tile-local bit j when stored: a
                           // permutation of tphys (the same addresses), so a
                           // pass may relabel its tile's positions in place
    int32_t swz[16];       // LDS slot of tile-local index t: the XOR of swz[j]
                           // over the set bits j of t (a bijection of the tile)
};

// Read-only Pauli pass (EVC) and H|psi> pass.
// The fields the Pauli pass reads per group come first (one 32-byte scalar
// load); the stride is a power of two.
struct EvcGroup {
    uint32_t xl;          // tile-local flip mask (0 for the diagonal group)
    int32_t hbit;         // tile-local half-space bit (the pair partner flips it)
    int32_t nt;           // term count
    int32_t need;         // bit0: real array used, bit1: imaginary array used
    int32_t wbits[4];     // tile-local bits of the per-thread cube index (Q <= 3)
    int32_t t0;           // first term
    int32_t pad[7];
    int32_t tbits[16];    // tile-local bits of the thread index (low to high)
};
static_assert(sizeof(EvcGroup) == 128, "EvcGroup layout");

// Bits kEvcWiShift and up of EvcTerm::ztw hold the term's index into the
// per-thread Walsh arrays: the z bits in cube-index coordinates, plus the
// cube size when the term reads the imaginary (or difference) array.
constexpr int kEvcWiShift = 24;

struct EvcTerm {
    double coef;          // a_t with the i^{nY} sign and pair factor folded in
    uint32_t ztw;         // bits 0..23: tile-local z bits on thread-index bits;
                          // bits 24..28: Walsh-array index (see above)
    uint32_t zb;          // z bits outside the tile in block-index coordinates
                          // (tile sign = parity of blockIdx & zb)
};

// Four terms are one 64-byte scalar load.
static_assert(sizeof(EvcTerm) == 16, "EvcTerm layout");

struct EvcPassArgs {
    int32_t ngroups;
    int32_t group0;
    int32_t part0;        // offset of this pass's block partials
    int32_t nblocks;
    int8_t tphys[16];
};

// H|psi> pass: fixed output cube for the whole pass.
struct HpsiGroup {
    uint32_t xl;          // tile-local flip mask
    uint32_t xt;          // flip bits on thread-index bits
    uint32_t xw;          // flip bits in cube coordinates
    int32_t t0, nt;
    int32_t pad;
};

// Bits kHpsiZwShift and up of HpsiTerm::ztw hold the term's z bits in cube
// coordinates (its index into the per-thread spectra).
constexpr int kHpsiZwShift = 24;

struct HpsiTerm {
    float are_f, aim_f;   // a_t * i^{nY}, rounded to single precision
    uint32_t ztw;         // bits 0..23: z bits on thread-index bits; bits 24..: cube z bits
    uint32_t zb;          // z bits outside the tile in tile-index coordinates
                          // (tile sign = parity of tile index & zb)
    double are, aim;      // a_t * i^{nY}
};
static_assert(sizeof(HpsiTerm) == 32, "HpsiTerm layout");

struct HpsiPassArgs {
    int32_t ngroups;
    int32_t group0;
    int32_t accumulate;   // 0: first pass writes lambda, 1: lambda += pass
    int32_t pad;
    int8_t tphys[16];
    int8_t tbits[16];     // thread-index bits (tile-local)
    int8_t wbits[8];      // cube bits (tile-local)
};

}  // namespace svq

namespace svq {

// ---------------------------------------------------------------------------
// Batched persistent launch: many independent instances (g = 0, all qubits
// local), every stage of every instance cut into tiles of 2^10 amplitudes,
// processed by single-wave blocks that pull (instance, stage, tile) items from
// one queue.  All descriptor fields are 32-bit (scalar loads).
// ---------------------------------------------------------------------------

constexpr int kBatchK = 10;          // tile bits of the batched stages
constexpr int kBatchKWide = 12;      // tile bits of the gate passes of large instances
constexpr int kBatchWideN = 16;      // instances of at least this many qubits use them
constexpr int kBatchLdsN = 13;       // instances of at most this many qubits run in LDS
constexpr int kBatchLdsThreads = 512;
constexpr int kBatchSpinLimit = 1 << 24;

enum ItemType : int32_t {
    IT_INIT = 0,    // write psi0 into the tile
    IT_FWD = 1,     // forward gate pass
    IT_HPSI = 2,    // lambda (+)= H psi, one pass
    IT_DOT = 3,     // tile partial of Re <psi|lambda>
    IT_ADJ = 4,     // reverse adjoint pass on psi and lambda
    IT_FINAL = 5,   // energy and gradient of the instance
    IT_FWD_W = 6,   // forward gate pass on 2^12-amplitude tiles (4-wave blocks)
    IT_ADJ_W = 7,   // reverse adjoint pass on 2^12-amplitude tiles
    IT_HPSI_W = 8,  // H|psi> pass on 2^12-amplitude tiles
};

// One item: tiles [tile0, tile0 + ntile) of one stage, handled by one block,
// which then publishes its completion once (one release per item, so the
// number of cross-XCD cache write-backs stays small).
struct BatchItem {
    int32_t inst, stage, tile0, ntile;
    int32_t chunk, pad[3];
};

struct BatchStage {
    int32_t type;        // ItemType
    int32_t ntiles;      // tiles of the stage
    int32_t desc;        // gate pass or H pass index
    int32_t accumulate;  // H pass: add into lambda
};

struct BatchPass {
    int32_t tphys[16];   // physical bit of tile-local bit j
    int32_t swz[16];     // LDS slot map, as PassArgs::swz
    int32_t phase0, nphase;
    int32_t pad[2];
};

struct BatchHPass {
    int32_t tphys[16];
    int32_t group0, ngroups;
    int32_t pad[2];
};

struct BatchInst {
    int32_t n, stage0, nstages, ntiles;
    int32_t nchunks, pad0[3];     // items per stage (energy/gradient partial slots)
    int64_t psi_off, lam_off;     // element offsets in the state arena
    uint32_t psi0_lo, psi0_hi;    // initial basis state
    int32_t epart_off, gpart_off; // energy partials (nchunks), gradient partials (m * nchunks)
    int32_t m, ntheta;
    int32_t pptr_off, pgate_off;  // CSR parameter -> gates
    int32_t grad_off, pad;
};

// An instance evaluated entirely in one workgroup's LDS (psi and lambda,
// 2 x 2^n complex64).  Its ops are in gate order with the gate's qubits on
// register bits 0/1 (OpDesc::spare = first qubit, OpDesc::pad = second or -1).
struct BatchLdsInst {
    int32_t n, m, op0, t0;        // qubits, gates, first op, first term
    int32_t nt, ntheta, grad_off, pptr_off;
    int32_t gv_off, inst;         // per-gate gradient slots; index in the batch
    uint32_t psi0_lo, psi0_hi;
};

struct BatchArgs {
    float2 *arena;
    const BatchItem *items;
    const BatchStage *stages;
    const BatchInst *insts;
    const BatchPass *passes;
    const BatchHPass *hpasses;
    const PhaseDesc *phases;
    const OpDesc *ops_fwd;
    const OpDesc *ops_inv;
    const HpsiGroup *hgroups;
    const HpsiTerm *hterms;
    const int32_t *pptr;
    const int32_t *pgate;
    double *epart;
    double *gpart;
    double *energies;
    double *grads;
    int32_t *done;            // per (instance, stage) completed tiles
    int32_t *head;            // queue head
    int32_t *error;           // set when a bounded wait expires
    uint64_t *t_done;         // per instance: realtime clock at completion
    uint64_t *t_start;        // realtime clock when the first block started
    int32_t nitems;
    int32_t spin_limit;
    // instances held in LDS (k_batch_lds)
    const BatchLdsInst *linst;
    const OpDesc *lops_fwd;
    const OpDesc *lops_inv;
    const void *lterms;       // WideTerm[] in logical (= physical) order
    double *gvals;            // per gate of an LDS instance: 2 Im <lambda|K|psi>
};

}  // namespace svq
