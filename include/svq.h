/*
 * svq -- single-GPU state-vector simulation under lazy qubit reordering.
 *
 * C ABI of libsvq.so.  Plain pointers and sizes only; every call returns an
 * svq_status and never throws.  Device pointers are HIP device memory on the
 * current device; "stream" is a hipStream_t passed as void* (NULL = the
 * default stream).
 *
 * Terms from "Lazy Qubit Reordering for Accelerating Parallel
 * State-Vector-based Quantum Circuit Simulation":
 *   - the state vector holds 2^n complex amplitudes, qubit q = bit q of the
 *     logical index, qubit 0 the least significant bit (Section
 *     "Preliminaries", eq. sv);
 *   - the buffer is split into 2^g chunks by its g most significant physical
 *     bits; those bits hold the "global" qubits Q_G, the others the local
 *     qubits Q_L (Section "State vector distribution", eq. sub_sv;
 *     Section "Qubit mapping", eq. qubit_division).  On one GPU the chunks
 *     stand in for the paper's processing elements;
 *   - a qubit reordering (QR) exchanges equal-size subsets of Q_L and Q_G,
 *     swapping the elements whose indices differ in the exchanged bit pairs
 *     (Section "Qubit reordering"); here it is an in-HBM bit permutation;
 *   - a gate (QSU, eq. update_sv_reorder) or Pauli string (EVC, eq. evc) is
 *     only ever applied to data inside one chunk (narrow access, constraint
 *     C2, eq. qr_map_cond).
 *
 * Physical layout: the handle keeps pos[q], the physical bit that holds
 * logical qubit q.  Calls that reorder qubits change pos[] but never the
 * logical state; sv_get_amplitudes always returns logical order.
 */
#ifndef SVQ_C_ABI_H
#define SVQ_C_ABI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct svq_state_s *svq_state;

typedef enum { SVQ_C64 = 0, SVQ_C128 = 1 } svq_dtype;

/* EAGER: breadth-first order, reorder as soon as an operator is wide (the ad
 * hoc baseline of the paper's evaluation).  LAZY: time-space tiling, Algs.
 * 1-3 for circuits and Alg. 6 with diagonalization for Pauli sums. */
typedef enum { SVQ_EAGER = 0, SVQ_LAZY = 1 } svq_sched;

typedef enum {
    SVQ_OK = 0,
    SVQ_EINVAL = -1,     /* bad argument; the handle is unchanged */
    SVQ_ENOMEM = -2,     /* a device allocation failed (or exceeded the optional
                            cap SVQ_MAX_ALLOC_BYTES, in bytes, read from the
                            environment); scratch is allocated before any
                            launch, so the handle is unchanged and usable */
    SVQ_EHIP = -3,       /* a HIP call failed; the handle is poisoned */
    SVQ_ESHAPE = -4,     /* sizes inconsistent (buffer too small, n out of range) */
    SVQ_EUNSUP = -5,     /* valid but not supported by this library */
    SVQ_EPOISONED = -6   /* an earlier HIP failure poisoned the handle */
} svq_status;

typedef enum {
    SVQ_H = 0, SVQ_X = 1, SVQ_Y = 2, SVQ_Z = 3, SVQ_S = 4, SVQ_T = 5,
    SVQ_RX = 6, SVQ_RY = 7, SVQ_RZ = 8,
    SVQ_CNOT = 9,      /* q[0] control, q[1] target */
    SVQ_CZ = 10,
    SVQ_CPHASE = 11,   /* diag(1,1,1,e^{i t}) */
    SVQ_GIVENS = 12,   /* rotation by t/2 in span{|q0=1,q1=0>, |q0=0,q1=1>} */
    SVQ_SWAP = 13,
    SVQ_U1 = 14,       /* dense 2x2 from mat[] */
    SVQ_U2 = 15        /* dense 4x4 from mat[] */
} svq_gate_kind;

/* One gate.  The gate's matrix uses local index l = sum_j bit_{q[j]} 2^j, so
 * q[0] is the low bit (the paper leaves the order open).  The angle is
 * scale * theta[param] + offset when param >= 0, else offset, so one
 * parameter may drive several gates through different affine maps (sv_grad
 * applies the chain rule).  Parametric kinds follow U(t) = exp(-i t K):
 * RX/RY/RZ K = sigma/2; CPHASE K = -|11><11|; GIVENS K = (X_q0 Y_q1 -
 * Y_q0 X_q1)/4.  scale and offset must be finite. */
typedef struct {
    int32_t kind;
    int32_t q[2];
    int32_t param;     /* index into theta[], or -1 for a fixed angle */
    double scale;      /* d angle / d theta[param] (ignored when param < 0) */
    double offset;     /* added to the angle; the whole angle when param < 0 */
    double mat[32];    /* U1: 2x2, U2: 4x4, row-major complex as (re, im) */
} svq_gate;

/* Pauli string (eq. pauli_form): X at q if only x has bit q, Z if only z,
 * Y if both.  coef is the real coefficient a_t of eq. hamiltonian. */
typedef struct {
    uint64_t x, z;
    double coef;
} svq_pauli;

typedef struct {
    int32_t n_qr;            /* qubit reorderings executed (eq. n_qr) */
    int32_t n_gate_passes;   /* fused gate passes, one HBM read+write each */
    int32_t n_evc_passes;    /* read-only Pauli passes */
    int32_t n_groups;        /* X/Y flip-mask groups of the Hamiltonian */
    int32_t n_phases;        /* register phases over all passes */
    int32_t tile_k;          /* tile width used (bits) */
    double bytes;            /* algorithmic HBM bytes of the launched passes (sv_grad:
                                the whole call, forward, H|psi>, dot and reverse) */
    double ms_plan;          /* host planning time, 0 when the plan was cached */
} svq_stats;

/* Create a state of n qubits (1 <= n <= 34), g emulated global qubits
 * (0 <= g < n, 8 <= n - g <= 32: a chunk holds at most 2^32 amplitudes), dtype c64 (float2, FP32 arithmetic) or c128
 * (double2).  dev_buf: borrowed device buffer of >= 2^n * 8 (c64) or 16
 * (c128) bytes that must outlive the handle, or NULL to let the library
 * allocate (and free on destroy).  The state starts as |0...0> with
 * pos[q] = q.  Errors: EINVAL (n, g, dtype), ESHAPE (buf_bytes), ENOMEM,
 * EHIP. */
svq_status sv_create(int n, int g, svq_dtype dtype, void *dev_buf, size_t buf_bytes,
                     void *stream, svq_state *out);
svq_status sv_destroy(svq_state st);

/* Set the logical basis state |index>, resetting the layout to pos[q] = q. */
svq_status sv_set_basis(svq_state st, uint64_t index);

/* Copy a host array of 2^n amplitudes in logical order (complex64 or
 * complex128 as the handle's dtype) into the state; layout reset to
 * identity. */
svq_status sv_set_amplitudes(svq_state st, const void *host_logical);

/* Copy the state to a host array in logical order.  May reorder the device
 * buffer back to the identity layout first (the logical state is kept). */
svq_status sv_get_amplitudes(svq_state st, void *host_logical);

/* The last plan this handle executed (sv_apply_circuit, sv_expectation,
 * sv_grad's circuit plan) as JSON text, for inspection and tests: schedule,
 * tile width k, low bits c, QR count (eq. n_qr), the schedule order, and the
 * steps in launch order -- {"type":"qr","swaps":[[a,b],...]} with physical bit
 * pairs, {"type":"gate_pass","tile_bits":[...],"tile_bits_out":[...],
 * "gates":G,"phases":F} (tile bit j is read from physical position
 * tile_bits[j] and written to tile_bits_out[j]) or
 * {"type":"pauli_pass","tile_bits":[...],"groups":X} -- plus the layouts
 * before and after.  "{}" before any plan ran.  *len_out (nullable) receives
 * the size including the terminating NUL; json_buf may be NULL to query it.
 * Errors: EINVAL (null handle), ESHAPE (cap too small; nothing written). */
svq_status sv_plan_dump(svq_state st, char *json_buf, size_t cap, size_t *len_out);

/* Physical position of every logical qubit (pos_out[n]). */
svq_status sv_get_layout(svq_state st, int32_t *pos_out);

/* Device pointer of the amplitude buffer (physical order). */
svq_status sv_device_ptr(svq_state st, void **ptr_out);

/* QSU (eq. update_sv_gate): psi <- U_{m-1} ... U_0 psi, run under the given
 * schedule.  LAZY uses flat time-space tiling (Algs. 1-3, Section "Flat
 * tiling") over the chunk-local qubits, then packs each QR tile's gates into
 * LDS-resident passes of 2^tile_k amplitudes.  EAGER reorders on every wide
 * gate in breadth-first order.  tile_k = 0 picks the tuned width.  theta may
 * be NULL when no gate has param >= 0.  Plans are cached per (gates'
 * structure, n, g, layout, schedule, tile); angles are re-read every call.
 * Errors: EINVAL (kind, qubits, param, non-finite angle), EHIP. */
svq_status sv_apply_circuit(svq_state st, const svq_gate *gates, int m, const double *theta,
                            int n_theta, svq_sched sched, int tile_k, svq_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * sv_apply_circuit, but the phase and op descriptor tables of the call live in
 * a static 4 MiB device array of the library (one per GPU, kept until the
 * process ends) instead of buffers the handle allocates, so the call makes no
 * device allocation.  The handle should borrow its state buffer (sv_create
 * with dev_buf).  Host-side plans are cached on the handle as usual.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU (two
 * streams or threads) race and must be serialised by the caller.  Errors: as
 * sv_apply_circuit, plus ESHAPE when the tables exceed 4 MiB (about 10,900
 * gates at 384 bytes each; nothing runs then). */
svq_status sv_apply_circuit_static(svq_state st, const svq_gate *gates, int m,
                                   const double *theta, int n_theta, svq_sched sched,
                                   int tile_k, svq_stats *stats);

/* Reorder to a new layout: new_pos[q] = physical bit of logical qubit q (a
 * permutation of 0..n-1).  An involutive relayout (a set of disjoint bit
 * transpositions, as every QR of Section "Qubit reordering" is) runs as one
 * in-place pass that touches only the fraction 1 - 2^{-s} of elements whose
 * exchanged bits differ; any other permutation runs as two such passes. */
svq_status sv_qr_permute(svq_state st, const int32_t *new_pos);

/* EVC (eq. evc): E = sum_t a_t <psi|P_t|psi>.  Pauli strings are grouped by
 * X/Y mask; LAZY tiles the groups with Alg. 6 using diagonalization (only the
 * X/Y sites must be local, eq. without_QR / eq. par_exp), EAGER visits terms
 * in index order and reorders as needed.  Per-chunk partial sums E_j (eq.
 * local_evc) are reduced in FP64 (eq. aggregation).  energy_host (sync) and/or
 * energy_dev (device double, async on the stream) receive E; chunk_dev
 * (nullable, 2^g doubles) receives the per-chunk sums.  Errors: EINVAL
 * (masks >= 2^n, non-finite coefficient), EHIP. */
svq_status sv_expectation(svq_state st, const svq_pauli *terms, int n_terms, svq_sched sched,
                          double *energy_host, double *energy_dev, double *chunk_dev,
                          svq_stats *stats);

/* QSU-based EVC, the comparison method of Section "Evaluation" (EVC part):
 * psi' = H|psi> is built by applying each Pauli string as a gate, in the
 * terms' index order, with ad hoc reordering that makes the string's X/Y
 * sites local (its Z sites are a diagonal phase and need no locality, as in
 * eq. par_exp); both psi and psi' are permuted at every QR.  Then
 * E = Re <psi|psi'> in FP64.  Each term costs one elementwise pass that reads
 * psi and psi' and writes psi'.  A string with more X/Y sites than local
 * qubits runs without a reorder.  Same outputs and errors as sv_expectation
 * (no chunk sums); stats->n_qr counts the reorders. */
svq_status sv_expectation_qsu(svq_state st, const svq_pauli *terms, int n_terms,
                              double *energy_host, double *energy_dev, svq_stats *stats);

/* H|psi> into a second handle of the same shape (out).  FP64 accumulation. */
svq_status sv_apply_hamiltonian(svq_state st, const svq_pauli *terms, int n_terms,
                                svq_state out);

/* Gradient of E(theta) = <psi0|U(theta)^dag H U(theta)|psi0> by the adjoint
 * method (objective eq. vqe): forward pass, lambda = H psi, then a reverse
 * sweep that un-applies every gate on psi and lambda (no per-layer
 * checkpoints: one forward and one adjoint state) while summing
 * dE/dtheta_p = sum over the gates j of p of scale_j * 2 Im <lambda|K_j|psi>
 * (FP64 per-block partials, then a deterministic FP64 reduction).  The
 * handle's current state is psi0.  The reverse sweep recomputes psi0 from
 * U(theta)psi0, so on return the handle holds psi0 again (equal to the input
 * up to rounding: about 1e-7 per call in complex64), in its original layout,
 * ready for the next parameter vector; U(theta)psi0 itself is not kept (it
 * would cost a third state or a second forward pass).  grad_host/grad_dev
 * receive n_theta doubles, energy_host/energy_dev E.  Scratch: lambda (one
 * state) plus (parametric gates of the largest pass) x 2^(n - k) doubles.
 * Errors: as sv_apply_circuit. */
svq_status sv_grad(svq_state st, const svq_gate *gates, int m, const double *theta,
                   int n_theta, const svq_pauli *terms, int n_terms, svq_sched sched,
                   double *energy_host, double *energy_dev, double *grad_host,
                   double *grad_dev, svq_stats *stats);

/* Parameter-shift gradient, the comparison method for sv_grad: every
 * parametric gate j of parameter p is re-evaluated with its angle shifted,
 * E(+-s) by a full QSU and EVC from psi0 under the given schedule, and
 * dE/dtheta_p = sum_j scale_j sum_s w_s [E(a_j + s) - E(a_j - s)].
 * rule SVQ_SHIFT_EXACT: s = pi/2, w = 1/2 for the one-frequency kinds (RX,
 * RY, RZ, CPHASE); for GIVENS (frequencies 1/2 and 1) the two-frequency rule
 * s = pi/2, 3pi/2 with w = (sqrt2 + 1)/(4 sqrt2), -(sqrt2 - 1)/(4 sqrt2)
 * (Wierichs et al., Quantum 6, 677 (2022)).  SVQ_SHIFT_TWO_TERM applies the
 * one-frequency rule to every gate (two evaluations per gate, exact only for
 * one-frequency gates).  The combination runs on the device in FP64.
 * The handle's state is psi0 and is handed back; psi0 is kept in a second
 * state buffer.  energy_host (nullable) adds one unshifted evaluation;
 * *n_evals_out (nullable) receives the number of evaluations.  Errors: as
 * sv_grad, EINVAL for another rule. */
enum { SVQ_SHIFT_EXACT = 0, SVQ_SHIFT_TWO_TERM = 1 };
svq_status sv_param_shift_grad(svq_state st, const svq_gate *gates, int m, const double *theta,
                               int n_theta, const svq_pauli *terms, int n_terms, svq_sched sched,
                               int rule, double *energy_host, double *grad_host, double *grad_dev,
                               int *n_evals_out, svq_stats *stats);

/* Host-only planning (no GPU needed), for inspection and tests.
 * Circuit: order_out[m] = gate index at each schedule position,
 * qr_tile_out[m] = QR tile of each position, pass_out[m] = gate pass of each
 * position, local_out[m] = bit mask of the local qubit set M(g(x)) at each
 * position; *n_qr_out = reorderings (eq. n_qr), *n_pass_out = gate passes.
 * Paulis (x-mask groups): order_out[nt], qr_tile_out[nt], pass_out[nt],
 * local_out[nt] likewise.  tile_k/low_bits/reg_bits = 0 pick defaults. */
svq_status sv_plan_circuit(int n, int g, const svq_gate *gates, int m, svq_sched sched,
                           int tile_k, int32_t *order_out, int32_t *qr_tile_out,
                           int32_t *pass_out, uint64_t *local_out, int32_t *n_qr_out,
                           int32_t *n_pass_out);
/* The same plan as sv_plan_circuit (initial layout pos[q] = q, low bits from
 * SVQ_LOW_BITS, default 4) as the JSON text of sv_plan_dump, including each
 * gate pass's store positions "tile_bits_out".  Host only.  Errors: EINVAL,
 * ESHAPE (cap too small). */
svq_status sv_plan_circuit_json(int n, int g, const svq_gate *gates, int m, svq_sched sched,
                                int tile_k, char *json_buf, size_t cap, size_t *len_out);
svq_status sv_plan_paulis(int n, int g, const svq_pauli *terms, int n_terms, svq_sched sched,
                          int tile_k, int32_t *order_out, int32_t *qr_tile_out,
                          int32_t *pass_out, uint64_t *local_out, int32_t *n_qr_out,
                          int32_t *n_pass_out);

/* ---- batched VQE -------------------------------------------------------
 * Many independent instances (each its own circuit, angles and Hamiltonian,
 * qubit counts 10..26, all qubits local: no emulated global qubits, so no
 * reordering) evaluated by one HIP graph that is captured once and replayed
 * per call.  Every stage of an instance (psi0, each gate pass, each H|psi>
 * pass, <psi|H psi>, each reverse adjoint pass, the final FP64 sums) is cut
 * into 2^10-amplitude tiles, grouped into items (a range of tiles each).  The
 * graph holds one launch per (stage level, item type): the k-th stages of all
 * instances that are gate passes run in one launch, and so on; stream order
 * carries the dependencies.  Instances of at most 13 qubits instead run
 * whole in one workgroup each, psi and lambda held in LDS (2 x 2^n complex64;
 * any Pauli string, no tiling), in one launch beside the others.  With
 * SVQ_BATCH_PERSISTENT=1 in the environment
 * at creation the graph instead holds one persistent launch whose single-wave
 * blocks pull items from a device queue and wait, with a bounded spin, for
 * the instance's previous stage.
 * The plans are built once (the schedule reused across VQE iterations,
 * Section "Scheduling time"); only the angles change per call. */
typedef struct svq_batch_s *svq_batch;

/* gates[i][0..m[i]), theta of instance i has n_theta[i] entries, terms[i]
 * [0..n_terms[i]), psi0[i] the initial basis state.  low_bits = 0 picks the
 * tuned value.  The library allocates the state arena (two states per
 * instance) and tables.  Errors: EINVAL (shapes, gates, masks), EUNSUP (an
 * instance above 13 qubits with a Pauli string whose X/Y sites fit no
 * 2^10-amplitude tile), ENOMEM, EHIP. */
svq_status sv_batch_create(int n_inst, const int32_t *n_qubits, const svq_gate *const *gates,
                           const int32_t *m, const int32_t *n_theta,
                           const svq_pauli *const *terms, const int32_t *n_terms,
                           const uint64_t *psi0, int low_bits, void *stream, svq_batch *out);

/* Run all instances for the given angles (theta[i] has n_theta[i] entries).
 * energies_host[n_inst] and grads_host[sum n_theta] (concatenated in instance
 * order) receive E and dE/dtheta; latency_ms_host[n_inst] (nullable) the
 * time from kernel start to the completion of each instance (device clock).
 * Synchronises the stream.  In the persistent form a dependency wait that
 * exceeds its bound returns EHIP and poisons the batch. */
svq_status sv_batch_run(svq_batch b, const double *const *theta, double *energies_host,
                        double *grads_host, double *latency_ms_host);
/* Shape of a batch: the algorithmic HBM bytes of one run (one write of every
 * psi, a read and a write of psi per gate pass, of psi and lambda per reverse
 * pass, a read of psi and a write of lambda per H|psi> pass plus a read of
 * lambda when it accumulates, and a read of both for the dot), the number of
 * stages and of work items.  All outputs nullable.  Errors: EINVAL. */
svq_status sv_batch_info(svq_batch b, double *bytes_per_run, int32_t *n_stages, int32_t *n_items);
svq_status sv_batch_destroy(svq_batch b);

/* ---- measured tuning ----------------------------------------------------
 * The tile width k and the count c of forced low (coalescing) bits decide how
 * many passes a circuit needs and how fast each pass streams.  These calls
 * time candidate plans with HIP events on the handle's stream (one warm run,
 * one timed run each), keep the fastest for the handle's size class
 * (n, g, dtype) and use it whenever tile_k = 0 / low_bits = 0.  They overwrite
 * the state.  k_out/c_out/ms_out (nullable) receive the winner. */
svq_status sv_tune_circuit(svq_state st, const svq_gate *gates, int m, const double *theta,
                           int n_theta, svq_sched sched, int *k_out, int *c_out, double *ms_out);
svq_status sv_tune_paulis(svq_state st, const svq_pauli *terms, int n_terms, int *k_out,
                          int *c_out, double *ms_out);
/* Batch: tries items per stage (chunks), low bits, and the size class from
 * which instances run their gate and H|psi> passes on 2^12-amplitude tiles
 * (12, 16, 20 qubits, or none); arguments as sv_batch_create plus the angles;
 * the winner is used by later sv_batch_create calls with low_bits = 0. */
svq_status sv_batch_tune(int n_inst, const int32_t *n_qubits, const svq_gate *const *gates,
                         const int32_t *m, const int32_t *n_theta, const svq_pauli *const *terms,
                         const int32_t *n_terms, const uint64_t *psi0, const double *const *theta,
                         void *stream, int *chunks_out, int *low_bits_out, double *ms_out);
/* Persist / restore the tuned table (text: kind n g dtype k c ms per line).
 * Kinds: 0 gate pass and 1 Pauli pass (k = tile bits, c = low coalescing
 * bits, per qubit count n, global bits g and dtype 0 = complex64 /
 * 1 = complex128); 2 batch (k = items per stage, c = low bits); 3 batch size
 * classes (k = smallest qubit count run on 2^12-amplitude tiles, c = 0).
 * sv_tune_load skips lines of other kinds or out-of-range values. */
svq_status sv_tune_save(const char *path);
svq_status sv_tune_load(const char *path);

/* Per-launch timing.  sv_profile(st, 1) clears the record and brackets every
 * later kernel launch of the handle with HIP events on its stream;
 * sv_profile(st, 0) stops recording.  sv_profile_read synchronises the stream
 * and returns the number of recorded launches of one kind and their summed
 * duration in ms.  Kinds: 0 gate pass, 1 QR pass, 2 EVC pass, 3 H|psi> pass,
 * 4 adjoint pass, 5 Pauli-as-gate pass of the QSU-based EVC. */
svq_status sv_profile(svq_state st, int enable);
svq_status sv_profile_read(svq_state st, int kind, int *count, double *total_ms);

/* Host-only level-1 planning over arbitrary operators given by target masks
 * (e.g. one 4-qubit GateFabric block per operator, the granularity of the
 * paper's figures).  method: 0 ad hoc (eager) in breadth-first order,
 * 1 flat tiling (Algs. 1-3), 2 hierarchical tiling (Algs. 4-5) with n_intra
 * intra qubits, 3 ad hoc in the given order (the index order of the
 * QSU-based EVC, a Pauli string's X/Y sites as targets); fill_highest
 * selects Alg. 3's boundary fill (0: lowest free qubit, as the text says).
 * An empty target set (a diagonal string) is allowed and never moves qubits.
 * order_out[m] = operator index per schedule position, local_out[m] = the
 * local set M(g(x)) per position, intra_out[m] (hierarchical, nullable) the
 * intra set per position; *n_qr_out counts changes of M (eq. n_qr) and
 * *n_inter_out (hierarchical) the QRs that change the inter qubits. */
svq_status sv_plan_ops(int n, int n_local, const uint64_t *targets, int m, int method,
                       int n_intra, int fill_highest, int32_t *order_out, uint64_t *local_out,
                       uint64_t *intra_out, int32_t *n_qr_out, int32_t *n_inter_out);

/* eq. comm_cost: Cost = w_intra * N_intra + w_inter * N_inter over the
 * reorders of a level-1 plan (method as in sv_plan_ops) on a cluster whose
 * g = n - n_local PE bits split into n_intra intra-node bits (positions
 * n_local .. n_local + n_intra - 1) and g - n_intra inter-node bits
 * (fig:qr_types: an inter reorder moves a qubit on or off an inter-node bit).
 * Hierarchical tiling (method 2) tracks Q_intra and Q_inter itself.  For the
 * other methods the paper does not say where evicted qubits go: each reorder
 * swaps its incoming qubits with its outgoing ones pairwise in ascending order
 * of position (the ad hoc method's own pairing), and counts as inter when an
 * incoming qubit leaves an inter position.  Weights
 * must be finite and non-negative (the paper takes w_inter tens of times
 * w_intra).  Host only.  Errors: EINVAL. */
svq_status sv_qr_cost(int n, int n_local, int n_intra, const uint64_t *targets, int m, int method,
                      int fill_highest, double w_intra, double w_inter, int32_t *n_intra_out,
                      int32_t *n_inter_out, double *cost_out);

/* The data movement of one gate pass alone: the gate-pass kernel run over
 * the handle's state with no gates, on tiles of the k local physical bit
 * positions tile_bits[0..k) (ascending; a real pass has the c lowest ones
 * among them), with nphase phases whose register bits alternate so that
 * each of the nphase - 1 phase changes is a full LDS transpose.  It reads
 * and writes every amplitude once and leaves the state unchanged.  One warm
 * launch, then reps timed launches (HIP events on the handle's stream);
 * *ms_out receives the average per launch.  The ceiling against which the
 * gate pass's HBM fraction is judged.  Errors: EINVAL, EHIP. */
svq_status sv_pass_ceiling(svq_state st, const int32_t *tile_bits, int k, int nphase, int reps,
                           double *ms_out);

/* A plain streaming copy of device memory (16-byte accesses, asynchronous on
 * the stream): the reference against which pass bandwidths and the HBM
 * traffic counters are calibrated.  bytes must be a multiple of 16; the
 * ranges must not overlap.  Errors: EINVAL, EHIP. */
svq_status sv_device_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *sv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SVQ_C_ABI_H */
