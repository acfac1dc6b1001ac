"""Benchmark of the state-vector hot path on one MI355X.

One step = one VQE energy evaluation of the 30-qubit fabric-style workload
(complex64, g = 5 emulated global qubits, 16 brick layers = 336 gates, 2000
Jordan-Wigner-like Pauli strings): prepare psi0, QSU under the lazy-QR
schedule, EVC under the lazy-QR schedule.  Inputs are synthetic and seeded
(workloads.config("fabric30")); the state lives in HBM for the whole run.

Printed: one JSON line.  ``value`` is QSU gates/s (gates per second of the QSU
part of the timed steps, measured with HIP events on the library's stream);
the EVC terms/s, the adjoint-vs-parameter-shift gradient rates (24-qubit
400-parameter workload), lazy/eager QR counts, the roofline of the gate pass
and the CPU-oracle baseline are extra keys of the same line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QSU gates/s + HBM GB/s frac at 30q; EVC terms/s; adjoint vs param-shift grad/s"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gate_pass_fabric30.json")
TRAFFIC_FILE_C128 = os.path.join(ROOT, "profiles", "traffic_gate_pass_fabric30_c128.json")


ELEM = {"c64": "float", "c128": "double"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "svq_dev.hpp", "plan.cpp"):
        with open(os.path.join(ROOT, "paper_2410_04252_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted_traffic(path, kernel, workload):
    """Per-launch HBM bytes of the gate pass from the committed counter
    summary, or None when it was taken on another workload, another kernel
    instance or older kernel sources."""
    if workload != "fabric30" or not os.path.exists(path):
        return None
    try:
        tf = json.load(open(path))
    except (OSError, ValueError):
        return None
    if tf.get("source_hash") != kernel_source_hash() or kernel not in tf.get("instances", []):
        return None
    return tf.get("bytes_per_launch")


def pass_ceiling(P, st, gate_pass_ms_per_run):
    """Every gate pass of the handle's last circuit plan run again without its
    gates (sv_pass_ceiling: the same tile bits and phase count, so the same
    loads, stores and LDS transposes): the data movement alone, per run."""
    plan = st.plan_dump()
    tot, npass = 0.0, 0
    for s in plan.get("steps", []):
        if s["type"] != "gate_pass":
            continue
        tot += P.sv_pass_ceiling(st.h, s["tile_bits"], s["phases"], reps=3)
        npass += 1
    return dict(empty_pass_ms_per_run=round(tot, 3), gate_pass_ms_per_run=round(gate_pass_ms_per_run, 3),
                passes=npass, frac_of_ceiling=round(tot / gate_pass_ms_per_run, 4) if gate_pass_ms_per_run else None)


def measure_main(P, W, torch, args):
    cfg = W.config(args.workload)
    circ, ham, g = cfg["circuit"], cfg["ham"], cfg["g"]
    n = circ.n
    dtype = args.dtype or cfg["dtype"]
    esz = 8 if dtype == "c64" else 16
    S = (1 << n) * esz
    st = P.State(n, g, dtype)
    h = st.h
    gates_c = P.gates_array(circ.gates)
    terms_c = P.paulis_array(ham)
    m, nt = len(circ.gates), len(ham.coef)
    theta = circ.theta
    e_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step(prof_events=None):
        P.sv_set_basis(h, circ.psi0_index)
        if prof_events:
            prof_events[0].record(stream)
        s1 = P.sv_apply_circuit(h, gates_c, m, theta, len(theta), P.LAZY, args.tile_k)
        if prof_events:
            prof_events[1].record(stream)
        _, s2 = P.sv_expectation(h, terms_c, nt, P.LAZY, energy_dev=e_dev.data_ptr(),
                                 want_host=False)
        if prof_events:
            prof_events[2].record(stream)
        return s1, s2

    log(f"[bench] workload {args.workload}: n={n} g={g} {dtype} gates={m} terms={nt}")
    tuned = None
    if args.tune:
        kq, cq, msq = st.tune(circ)
        ke, ce, mse = st.tune_paulis(ham)
        tuned = dict(gate_k=kq, gate_c=cq, qsu_ms=msq, evc_k=ke, evc_c=ce, evc_ms=mse)
        log(f"[bench] tuned: gate pass k={kq} c={cq} ({msq:.2f} ms), EVC k={ke} c={ce} ({mse:.2f} ms)")
    t0 = time.time()
    s1, s2 = step()          # plans are built (and cached) here
    torch.cuda.synchronize()
    log(f"[bench] first step (incl. planning {s1.ms_plan:.1f} + {s2.ms_plan:.1f} ms): "
        f"{time.time() - t0:.2f} s")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    P.sv_profile(h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    qsu_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    evc_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    n_gp, t_gp = P.sv_profile_read(h, P.PROF_GATE)
    n_qr, t_qr = P.sv_profile_read(h, P.PROF_QR)
    n_ev, t_ev = P.sv_profile_read(h, P.PROF_EVC)
    P.sv_profile(h, 0)
    energy = float(e_dev.item())
    log(f"[bench] step {ms_step:.2f} ms: QSU {qsu_ms:.2f} ms ({s1.n_gate_passes} passes, "
        f"{s1.n_qr} QR), EVC {evc_ms:.2f} ms ({s2.n_evc_passes} passes, {s2.n_qr} QR), E={energy:.8f}")
    gp_avg_ms = t_gp / max(1, n_gp)
    gp_bytes = 2.0 * S                     # one read + one write of the state per launch
    achieved = gp_bytes / (gp_avg_ms * 1e-3) / 1e9
    evc_roof = evc_roofline(n, nt, t_ev / args.steps, dtype)
    # the same passes without their gates (after the timed region)
    ceiling = None
    if not args.no_ceiling:
        P.sv_set_basis(h, circ.psi0_index)
        P.sv_apply_circuit(h, gates_c, m, theta, len(theta), P.LAZY, args.tile_k)
        ceiling = pass_ceiling(P, st, t_gp / args.steps)
        log(f"[bench] the {ceiling['passes']} gate passes without gates: {ceiling['empty_pass_ms_per_run']:.2f} ms "
            f"per run against {ceiling['gate_pass_ms_per_run']:.2f} ms with them")
    if args.no_eager:
        st.close()
        return dict(
            n=n, g=g, dtype=dtype, m=m, nt=nt, S=S, ms_step=ms_step, qsu_ms=qsu_ms, evc_ms=evc_ms,
            energy=energy, qsu_evc=None, tuned=tuned,
            qsu=dict(gates_per_s=m / (qsu_ms * 1e-3), ms=qsu_ms, gate_passes=s1.n_gate_passes,
                     qr_lazy=s1.n_qr, plan_ms=s1.ms_plan,
                     algorithmic_gbs=s1.bytes / (qsu_ms * 1e-3) / 1e9,
                     hbm_frac=s1.bytes / (qsu_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     gate_pass_avg_ms=gp_avg_ms, qr_pass_avg_ms=t_qr / max(1, n_qr)),
            evc=dict(terms_per_s=nt / (evc_ms * 1e-3), ms=evc_ms, evc_passes=s2.n_evc_passes,
                     groups=s2.n_groups, qr_lazy=s2.n_qr, evc_pass_avg_ms=t_ev / max(1, n_ev),
                     plan_ms=s2.ms_plan, roofline=evc_roof),
            roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                          kernel="k_gate_pass<%s,%d,4,false,true>" % (ELEM[dtype], s1.tile_k or 12),
                          bytes_per_launch=gp_bytes, launches=n_gp, avg_ms=gp_avg_ms,
                          ceiling=ceiling))
    # eager comparison (one run, not part of the timed steps)
    P.sv_set_basis(h, circ.psi0_index)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    se = P.sv_apply_circuit(h, gates_c, m, theta, len(theta), P.EAGER, args.tile_k)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    eager_first_ms = (tb - ta) * 1e3
    P.sv_set_basis(h, circ.psi0_index)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    se = P.sv_apply_circuit(h, gates_c, m, theta, len(theta), P.EAGER, args.tile_k)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - ta) * 1e3
    _, se2 = P.sv_expectation(h, terms_c, nt, P.EAGER)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    P.sv_set_basis(h, circ.psi0_index)
    P.sv_apply_circuit(h, gates_c, m, theta, len(theta), P.LAZY, args.tile_k)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    _, se2 = P.sv_expectation(h, terms_c, nt, P.EAGER)
    torch.cuda.synchronize()
    evc_eager_ms = (time.perf_counter() - ta) * 1e3
    log(f"[bench] eager QSU {eager_ms:.2f} ms ({se.n_qr} QR, {se.n_gate_passes} passes); "
        f"eager EVC {evc_eager_ms:.2f} ms ({se2.n_qr} QR)")
    qsu_evc = measure_qsu_evc(P, W, torch, st, ham, args) if args.qsu_terms > 0 else None
    st.close()
    out = dict(
        n=n, g=g, dtype=dtype, m=m, nt=nt, S=S, ms_step=ms_step, qsu_ms=qsu_ms, evc_ms=evc_ms,
        energy=energy,
        qsu=dict(gates_per_s=m / (qsu_ms * 1e-3), ms=qsu_ms, gate_passes=s1.n_gate_passes,
                 qr_lazy=s1.n_qr, qr_eager=se.n_qr, eager_ms=eager_ms,
                 eager_gate_passes=se.n_gate_passes, plan_ms=s1.ms_plan,
                 algorithmic_gbs=s1.bytes / (qsu_ms * 1e-3) / 1e9,
                 hbm_frac=s1.bytes / (qsu_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 gate_pass_avg_ms=gp_avg_ms, qr_pass_avg_ms=t_qr / max(1, n_qr)),
        evc=dict(terms_per_s=nt / (evc_ms * 1e-3), ms=evc_ms, evc_passes=s2.n_evc_passes,
                 groups=s2.n_groups, qr_lazy=s2.n_qr, qr_eager=se2.n_qr, eager_ms=evc_eager_ms,
                 evc_pass_avg_ms=t_ev / max(1, n_ev), plan_ms=s2.ms_plan,
                 read_gbs=s2.n_evc_passes * S / (max(1e-9, t_ev / max(1, args.steps)) * 1e-3) / 1e9,
                 roofline=evc_roof),
        qsu_evc=qsu_evc, tuned=tuned,
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                      kernel="k_gate_pass<%s,%d,4,false,true>" % (ELEM[dtype], s1.tile_k or 12),
                      bytes_per_launch=gp_bytes, launches=n_gp, avg_ms=gp_avg_ms, ceiling=ceiling),
    )
    return out


FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def evc_roofline(n, nt, evc_pass_ms_per_step, dtype):
    """ALU roofline of the Pauli passes.  Algorithmic work: the direct
    evaluation of eq. evc, each Pauli string over its 2^(n-1) amplitude pairs
    (i, i xor x) with one complex product conj(psi_{i^x}) psi_i (6 flops) and
    one signed accumulation (2 flops): 4 * 2^n flops per string.  The kernel
    shares the products of a flip-mask group and the signs of its strings
    (Walsh-Hadamard), so it executes fewer."""
    flops = 4.0 * (1 << n) * nt
    achieved = flops / (evc_pass_ms_per_step * 1e-3) / 1e12
    peak = FP32_PEAK_TFLOPS if dtype == "c64" else FP64_PEAK_TFLOPS
    return dict(bound="alu", achieved=round(achieved, 2), peak=peak, unit="TFLOP/s",
                frac=round(achieved / peak, 4), traffic=None, kernel="k_evc_pass",
                flops_per_step=flops, pass_ms_per_step=evc_pass_ms_per_step)


def measure_copy_gbs(P, torch, nbytes=8 << 30):
    """Achievable device bandwidth: the library's plain streaming copy of
    8 GiB (bytes read + written over the kernel time, best of three)."""
    a = torch.empty(nbytes // 8, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    stream = torch.cuda.current_stream()
    P.sv_device_copy(a.data_ptr(), b.data_ptr(), nbytes, stream)
    best = 1e30
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.sv_device_copy(a.data_ptr(), b.data_ptr(), nbytes, stream)
        e1.record(stream)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def qr_trend(P, W):
    """The paper's trend configuration on the host planner: GateFabric with
    4n layers at 30 qubits, one operator per 4-qubit block, g = 5."""
    ops = W.block_ops(30, 120)
    return dict(n=30, layers=120, block_ops=len(ops),
                flat=P.sv_plan_ops(30, 25, ops, P.PLAN_FLAT)["n_qr"],
                adhoc=P.sv_plan_ops(30, 25, ops, P.PLAN_ADHOC)["n_qr"])


def comm_cost_sweep(P, W):
    """eq. comm_cost on the host planner: GateFabric with 4n layers (block
    operators) on 32 PEs, g = 5 with 3 intra-node and 2 inter-node PE bits,
    for flat and hierarchical tiling, at w_inter / w_intra = 10 and 30."""
    out = {}
    for n in (30, 36):
        ops = W.block_ops(n, 4 * n)
        row = {}
        for name, method in (("flat", P.PLAN_FLAT), ("hierarchical", P.PLAN_HIERARCHICAL)):
            ni, ne, c10 = P.sv_qr_cost(n, n - 5, 3, ops, method, 1.0, 10.0)
            c30 = P.sv_qr_cost(n, n - 5, 3, ops, method, 1.0, 30.0)[2]
            row[name] = dict(n_intra=ni, n_inter=ne, cost_w10=c10, cost_w30=c30)
        out[str(n)] = row
    return out


def measure_qsu_evc(P, W, torch, st, ham, args):
    """The QSU-based comparison method on the first qsu_terms strings (index
    order): each string applied as a gate into psi' (one elementwise pass per
    string), ad hoc reorders, then one <psi|psi'>.  Its reorder count over all
    strings comes from the planner."""
    n, g = ham.n, st.g
    k = min(args.qsu_terms, len(ham.coef))
    sub = W.Hamiltonian(n, ham.x[:k], ham.z[:k], ham.coef[:k])
    st.expectation_qsu(sub)                     # warm
    torch.cuda.synchronize()
    P.sv_profile(st.h, 1)
    t0 = time.perf_counter()
    _, sq = st.expectation_qsu(sub)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    npg, tpg = P.sv_profile_read(st.h, P.PROF_PAULI_GATE)
    P.sv_profile(st.h, 0)
    sup = [tuple(q for q in range(n) if (int(x) >> q) & 1) for x in ham.x]
    nqr_all = P.sv_plan_ops(n, n - g, sup, P.PLAN_ADHOC_INDEX)["n_qr"]
    S = (1 << n) * (8 if st.dtype == P.C64 else 16)
    pg_avg = tpg / max(1, npg)
    log(f"[bench] QSU-based EVC: {k} strings in {ms:.1f} ms ({k / ms * 1e3:.0f} terms/s), "
        f"{sq.n_qr} QR; all {len(ham.coef)} strings need {nqr_all} QR")
    return dict(terms_sampled=k, ms=ms, terms_per_s=k / (ms * 1e-3), qr_sample=sq.n_qr,
                qr_all_terms=nqr_all, pauli_gate_avg_ms=pg_avg,
                pauli_gate_gbs=3.0 * S / (pg_avg * 1e-3) / 1e9 if pg_avg > 0 else None)


def measure_c128(P, W, torch, args):
    """The FP64 path on the same 30-qubit workload (complex128, 16 GiB): lazy
    QSU and EVC, two timed repetitions after one warm run."""
    cfg = W.config(args.workload)
    circ, ham, g = cfg["circuit"], cfg["ham"], cfg["g"]
    n = circ.n
    st = P.State(n, g, "c128")
    h = st.h
    gc, tc = P.gates_array(circ.gates), P.paulis_array(ham)
    m, nt = len(circ.gates), len(ham.coef)

    def once():
        P.sv_set_basis(h, circ.psi0_index)
        s1 = P.sv_apply_circuit(h, gc, m, circ.theta, len(circ.theta), P.LAZY, 0)
        e, s2 = P.sv_expectation(h, tc, nt, P.LAZY)
        return s1, s2, e

    once()
    torch.cuda.synchronize()
    P.sv_profile(h, 1)
    reps = 2
    for _ in range(reps):
        s1, s2, e = once()
    n_gp, t_gp = P.sv_profile_read(h, P.PROF_GATE)
    n_ev, t_ev = P.sv_profile_read(h, P.PROF_EVC)
    n_qr, t_qr = P.sv_profile_read(h, P.PROF_QR)
    P.sv_profile(h, 0)
    ceiling = None
    if not args.no_ceiling:
        P.sv_set_basis(h, circ.psi0_index)
        P.sv_apply_circuit(h, gc, m, circ.theta, len(circ.theta), P.LAZY, 0)
        ceiling = pass_ceiling(P, st, t_gp / reps)
    st.close()
    S = (1 << n) * 16
    gp_avg = t_gp / max(1, n_gp)
    qr_avg = t_qr / max(1, n_qr)
    qsu_ms = (t_gp + qr_avg * s1.n_qr * reps) / reps
    gbs = 2 * S / (gp_avg * 1e-3) / 1e9
    log(f"[bench] c128: gate pass {gp_avg:.2f} ms ({gbs:.0f} GB/s), "
        f"{s1.n_gate_passes} passes; EVC passes {t_ev / reps:.1f} ms; E={e:.12f}")
    kname = "k_gate_pass<double,%d,4,false,true>" % (s1.tile_k or 12)
    traffic = counted_traffic(TRAFFIC_FILE_C128, kname, args.workload)
    return dict(workload=args.workload, dtype="c128", gate_passes=s1.n_gate_passes, tile_k=s1.tile_k,
                qr_lazy=s1.n_qr, gate_pass_avg_ms=gp_avg, qr_pass_avg_ms=qr_avg,
                qsu_ms_kernels=qsu_ms, qsu_gates_per_s_kernels=m / (qsu_ms * 1e-3),
                evc_pass_ms=t_ev / reps, evc_terms_per_s_kernels=nt / (t_ev / reps * 1e-3),
                energy=e,
                roofline=dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=round(gbs / HBM_PEAK_GBS, 4), traffic=traffic,
                              kernel=kname, bytes_per_launch=2 * S, launches=n_gp, avg_ms=gp_avg,
                              ceiling=ceiling),
                evc_roofline=evc_roofline(n, nt, t_ev / reps, "c128"))


def measure_grad(P, W, torch, args):
    """cfg: 24 qubits, 400 parameters, 1000 strings, complex64.  The adjoint
    gradient (sv_grad) against the GPU parameter-shift driver
    (sv_param_shift_grad) under the exact rules (two evaluations per CPHASE,
    four per GIVENS) and under the nominal two evaluations per parameter."""
    import numpy as np
    cfg = W.config("grad24")
    circ, ham = cfg["circuit"], cfg["ham"]
    n = circ.n
    g = cfg["g"]
    st = P.State(n, g, "c64")
    h = st.h
    gates_c = P.gates_array(circ.gates)
    terms_c = P.paulis_array(ham)
    m, nt, npar = len(circ.gates), len(ham.coef), len(circ.theta)
    theta = circ.theta.copy()
    S = (1 << n) * 8
    log(f"[bench] gradient workload grad24: n={n} params={npar} gates={m} terms={nt}")
    # adjoint
    P.sv_set_basis(h, circ.psi0_index)
    P.sv_grad(h, gates_c, m, theta, npar, terms_c, nt, P.LAZY)
    torch.cuda.synchronize()
    reps = 3
    P.sv_profile(h, 1)
    t0 = time.perf_counter()
    for _ in range(reps):
        P.sv_set_basis(h, circ.psi0_index)
        e_adj, g_adj, sg = P.sv_grad(h, gates_c, m, theta, npar, terms_c, nt, P.LAZY)
    torch.cuda.synchronize()
    adj_ms = (time.perf_counter() - t0) * 1e3 / reps
    n_adj, t_adj = P.sv_profile_read(h, P.PROF_ADJ)
    P.sv_profile(h, 0)
    adj_avg = t_adj / max(1, n_adj)
    adj_gbs = 4 * S / (adj_avg * 1e-3) / 1e9
    # parameter shift on the GPU, exact rules and the nominal two-term rule
    P.sv_set_basis(h, circ.psi0_index)
    out = {}
    for name, rule in (("exact", P.SHIFT_EXACT), ("two_term", P.SHIFT_TWO_TERM)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, g_ps, nev, _ = P.sv_param_shift_grad(h, gates_c, m, theta, npar, terms_c, nt, P.LAZY,
                                                rule, want_energy=False)
        torch.cuda.synchronize()
        out[name] = ((time.perf_counter() - t0) * 1e3, nev, g_ps)
    ps_ms, nev_exact, g_ps = out["exact"]
    nominal_ms, nev_two, _ = out["two_term"]
    rel = float(np.linalg.norm(g_adj - g_ps) / max(1e-300, np.linalg.norm(g_ps)))
    st.close()
    log(f"[bench] adjoint {adj_ms:.2f} ms/grad ({sg.bytes / (adj_ms * 1e-3) / 1e9:.0f} GB/s of "
        f"algorithmic traffic; reverse pass {adj_avg:.2f} ms, {adj_gbs:.0f} GB/s); "
        f"param-shift {ps_ms:.1f} ms/grad ({nev_exact} evaluations), nominal {nominal_ms:.1f} ms "
        f"({nev_two}); rel diff {rel:.2e}")
    return dict(workload="grad24", n=n, g=g, params=npar, terms=nt, adjoint_ms=adj_ms,
                adjoint_grad_per_s=1e3 / adj_ms, adjoint_bytes=sg.bytes,
                adjoint_gbs=sg.bytes / (adj_ms * 1e-3) / 1e9,
                adjoint_roofline=dict(bound="hbm", achieved=round(adj_gbs, 1), peak=HBM_PEAK_GBS,
                                      unit="GB/s", frac=round(adj_gbs / HBM_PEAK_GBS, 4),
                                      kernel="k_gate_pass<float,%d,4,true,true>" % sg.tile_k,
                                      bytes_per_launch=4 * S, launches=n_adj, avg_ms=adj_avg),
                param_shift_ms=ps_ms, param_shift_grad_per_s=1e3 / ps_ms,
                param_shift_evaluations=nev_exact,
                param_shift_nominal_ms=nominal_ms, param_shift_nominal_evaluations=nev_two,
                speedup=ps_ms / adj_ms, speedup_vs_nominal=nominal_ms / adj_ms,
                rel_diff_adjoint_vs_shift=rel)


def _qsu_evc_leg(P, torch, circ, ham, g, dtype, reps=2, with_eager=True, tile_k=0):
    """Lazy QSU and EVC of one workload: kernel times from the library's
    per-launch events, pass and QR counts; eager QR counts from the planner."""
    n = circ.n
    S = (1 << n) * (8 if dtype == "c64" else 16)
    st = P.State(n, g, dtype)
    h = st.h
    gc, tc = P.gates_array(circ.gates), P.paulis_array(ham)
    m, nt = len(circ.gates), len(ham.coef)

    def once():
        P.sv_set_basis(h, circ.psi0_index)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s1 = P.sv_apply_circuit(h, gc, m, circ.theta, len(circ.theta), P.LAZY, tile_k)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e, s2 = P.sv_expectation(h, tc, nt, P.LAZY)
        t2 = time.perf_counter()
        return s1, s2, e, (t1 - t0) * 1e3, (t2 - t1) * 1e3

    once()
    P.sv_profile(h, 1)
    res = [once() for _ in range(reps)]
    n_gp, t_gp = P.sv_profile_read(h, P.PROF_GATE)
    n_qr, t_qr = P.sv_profile_read(h, P.PROF_QR)
    n_ev, t_ev = P.sv_profile_read(h, P.PROF_EVC)
    P.sv_profile(h, 0)
    st.close()
    s1, s2, e = res[-1][0], res[-1][1], res[-1][2]
    qsu_ms = min(r[3] for r in res)
    evc_ms = min(r[4] for r in res)
    gp_avg = t_gp / max(1, n_gp)
    out = dict(n=n, g=g, dtype=dtype, gates=m, terms=nt, energy=e,
               qsu_ms=qsu_ms, gates_per_s=m / (qsu_ms * 1e-3), gate_passes=s1.n_gate_passes,
               tile_k=s1.tile_k, qr_lazy=s1.n_qr, gate_pass_avg_ms=gp_avg,
               gate_pass_gbs=2 * S / (gp_avg * 1e-3) / 1e9,
               gate_pass_hbm_frac=2 * S / (gp_avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
               qr_pass_avg_ms=t_qr / max(1, n_qr) if n_qr else None,
               evc_ms=evc_ms, terms_per_s=nt / (evc_ms * 1e-3), evc_passes=s2.n_evc_passes,
               evc_qr_lazy=s2.n_qr, evc_pass_avg_ms=t_ev / max(1, n_ev),
               evc_roofline=evc_roofline(n, nt, t_ev / reps, dtype))
    if with_eager:
        out["qr_eager"] = P.sv_plan_circuit(n, g, circ.gates, P.EAGER, s1.tile_k)["n_qr"]
        out["evc_qr_eager"] = P.sv_plan_paulis(n, g, ham, P.EAGER)["n_qr"]
    return out


def measure_legs(P, W, torch, args):
    """The other configurations: the 12-qubit hardware-efficient ansatz
    (complex128, lazy and eager, energy against the oracle), the 28-qubit
    fabric (complex64) and the 32-qubit fabric (complex64 and complex128,
    10^4 strings), whose energy is checked against the host oracle at reduced
    depth (2 brick layers, 16 of the strings)."""
    import numpy as np
    import oracle
    legs = {}
    c = W.config("hea12")
    e_ref = oracle.energy(c["circuit"], c["ham"])
    hea = {}
    for name, sched in (("lazy", P.LAZY), ("eager", P.EAGER)):
        st = P.State(12, c["g"], "c128")
        st.set_basis(0)
        s1 = st.apply(c["circuit"], sched=sched, tile_k=c["k"])
        e, s2 = st.expectation(c["ham"], sched=sched)
        st.close()
        hea[name] = dict(qr=s1.n_qr, gate_passes=s1.n_gate_passes, evc_qr=s2.n_qr,
                         energy_abs_err=abs(e - e_ref))
    legs["hea12"] = dict(n=12, g=c["g"], dtype="c128", tile_k=c["k"], energy_ref=e_ref, **hea)
    log(f"[bench] hea12 c128: QR lazy {hea['lazy']['qr']} eager {hea['eager']['qr']}; "
        f"|dE| {hea['lazy']['energy_abs_err']:.1e}")
    c = W.config("fabric28")
    legs["fabric28"] = _qsu_evc_leg(P, torch, c["circuit"], c["ham"], c["g"], "c64")
    L = legs["fabric28"]
    log(f"[bench] fabric28 c64: QSU {L['qsu_ms']:.1f} ms ({L['gates_per_s']:.0f} gates/s, "
        f"{L['gate_passes']} passes, QR {L['qr_lazy']} vs eager {L['qr_eager']}), gate pass "
        f"{L['gate_pass_gbs']:.0f} GB/s; EVC {L['evc_ms']:.1f} ms ({L['terms_per_s']:.0f} terms/s)")
    if args.no_fabric32:
        return legs
    c = W.config("fabric32")
    circ, ham, g = c["circuit"], c["ham"], c["g"]
    f32 = {}
    for dtype in ("c64", "c128"):
        f32[dtype] = _qsu_evc_leg(P, torch, circ, ham, g, dtype, reps=1)
        L = f32[dtype]
        log(f"[bench] fabric32 {dtype}: QSU {L['qsu_ms']:.1f} ms ({L['gate_passes']} passes, QR "
            f"{L['qr_lazy']} vs eager {L['qr_eager']}), gate pass {L['gate_pass_gbs']:.0f} GB/s; "
            f"EVC {L['evc_ms']:.0f} ms ({L['terms_per_s']:.0f} terms/s, QR {L['evc_qr_lazy']} vs "
            f"{L['evc_qr_eager']})")
    # reduced depth against the oracle (2 layers of the same seeded ansatz).
    # Two layers move the 10 electrons of psi0 only near the boundary of the
    # occupied orbitals, so the check uses strings whose sites all lie there
    # (qubits 4..15), 8 diagonal and 8 with X/Y sites, drawn from the 10^4.
    short = W.fabric(32, 2, W.SEED_BASE + 3)
    rng = np.random.default_rng(3232)
    band = ((1 << 16) - 1) & ~((1 << 4) - 1)
    inside = [i for i in range(len(ham.coef))
              if (int(ham.x[i]) | int(ham.z[i])) & ~band == 0]
    diag = [i for i in inside if int(ham.x[i]) == 0]
    offd = [i for i in inside if int(ham.x[i]) != 0]
    pick = np.sort(np.concatenate([rng.choice(diag, size=min(8, len(diag)), replace=False),
                                   rng.choice(offd, size=min(8, len(offd)), replace=False)]))
    sub = W.Hamiltonian(32, ham.x[pick], ham.z[pick], ham.coef[pick])
    e_gpu = {}
    for dtype in ("c64", "c128"):
        st = P.State(32, g, dtype)
        st.set_basis(short.psi0_index)
        st.apply(short)
        e_gpu[dtype], _ = st.expectation(sub)
        st.close()
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    log("[bench] fabric32 reduced depth: host oracle (2 layers, 2^32 complex128)")
    psi = oracle.basis_state(32, short.psi0_index)
    oracle.apply_circuit_inplace(psi, short.gates, short.theta)
    e_ref = oracle.expectation(psi, sub)
    del psi
    scale = max(abs(e_ref), 1e-2 * float(np.abs(sub.coef).sum()))
    for dtype in ("c64", "c128"):
        f32[dtype]["reduced_depth_check"] = dict(
            layers=2, strings=len(pick), energy=e_gpu[dtype], energy_ref=e_ref,
            abs_err=abs(e_gpu[dtype] - e_ref), rel_err=abs(e_gpu[dtype] - e_ref) / scale)
    log(f"[bench] fabric32 reduced depth: E_ref={e_ref:.12f}, |dE| c64 "
        f"{abs(e_gpu['c64'] - e_ref):.1e}, c128 {abs(e_gpu['c128'] - e_ref):.1e} "
        f"({time.perf_counter() - t0:.0f} s on the host)")
    legs["fabric32"] = f32
    return legs


def measure_batch(P, W, torch, args):
    """256 independent instances (n uniform in 10..22, 6 fabric layers, 200
    JW-like terms): QSU + EVC + adjoint gradient of all of them in one
    captured graph (one launch per stage level and item type), against a
    one-at-a-time loop."""
    import numpy as np
    inst = [(d["circuit"], d["ham"]) for d in W.batch_instances()]
    ninst = len(inst)
    log(f"[bench] batch: {ninst} instances, n in [{min(c.n for c, _ in inst)}, "
        f"{max(c.n for c, _ in inst)}]")
    tuned = None
    if args.tune:
        tb = P.Batch(inst)
        ch, lb, tms = tb.tune()
        tb.close()
        tuned = dict(chunks=ch, low_bits=lb, ms=tms)
        log(f"[bench] batch tuned: {ch} items per stage, {lb} low bits ({tms:.1f} ms)")
    t0 = time.perf_counter()
    b = P.Batch(inst)
    create_ms = (time.perf_counter() - t0) * 1e3
    batch_bytes, n_stages, n_items = b.info()
    b.run()                       # first run captures the graph
    torch.cuda.synchronize()
    reps = 5
    times, lats = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        _, _, lat = b.run()
        times.append((time.perf_counter() - t0) * 1e3)
        lats.append(lat)
    b.close()
    run_ms = float(np.median(times))
    lat = lats[int(np.argsort(times)[reps // 2])]
    # one at a time: one handle per instance, sv_grad each, host-synchronised
    states = [P.State(c.n, 0, "c64") for c, _ in inst]
    gcs = [P.gates_array(c.gates) for c, _ in inst]
    tcs = [P.paulis_array(h) for _, h in inst]

    def loop():
        done = []
        t0 = time.perf_counter()
        for (c, h), st, gc, tc in zip(inst, states, gcs, tcs):
            P.sv_set_basis(st.h, c.psi0_index)
            P.sv_grad(st.h, gc, len(c.gates), c.theta, c.n_params, tc, len(h.coef), P.LAZY)
            done.append((time.perf_counter() - t0) * 1e3)
        return done

    loop()
    torch.cuda.synchronize()
    done = loop()
    for st in states:
        st.close()
    loop_ms = done[-1]
    log(f"[bench] batch {run_ms:.2f} ms ({ninst / run_ms * 1e3:.0f} inst/s, p50 {np.percentile(lat, 50):.2f} "
        f"p99 {np.percentile(lat, 99):.2f} ms); one at a time {loop_ms:.1f} ms")
    gbs = batch_bytes / (run_ms * 1e-3) / 1e9
    ns = np.array([c.n for c, _ in inst])
    lat_small = float(np.percentile(lat[ns <= 13], 50)) if np.any(ns <= 13) else None
    lat_large = float(np.percentile(lat[ns >= 16], 50)) if np.any(ns >= 16) else None
    log(f"[bench] batch algorithmic traffic {batch_bytes / 1e9:.1f} GB per run: {gbs:.0f} GB/s "
        f"({gbs / HBM_PEAK_GBS * 100:.1f}% of HBM peak), {n_stages} stages, {n_items} items")
    return dict(workload="batch256", instances=ninst, create_ms=create_ms, tuned=tuned,
                mode="level-synchronous launches in one graph", batch_ms=run_ms,
                algorithmic_bytes=batch_bytes, algorithmic_gbs=gbs, hbm_frac=gbs / HBM_PEAK_GBS,
                stages=n_stages, items=n_items, instances_per_s=ninst / run_ms * 1e3,
                latency_p50_ms=float(np.percentile(lat, 50)),
                latency_p50_ms_lds_instances=lat_small, latency_p50_ms_wide_instances=lat_large,
                latency_p99_ms=float(np.percentile(lat, 99)),
                loop_ms=loop_ms, loop_instances_per_s=ninst / loop_ms * 1e3,
                loop_latency_p50_ms=float(np.percentile(done, 50)),
                loop_latency_p99_ms=float(np.percentile(done, 99)),
                speedup=loop_ms / run_ms)


def measure_cpu(W, main, budget_s):
    import numpy as np
    import oracle
    cfg = W.config(main["workload"])
    circ, ham = cfg["circuit"], cfg["ham"]
    n = circ.n
    log(f"[bench] cpu baseline: oracle on {oracle.threads()} threads, n={n} complex128")
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[circ.psi0_index] = 1.0
    done, t_q = 0, 0.0
    while done < len(circ.gates) and t_q < budget_s * 0.6:
        t0 = time.perf_counter()
        oracle.apply_circuit_inplace(psi, circ.gates[done:done + 1], circ.theta)
        t_q += time.perf_counter() - t0
        done += 1
    terms_done, t_e = 0, 0.0
    while terms_done < len(ham.coef) and t_e < budget_s * 0.4:
        one = W.Hamiltonian(n, ham.x[terms_done:terms_done + 1], ham.z[terms_done:terms_done + 1],
                            ham.coef[terms_done:terms_done + 1])
        t0 = time.perf_counter()
        oracle.expectation(psi, one)
        t_e += time.perf_counter() - t0
        terms_done += 1
    del psi
    cpu_model, ram_gib = None, None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    ram_gib = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return dict(value=done / t_q, unit="gates/s", cores=oracle.threads(), kind="oracle",
                cpu_model=cpu_model, ram_gib=ram_gib,
                sample=f"first {done} gates of the {n}-qubit circuit on a 2^{n} complex128 state "
                       f"({t_q:.1f} s); EVC: {terms_done} Pauli strings ({t_e:.1f} s)",
                evc_terms_per_s=terms_done / t_e)


def _pmc_rows(d, counter):
    """(kernel name, value) of every dispatch in a rocprofv3 --pmc CSV tree."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((r.get("Kernel_Name", ""), float(r["Counter_Value"])))
    return rows


def _avg(rows, pat):
    v = [x for k, x in rows if pat in k]
    return (sum(v) / len(v) if v else None), len(v)


def hbm_bytes(rd_dir, wr_dir, pat):
    """HBM bytes per dispatch of the kernels whose name contains pat, from the
    L2-to-fabric request counters summed over all 16 channels of all 8 XCDs:
    a read request moves a 128-byte line (32 bytes when flagged 32B), a write
    request 64 bytes (32 when not flagged 64B).  Runs: rd_dir with
    TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum, wr_dir with TCC_EA0_WRREQ_sum
    TCC_EA0_WRREQ_64B_sum."""
    rq, n1 = _avg(_pmc_rows(rd_dir, "TCC_EA0_RDREQ_sum"), pat)
    r32, _ = _avg(_pmc_rows(rd_dir, "TCC_EA0_RDREQ_32B_sum"), pat)
    wq, n2 = _avg(_pmc_rows(wr_dir, "TCC_EA0_WRREQ_sum"), pat)
    w64, _ = _avg(_pmc_rows(wr_dir, "TCC_EA0_WRREQ_64B_sum"), pat)
    rd = 128.0 * (rq - r32) + 32.0 * r32
    wr = 64.0 * w64 + 32.0 * (wq - w64)
    return rd, wr, (n1, n2)


def ingest_pmc(rd_dir, wr_dir, copy_rd_dir, copy_wr_dir, dtype="c64", tile_k=0):
    """Per-launch HBM traffic of the gate pass from the request counters,
    checked on a plain copy of known size (1 GiB read, 1 GiB written per
    launch), which must read 1.0 of its bytes."""
    rd, wr, n = hbm_bytes(rd_dir, wr_dir, "k_gate_pass")
    crd, cwr, _ = hbm_bytes(copy_rd_dir, copy_wr_dir, "k_copy")
    names = sorted({k.split("(")[0].replace("void svq::", "").replace(" ", "")
                    for k, _ in _pmc_rows(rd_dir, "TCC_EA0_RDREQ_sum") if "k_gate_pass" in k})
    S = (1 << 30) * (8 if dtype == "c64" else 16)
    out = dict(kernel="k_gate_pass (fabric30, lazy, %s)" % dtype, source_hash=kernel_source_hash(),
               method="TCC_EA0_RDREQ_sum x 128 B (32 B requests x 32), TCC_EA0_WRREQ_64B_sum x 64 B "
                      "(others x 32), summed over 16 channels x 8 XCDs",
               instances=names, read_bytes_per_launch=rd, write_bytes_per_launch=wr, launches=list(n),
               copy_read_ratio=crd / float(1 << 30), copy_write_ratio=cwr / float(1 << 30),
               bytes_per_launch=rd + wr, algorithmic_bytes_per_launch=2 * S,
               ratio_to_algorithmic=(rd + wr) / (2 * S))
    path = TRAFFIC_FILE if dtype == "c64" else TRAFFIC_FILE_C128
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fabric30")
    ap.add_argument("--dtype", default=None)
    ap.add_argument("--tile-k", type=int, default=0)
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-c128", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the hea12 / fabric28 / fabric32 configuration legs")
    ap.add_argument("--no-fabric32", action="store_true", help="skip the 32-qubit legs")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip re-running the gate passes without gates (profiling runs)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--tune", action="store_true",
                    help="run the measured tuner on the workload before timing")
    ap.add_argument("--tune-save", default=None, help="write the tuned table to this file")
    ap.add_argument("--no-eager", action="store_true",
                    help="skip the eager-schedule and QSU-based comparisons (profiling runs)")
    ap.add_argument("--qsu-terms", type=int, default=64,
                    help="Pauli strings timed with the QSU-based comparison method (0: skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only three plain 1 GiB device copies (traffic-counter calibration)")
    ap.add_argument("--ingest-pmc", nargs=4, metavar=("RD_DIR", "WR_DIR", "COPY_RD_DIR",
                                                       "COPY_WR_DIR"),
                    help="turn rocprofv3 --pmc request-counter runs of this benchmark and of "
                         "--copy-probe into the per-launch HBM traffic of the gate pass")
    args = ap.parse_args()
    if args.ingest_pmc:
        ingest_pmc(*args.ingest_pmc, dtype=args.dtype or "c64", tile_k=args.tile_k)
        return
    if args.gpus != 1:
        print("bench.py: measures one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2410_04252_amd as P
    import workloads as W
    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.zeros((1 << 30) // 8, dtype=torch.complex64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            P.sv_device_copy(a.data_ptr(), b.data_ptr(), 1 << 30, torch.cuda.current_stream())
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "launches": 3}))
        return
    res = measure_main(P, W, torch, args)
    res["workload"] = args.workload
    res["roofline"]["traffic"] = counted_traffic(
        TRAFFIC_FILE if res["dtype"] == "c64" else TRAFFIC_FILE_C128,
        res["roofline"]["kernel"], args.workload)
    if not args.no_eager:
        copy_gbs = measure_copy_gbs(P, torch)
        res["roofline"]["copy_gbs"] = round(copy_gbs, 1)
        res["roofline"]["frac_of_copy"] = round(res["roofline"]["achieved"] / copy_gbs, 4)
        log(f"[bench] plain device copy {copy_gbs:.0f} GB/s; gate pass at "
            f"{res['roofline']['frac_of_copy'] * 100:.1f}% of it")
        res["qsu"]["qr_trend_30q_120_layers"] = qr_trend(P, W)
        res["qsu"]["comm_cost_32pe"] = comm_cost_sweep(P, W)
    c128 = None if (args.no_c128 or res["dtype"] != "c64") else measure_c128(P, W, torch, args)
    grad = None if args.no_grad else measure_grad(P, W, torch, args)
    legs = None if args.no_legs else measure_legs(P, W, torch, args)
    batch = None if args.no_batch else measure_batch(P, W, torch, args)
    if args.tune_save:
        P.sv_tune_save(args.tune_save)
    cpu = None if args.no_cpu else measure_cpu(W, res, args.cpu_budget)
    line = {
        "metric": METRIC,
        "value": round(res["qsu"]["gates_per_s"], 2),
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if res["dtype"] == "c64" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_qubits": res["n"], "g_global": res["g"],
                   "state": res["dtype"], "gates": res["m"], "pauli_terms": res["nt"],
                   "ansatz": "fabric-style (Givens, Givens, CPHASE blocks), 16 brick layers",
                   "hamiltonian": "Jordan-Wigner-like, coefficients N(0, 0.1)"},
        "qsu": res["qsu"],
        "evc": res["evc"],
        "qsu_evc": res["qsu_evc"],
        "tuned": res["tuned"],
        "c128": c128,
        "grad": grad,
        "batch": batch,
        "legs": legs,
        "energy": res["energy"],
        "roofline": res["roofline"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
