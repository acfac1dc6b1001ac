"""Host logic of the C-ABI library (no GPU needed): exported symbols, and the
C++ planner against the oracle's schedules written from Algs. 1-3, 6 and the
ad hoc method."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import schedule as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2410_04252_amd as P
    return P


def test_library_exports_every_declared_symbol(P):
    hdr = open(os.path.join(ROOT, "include", "svq.h")).read()
    declared = set(re.findall(r"\b(sv_[a-z_]+)\s*\(", hdr))
    assert declared, "no declarations found"
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [name for name in sorted(declared) if not hasattr(lib, name)]
    assert not missing, missing
    assert set(P.EXPORTS) <= declared


def _targets(circ):
    return [tuple(q for q in gt[1]) for gt in circ.gates]


def _merge_tiles(tiles):
    out = []
    for QL, G in tiles:
        if out and out[-1][0] == QL:
            out[-1] = (QL, out[-1][1] + list(G))
        else:
            out.append((QL, list(G)))
    return out


def _mask(qs):
    return sum(1 << q for q in qs)


CIRCUITS = [
    ("hea12", lambda: W.hea(12, 4, 4253), 2),
    ("fabric16", lambda: W.fabric(16, 8, 3), 3),
    ("fabric20", lambda: W.fabric(20, 20, 4), 5),
    ("fabric24", lambda: W.fabric(24, 12, 5), 5),
    ("random14", lambda: W.random_circuit(14, 150, 6), 4),
    ("random18", lambda: W.random_circuit(18, 300, 7), 6),
]


@pytest.mark.parametrize("name,make,g", CIRCUITS, ids=[c[0] for c in CIRCUITS])
def test_lazy_plan_matches_flat_tiling(P, name, make, g):
    circ = make()
    n = circ.n
    nL = n - g
    plan = P.sv_plan_circuit(n, g, circ.gates, P.LAZY, 0)
    order, M, tiles = S.flat_tiling(n, _targets(circ), nL)
    assert plan["n_qr"] == S.n_qr(M, nL)
    # every gate runs under the local set the paper's algorithm assigns it
    want = {op: _mask(m) for op, m in zip(order, M)}
    got = dict(zip(plan["order"], plan["local"]))
    assert got == want
    # QR tiles hold the same gate sets
    merged = _merge_tiles(tiles)
    by_tile = {}
    for op, t in zip(plan["order"], plan["qr_tile"]):
        by_tile.setdefault(t, set()).add(op)
    assert [set(G) for _, G in merged] == [by_tile[t] for t in sorted(by_tile)]


@pytest.mark.parametrize("name,make,g", CIRCUITS, ids=[c[0] for c in CIRCUITS])
def test_eager_plan_matches_ad_hoc(P, name, make, g):
    circ = make()
    n = circ.n
    nL = n - g
    plan = P.sv_plan_circuit(n, g, circ.gates, P.EAGER, 0)
    order, M, qrs = S.ad_hoc(n, _targets(circ), nL)
    assert plan["n_qr"] == len(qrs) == S.n_qr(M, nL)
    want = {op: _mask(m) for op, m in zip(order, M)}
    got = dict(zip(plan["order"], plan["local"]))
    assert got == want


@pytest.mark.parametrize("sched", [0, 1])
@pytest.mark.parametrize("name,make,g", CIRCUITS, ids=[c[0] for c in CIRCUITS])
def test_execution_order_is_valid(P, name, make, g, sched):
    """The executed order (after packing into passes) keeps every dependency
    (constraint C1) and runs every gate with its qubits local (C2)."""
    circ = make()
    n = circ.n
    plan = P.sv_plan_circuit(n, g, circ.gates, sched, 0)
    order = plan["order"]
    assert sorted(order) == list(range(len(circ.gates)))
    pos = {op: i for i, op in enumerate(order)}
    last = {}
    for i, gt in enumerate(circ.gates):
        for q in gt[1]:
            if q in last:
                assert pos[last[q]] < pos[i]
            last[q] = i
    for op, loc in zip(order, plan["local"]):
        assert _mask(circ.gates[op][1]) & ~loc == 0
        assert bin(loc).count("1") == n - g
    # passes are contiguous runs in the executed order
    ps = plan["pass_"]
    assert all(ps[i] <= ps[i + 1] for i in range(len(ps) - 1))


HAMS = [
    ("jw12", lambda: W.jw_terms(12, 150, 8), 2),
    ("jw14", lambda: W.jw_terms(14, 300, 9), 3),
    ("jw16", lambda: W.jw_terms(16, 400, 10), 4),
]


@pytest.mark.parametrize("name,make,g", HAMS, ids=[h[0] for h in HAMS])
def test_lazy_pauli_plan_matches_alg6(P, name, make, g):
    ham = make()
    n = ham.n
    nL = n - g
    plan = P.sv_plan_paulis(n, g, ham, P.LAZY, 0)
    sup = [S.pauli_support(int(x), int(z), True) for x, z in zip(ham.x, ham.z)]
    tiles = S.tiling_pauli(n, sup, nL)
    assert plan["n_qr"] == S.tiles_n_qr(tiles, nL)
    # each flip-mask group is evaluated under the local set Alg. 6 gives it
    xs = [int(v) for v in ham.x]
    groups = list(dict.fromkeys(xs))
    term_tile = {}
    for QL, G in tiles:
        for t in G:
            term_tile[t] = _mask(QL)
    got = dict(zip(plan["order"], plan["local"]))
    for gi, x in enumerate(groups):
        ts = [t for t in range(len(xs)) if xs[t] == x]
        assert {term_tile[t] for t in ts} == {got[gi]}


@pytest.mark.parametrize("name,make,g", HAMS, ids=[h[0] for h in HAMS])
def test_eager_pauli_plan_counts(P, name, make, g):
    """Index-order evaluation with ad hoc reordering on the X/Y supports."""
    ham = make()
    n = ham.n
    nL = n - g
    plan = P.sv_plan_paulis(n, g, ham, P.EAGER, 0)
    targets = [tuple(q for q in range(n) if (int(x) >> q) & 1) for x in ham.x]
    _, M, qrs = S.ad_hoc(n, targets, nL, order=list(range(len(targets))))
    assert plan["n_qr"] == len(qrs)


@pytest.mark.parametrize("cfg", ["hea12", "fabric28", "fabric30", "fabric32"])
def test_lazy_needs_fewer_reorders_than_eager(P, cfg):
    c = W.config(cfg)
    circ, g = c["circuit"], c["g"]
    lazy = P.sv_plan_circuit(circ.n, g, circ.gates, P.LAZY, 0)["n_qr"]
    eager = P.sv_plan_circuit(circ.n, g, circ.gates, P.EAGER, 0)["n_qr"]
    _, M, _ = S.flat_tiling(circ.n, _targets(circ), circ.n - g)
    _, M2, _ = S.ad_hoc(circ.n, _targets(circ), circ.n - g)
    assert lazy == S.n_qr(M, circ.n - g)
    assert eager == S.n_qr(M2, circ.n - g)
    assert lazy < eager


def test_plan_errors(P):
    good = [("RY", (0,), 0)]
    with pytest.raises(P.SvqError) as e:
        P.sv_plan_circuit(12, 2, [("RY", (12,), 0)], P.LAZY)
    assert e.value.status == -1
    with pytest.raises(P.SvqError):
        P.sv_plan_circuit(12, 2, [("CNOT", (3, 3), -1)], P.LAZY)
    with pytest.raises(P.SvqError):
        P.sv_plan_circuit(0, 0, good, P.LAZY)
    with pytest.raises(P.SvqError):
        P.sv_plan_circuit(12, 8, good, P.LAZY)        # fewer than 8 local qubits
    bad = W.Hamiltonian(12, np.array([1 << 12], dtype=np.uint64), np.array([0], dtype=np.uint64),
                        np.array([1.0]))
    with pytest.raises(P.SvqError):
        P.sv_plan_paulis(12, 2, bad, P.LAZY)
    nan = W.Hamiltonian(12, np.array([1], dtype=np.uint64), np.array([0], dtype=np.uint64),
                        np.array([float("nan")]))
    with pytest.raises(P.SvqError):
        P.sv_plan_paulis(12, 2, nan, P.LAZY)


def test_create_rejects_bad_shapes_before_touching_the_gpu(P):
    for n, g in ((0, 0), (35, 3), (12, 12), (12, 5), (40, 2)):
        with pytest.raises(P.SvqError) as e:
            P.sv_create(n, g, P.C64)
        assert e.value.status == -1
    with pytest.raises(P.SvqError):
        P.sv_create(12, 2, 7)


def test_plan_time_is_small(P):
    """Scheduling cost stays negligible (Section "Scheduling time"): well under
    a second for the 32-qubit, 10^4-term configuration."""
    import time
    c = W.config("fabric32")
    t0 = time.time()
    P.sv_plan_circuit(32, 6, c["circuit"].gates, P.LAZY)
    t1 = time.time()
    P.sv_plan_paulis(32, 6, c["ham"], P.LAZY)
    t2 = time.time()
    assert t1 - t0 < 0.05
    assert t2 - t1 < 5.0


@pytest.mark.parametrize("name,n,g,nt,seed", [("jw20", 20, 4, 600, 61), ("jw24", 24, 5, 1500, 62),
                                              ("rand14", 14, 3, 200, 63)])
def test_pauli_passes_cover_every_group_once(P, name, n, g, nt, seed):
    """Level 2 of the Pauli plan (our packing of flip-mask groups into
    passes) evaluates every group exactly once, in passes whose order never
    goes back, and every group's flip mask lies in its pass's local set."""
    ham = W.jw_terms(n, nt, seed) if name.startswith("jw") else W.random_pauli(n, nt, seed)
    plan = P.sv_plan_paulis(n, g, ham, P.LAZY, 0)
    groups = list(dict.fromkeys(int(x) for x in ham.x))
    order = plan["order"]
    assert sorted(order) == list(range(len(order)))
    assert len(order) <= len(groups)
    ps = plan["pass_"]
    assert all(ps[i] <= ps[i + 1] for i in range(len(ps) - 1))
    for gi, loc in zip(order, plan["local"]):
        assert groups[gi] & ~loc == 0
