"""Pins of the oracle's schedules (Algs. 1-6, ad hoc) against the paper's
worked examples and against invariants that any valid schedule satisfies."""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import schedule as S
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def fabric_block_ops(n, layers):
    return W.block_ops(n, layers)


def _fig_circuit():
    ops = []
    for _ in range(6):
        ops += [tuple(range(4 * j, 4 * j + 4)) for j in range(4)]
        ops += [tuple(range(4 * j + 2, 4 * j + 6)) for j in range(3)]
    return ops


def test_qsu_qct_depths():
    """fig:qsu_qct: U0>U2, U1>U2, U2>U3, U2>U4 give depths 0,0,1,2,2 (targets
    chosen to realise exactly these direct dependencies)."""
    targets = [(0, 1), (2, 3), (1, 2), (1,), (2,)]
    assert S.depths(targets) == [0, 0, 1, 2, 2]
    order = S.depth_order(targets)
    assert order.index(2) > order.index(0) and order.index(2) > order.index(1)
    assert order.index(3) > order.index(2) and order.index(4) > order.index(2)


def test_flat_tiling_worked_example():
    gold = json.load(open(os.path.join(GOLD, "flat_tiling_fig.json")))
    ps = gold["paper_states"]
    ops = _fig_circuit()
    order, M, tiles = S.flat_tiling(gold["n"], ops, gold["n_L"])
    allq = set(range(gold["n"]))
    assert S.n_qr(M, gold["n_L"]) == ps["qr_count"]
    a, b = ps["same_mapping_positions"]
    assert M[a] == M[b]
    i, j = ps["first_qr_between"]
    assert M[i] != M[j] and sorted(allq - M[j]) == ps["global_after_first_qr"]
    i, j = ps["second_qr_between"]
    assert M[i] != M[j] and sorted(allq - M[j]) == ps["global_after_second_qr_reading"]


def test_hierarchical_tiling_worked_example():
    gold = json.load(open(os.path.join(GOLD, "hierarchical_tiling_fig.json")))
    ops = _fig_circuit()
    _, _, _, ev = S.hierarchical_tiling(gold["n"], ops, gold["n_L"], gold["n_intra"], fill="highest")
    got = [{"before": p, "kind": k, "intra": sorted(a), "inter": sorted(b)} for p, k, a, b in ev]
    assert got == gold["paper_states"]["events"]
    inter = sum(e["kind"] == "inter" for e in got)
    intra = sum(e["kind"] == "intra" for e in got)
    assert (inter, intra) == (2, 3)       # "two inter-QRs and three intra-QRs"


def _evc_strings():
    # Z0 Y1 X3 Y4 Z7 ; X2 Z6 X7 ; X0 Y3 Z4 X6
    def mk(spec):
        x = z = 0
        for tok in spec.split():
            ch, q = tok[0], int(tok[1:])
            if ch in "XY":
                x |= 1 << q
            if ch in "YZ":
                z |= 1 << q
        return x, z
    gold = json.load(open(os.path.join(GOLD, "evc_fig.json")))
    return gold, [mk(s) for s in gold["strings"]]


def test_evc_worked_example():
    gold, strs = _evc_strings()
    n, nL = gold["n"], gold["n_L"]
    ps = gold["paper_states"]
    full = [S.pauli_support(x, z, False) for x, z in strs]
    assert [q for q in range(n) if full[1] >> q & 1] == ps["T(P1)"]
    tiles = S.tiling_pauli(n, full, nL)
    assert S.tiles_n_qr(tiles, nL) == ps["efficient_order_qrs"]
    assert [i for _, G in tiles for i in G] == ps["efficient_order"]
    _, M, _ = S.ad_hoc(n, [tuple(q for q in range(n) if s >> q & 1) for s in full], nL,
                       order=[0, 1, 2])
    assert S.n_qr(M, nL) == ps["index_order_qrs"]
    diag = [S.pauli_support(x, z, True) for x, z in strs]
    assert [sorted(q for q in range(n) if s >> q & 1) for s in diag] == [[1, 3, 4], [2, 7], [0, 3, 6]]
    tiles_d = S.tiling_pauli(n, diag, nL)
    assert len(tiles_d) <= len(tiles)


def _valid(n, targets, nL, order, M):
    assert sorted(order) == list(range(len(targets)))          # each op once
    pos = {op: i for i, op in enumerate(order)}
    last = {}
    for i, t in enumerate(targets):                             # C1
        for q in t:
            if q in last:
                assert pos[last[q]] < pos[i]
            last[q] = i
    for x, op in enumerate(order):                               # C2
        assert set(targets[op]) <= M[x]
        assert len(M[x]) == nL


@settings(max_examples=60, deadline=None)
@given(st.integers(6, 14), st.integers(1, 4), st.integers(0, 10_000), st.integers(1, 60))
def test_flat_and_adhoc_invariants(n, g, seed, m):
    rng = np.random.default_rng(seed)
    nL = n - g
    targets = []
    for _ in range(m):
        a = int(rng.integers(1, 3))
        targets.append(tuple(int(v) for v in rng.choice(n, size=a, replace=False)))
    order, M, tiles = S.flat_tiling(n, targets, nL)
    _valid(n, targets, nL, order, M)
    assert S.n_qr(M, nL) <= len(tiles)
    o2, M2, _ = S.ad_hoc(n, targets, nL)
    _valid(n, targets, nL, o2, M2)


def test_qr_trend_with_n():
    """Section 'Quantum state update' (evaluation): with 4n GateFabric layers on
    a fixed PE count, flat tiling needs fewer QRs as n grows while the ad hoc
    method needs more."""
    g = 5
    flat, adhoc = [], []
    for n in (16, 20, 24):
        ops = fabric_block_ops(n, 4 * n)
        _, M, _ = S.flat_tiling(n, ops, n - g)
        _, M2, _ = S.ad_hoc(n, ops, n - g)
        flat.append(S.n_qr(M, n - g))
        adhoc.append(S.n_qr(M2, n - g))
    assert flat[0] >= flat[1] >= flat[2]
    assert adhoc[0] < adhoc[1] < adhoc[2]
    assert all(f < a for f, a in zip(flat, adhoc))


def test_tiling_pauli_is_maximal_first():
    """Alg. 6 picks, at every step, a local set covering the most remaining
    strings (checked by brute force over all sets)."""
    from itertools import combinations
    n, nL = 8, 5
    rng = np.random.default_rng(2)
    sup = [int(sum(1 << int(q) for q in rng.choice(n, size=int(rng.integers(1, 4)), replace=False)))
           for _ in range(25)]
    tiles = S.tiling_pauli(n, sup, nL)
    remain = set(range(len(sup)))
    for QL, G in tiles:
        best = max(sum(1 for i in remain if sup[i] & ~sum(1 << q for q in c) == 0)
                   for c in combinations(range(n), nL))
        assert len(G) == best
        remain -= set(G)
    assert not remain
