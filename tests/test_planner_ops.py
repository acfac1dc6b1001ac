"""Level-1 planning over arbitrary operators (host only): the product's flat,
ad hoc and hierarchical tilings against the paper's worked examples and the
oracle, and the QR-count trend of the paper's evaluation."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import schedule as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def P():
    import paper_2410_04252_amd as P
    return P


def _fig_ops():
    ops = []
    for _ in range(6):
        ops += [tuple(range(4 * j, 4 * j + 4)) for j in range(4)]
        ops += [tuple(range(4 * j + 2, 4 * j + 6)) for j in range(3)]
    return ops


def _mask(qs):
    return sum(1 << q for q in qs)


def test_flat_tiling_figure(P):
    gold = json.load(open(os.path.join(GOLD, "flat_tiling_fig.json")))
    ps = gold["paper_states"]
    r = P.sv_plan_ops(gold["n"], gold["n_L"], _fig_ops(), P.PLAN_FLAT)
    allm = (1 << gold["n"]) - 1
    M = r["local"]
    assert r["n_qr"] == ps["qr_count"]
    a, b = ps["same_mapping_positions"]
    assert M[a] == M[b]
    i, j = ps["first_qr_between"]
    assert M[i] != M[j]
    assert [q for q in range(16) if (allm & ~M[j]) >> q & 1] == ps["global_after_first_qr"]
    i, j = ps["second_qr_between"]
    assert [q for q in range(16) if (allm & ~M[j]) >> q & 1] == ps["global_after_second_qr_reading"]


def test_hierarchical_tiling_figure(P):
    gold = json.load(open(os.path.join(GOLD, "hierarchical_tiling_fig.json")))
    n = gold["n"]
    r = P.sv_plan_ops(n, gold["n_L"], _fig_ops(), P.PLAN_HIERARCHICAL, gold["n_intra"],
                      fill_highest=True)
    events = []
    allm = (1 << n) - 1
    for x in range(1, len(r["order"])):
        if (r["local"][x], r["intra"][x]) != (r["local"][x - 1], r["intra"][x - 1]):
            inter_new = allm & ~r["local"][x] & ~r["intra"][x]
            inter_old = allm & ~r["local"][x - 1] & ~r["intra"][x - 1]
            events.append({"before": x, "kind": "intra" if inter_new == inter_old else "inter",
                           "intra": [q for q in range(n) if r["intra"][x] >> q & 1],
                           "inter": [q for q in range(n) if inter_new >> q & 1]})
    assert events == gold["paper_states"]["events"]
    assert r["n_inter"] == 2 and r["n_qr"] == 5


@pytest.mark.parametrize("fill", [False, True])
@pytest.mark.parametrize("seed", range(6))
def test_hierarchical_matches_oracle(P, seed, fill):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(10, 17))
    nL = n - int(rng.integers(3, 6))
    n_intra = int(rng.integers(1, n - nL))
    ops = [tuple(int(v) for v in rng.choice(n, size=int(rng.integers(1, 5)), replace=False))
           for _ in range(int(rng.integers(20, 90)))]
    order, M, tiles, events = S.hierarchical_tiling(n, ops, nL, n_intra,
                                                    fill="highest" if fill else "lowest")
    r = P.sv_plan_ops(n, nL, ops, P.PLAN_HIERARCHICAL, n_intra, fill_highest=fill)
    assert r["order"] == order
    assert r["local"] == [_mask(m) for m in M]
    assert r["n_inter"] == sum(1 for e in events if e[1] == "inter")


@pytest.mark.parametrize("seed", range(6))
def test_flat_and_adhoc_ops_match_oracle(P, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(8, 18))
    nL = n - int(rng.integers(1, 5))
    ops = [tuple(int(v) for v in rng.choice(n, size=int(rng.integers(1, 5)), replace=False))
           for _ in range(int(rng.integers(10, 120)))]
    order, M, _ = S.flat_tiling(n, ops, nL)
    r = P.sv_plan_ops(n, nL, ops, P.PLAN_FLAT)
    assert r["order"] == order and r["local"] == [_mask(m) for m in M]
    assert r["n_qr"] == S.n_qr(M, nL)
    order, M, _ = S.ad_hoc(n, ops, nL)
    r = P.sv_plan_ops(n, nL, ops, P.PLAN_ADHOC)
    assert r["order"] == order and r["local"] == [_mask(m) for m in M]


def test_qr_count_sweep_block_level(P):
    """GateFabric with 4n layers on 32 PEs (g = 5), one operator per 4-qubit
    block as in the paper's evaluation: flat tiling needs fewer QRs as n grows
    and far fewer than the ad hoc method, whose count grows with n."""
    g = 5
    flat, adhoc = {}, {}
    for n in range(16, 37, 2):
        ops = W.block_ops(n, 4 * n)
        flat[n] = P.sv_plan_ops(n, n - g, ops, P.PLAN_FLAT)["n_qr"]
        adhoc[n] = P.sv_plan_ops(n, n - g, ops, P.PLAN_ADHOC)["n_qr"]
        if n <= 22:
            _, M, _ = S.flat_tiling(n, ops, n - g)
            _, M2, _ = S.ad_hoc(n, ops, n - g)
            assert flat[n] == S.n_qr(M, n - g) and adhoc[n] == S.n_qr(M2, n - g)
    ns = sorted(flat)
    assert all(flat[a] >= flat[b] for a, b in zip(ns, ns[1:]))
    assert all(adhoc[a] < adhoc[b] for a, b in zip(ns, ns[1:]))
    ratio = [adhoc[n] / flat[n] for n in ns]
    assert all(a < b for a, b in zip(ratio, ratio[1:]))
    assert all(flat[n] < adhoc[n] for n in ns)


def test_hierarchical_trades_inter_for_intra(P):
    """Section 'Hierarchical tiling' (evaluation): with a two-level network the
    hierarchical method has more QRs in total but fewer inter QRs than flat
    tiling, all of whose QRs change inter qubits at these sizes."""
    g, n_intra = 5, 3
    for n in (24, 28, 30):
        ops = W.block_ops(n, 4 * n)
        fl = P.sv_plan_ops(n, n - g, ops, P.PLAN_FLAT)["n_qr"]
        h = P.sv_plan_ops(n, n - g, ops, P.PLAN_HIERARCHICAL, n_intra, fill_highest=True)
        assert h["n_qr"] >= fl
        assert h["n_inter"] < fl


def test_evc_qr_sweep_alg6_vs_qsu_based(P):
    """EVC (Section 'Evaluation', EVC part): Alg. 6 with diagonalization needs
    far fewer QRs than the QSU-based method (index order, each Pauli string a
    gate on its whole support, ad hoc reordering), and the gap widens with the
    term count.  The QSU-based method makes each string's X/Y sites local (Z
    sites are a diagonal phase); its index-order ad hoc plan equals the
    oracle's."""
    g = 5
    ratios = []
    for n, nt in ((20, 400), (24, 1000), (28, 2000), (30, 2000)):
        ham = W.jw_terms(n, nt, 4000 + n)
        sup = [tuple(q for q in range(n) if (int(x) >> q) & 1) for x in ham.x]
        qsu = P.sv_plan_ops(n, n - g, sup, P.PLAN_ADHOC_INDEX)
        lazy = P.sv_plan_paulis(n, g, ham, P.LAZY)["n_qr"]
        if n <= 24:
            order, M, qrs = S.ad_hoc(n, sup, n - g, order=list(range(len(sup))))
            assert qsu["order"] == order and qsu["local"] == [_mask(m) for m in M]
            assert qsu["n_qr"] == len(qrs)
        assert lazy < qsu["n_qr"]
        ratios.append(qsu["n_qr"] / max(1, lazy))
    assert ratios[-1] > 20


# ---- eq. comm_cost: intra and inter reorders --------------------------------

def test_qr_kinds_oracle_hand_example():
    """n = 6, n_L = 3, one intra PE bit (position 3), inter bits 4 and 5.
    {0,1,2} -> {0,1,3}: qubit 3 comes from the intra position (intra), qubit 2
    takes position 3.  -> {0,1,4}: qubit 4 comes from inter position 4
    (inter), qubit 3 goes there.  -> {0,1,2}: qubit 2 comes from position 3
    (intra)."""
    M = [{0, 1, 2}, {0, 1, 3}, {0, 1, 4}, {0, 1, 2}]
    assert S.qr_kinds_by_position(M, 6, 3, 1) == (2, 1)
    assert S.qr_kinds_by_position(M, 6, 3, 0) == (0, 3)     # every PE bit inter
    assert S.qr_kinds_by_position(M, 6, 3, 3) == (3, 0)     # every PE bit intra
    assert S.comm_cost(2, 1, 1.0, 10.0) == 12.0


@pytest.mark.parametrize("seed", range(8))
def test_qr_kinds_oracle_against_ad_hoc_transpositions(seed):
    """The ad hoc method records its own position pairs: a reorder is inter
    exactly when one of its pairs touches an inter position."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(8, 16))
    nL = n - int(rng.integers(2, 5))
    n_intra = int(rng.integers(0, n - nL + 1))
    ops = [tuple(int(v) for v in rng.choice(n, size=int(rng.integers(1, 4)), replace=False))
           for _ in range(60)]
    _, M, qrs = S.ad_hoc(n, ops, nL)
    want_inter = sum(1 for pairs in qrs if any(max(a, b) >= nL + n_intra for a, b in pairs))
    assert S.qr_kinds_by_position(M, n, nL, n_intra) == (len(qrs) - want_inter, want_inter)


def test_qr_cost_figure_counts(P):
    gold = json.load(open(os.path.join(GOLD, "hierarchical_tiling_fig.json")))
    n, nL, ni = gold["n"], gold["n_L"], gold["n_intra"]
    pc = gold["paper_counts"]
    fl = P.sv_qr_cost(n, nL, ni, _fig_ops(), P.PLAN_FLAT, 1.0, 20.0)
    hi = P.sv_qr_cost(n, nL, ni, _fig_ops(), P.PLAN_HIERARCHICAL, 1.0, 20.0, fill_highest=True)
    assert fl[:2] == (pc["flat"]["intra"], pc["flat"]["inter"])
    assert hi[:2] == (pc["hierarchical"]["intra"], pc["hierarchical"]["inter"])
    assert hi[2] < fl[2] == 60.0


@pytest.mark.parametrize("seed", range(10))
def test_qr_cost_matches_oracle(P, seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(8, 18))
    nL = n - int(rng.integers(2, 6))
    n_intra = int(rng.integers(0, n - nL + 1))
    ops = [tuple(int(v) for v in rng.choice(n, size=int(rng.integers(1, min(5, nL) + 1)), replace=False))
           for _ in range(int(rng.integers(10, 90)))]
    w = (1.0, float(rng.integers(10, 40)))
    _, M, _ = S.flat_tiling(n, ops, nL)[:3]
    want = S.qr_kinds_by_position(M, n, nL, n_intra)
    got = P.sv_qr_cost(n, nL, n_intra, ops, P.PLAN_FLAT, *w)
    assert got[:2] == want and got[2] == S.comm_cost(*want, *w)
    _, M, _ = S.ad_hoc(n, ops, nL)
    assert P.sv_qr_cost(n, nL, n_intra, ops, P.PLAN_ADHOC, *w)[:2] == \
        S.qr_kinds_by_position(M, n, nL, n_intra)
    for fill in ("lowest", "highest"):
        ev = S.hierarchical_tiling(n, ops, nL, n_intra, fill=fill)[3]
        want = S.hierarchical_kinds(ev, n, nL, n_intra)
        got = P.sv_qr_cost(n, nL, n_intra, ops, P.PLAN_HIERARCHICAL, *w, fill_highest=fill == "highest")
        assert got[:2] == want and got[2] == S.comm_cost(*want, *w)


@pytest.mark.parametrize("n", [30, 36])
def test_comm_cost_gatefabric_sweep(P, n):
    """eq. comm_cost on the evaluation's GateFabric configuration (4n layers,
    block operators, 32 PEs: g = 5 with 8 GPUs per node, so 3 intra and 2
    inter PE bits): the library's N_intra / N_inter equal the oracle's for
    flat and hierarchical tiling; the hierarchical method makes fewer inter
    reorders, and its weighted cost is lower once w_inter / w_intra reaches
    tens (30)."""
    g, n_intra = 5, 3
    nL = n - g
    ops = W.block_ops(n, 4 * n)
    _, M, _ = S.flat_tiling(n, ops, nL)[:3]
    fl = S.qr_kinds_by_position(M, n, nL, n_intra)
    hi = S.hierarchical_kinds(S.hierarchical_tiling(n, ops, nL, n_intra)[3], n, nL, n_intra)
    assert P.sv_qr_cost(n, nL, n_intra, ops, P.PLAN_FLAT)[:2] == fl
    assert P.sv_qr_cost(n, nL, n_intra, ops, P.PLAN_HIERARCHICAL)[:2] == hi
    assert hi[1] < fl[1]
    assert S.comm_cost(*hi, 1.0, 30.0) < S.comm_cost(*fl, 1.0, 30.0)


def test_qr_cost_rejects_bad_arguments(P):
    ops = [(0, 1), (2, 3)]
    for args in ((6, 4, 3, ops, P.PLAN_FLAT),      # n_local + n_intra > n
                 (6, 4, -1, ops, P.PLAN_FLAT),     # negative n_intra
                 (6, 4, 1, ops, 7)):               # no such method
        with pytest.raises(P.SvqError) as ei:
            P.sv_qr_cost(*args)
        assert P.STATUS[ei.value.status] == "EINVAL"
    for w in ((float("nan"), 1.0), (1.0, float("inf")), (-1.0, 10.0)):
        with pytest.raises(P.SvqError) as ei:
            P.sv_qr_cost(6, 4, 1, ops, P.PLAN_FLAT, *w)
        assert P.STATUS[ei.value.status] == "EINVAL"
    # no reorder at all: zero cost whatever the weights
    assert P.sv_qr_cost(6, 4, 1, ops, P.PLAN_FLAT, 1.0, 30.0) == (0, 0, 0.0)
