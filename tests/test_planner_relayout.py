"""Host-only checks of gate-pass plans whose stores relabel tile positions:
replaying the steps reproduces the final layout; every pass's tile holds its
gates' qubits and the c lowest positions; every store permutes only its own
tile; every QR exchanges local with global positions.  Also: relabelling
stores never need more passes than plain stores."""
import pytest

import workloads as W


@pytest.fixture(scope="module")
def P():
    import paper_2410_04252_amd as P
    return P


CASES = {
    "fabric30": (lambda: W.config("fabric30")["circuit"], 5),
    "fabric20": (lambda: W.fabric(20, 12, 5), 3),
    "random16": (lambda: W.random_circuit(16, 400, 7), 3),
    "hea14": (lambda: W.hea(14, 6, 8), 2),
}


def _replay(d, circ, c):
    n, nL = circ.n, circ.n - d["g"]
    lay = list(range(n))
    order, o = d["order"], 0
    for s in d["steps"]:
        if s["type"] == "qr":
            for a, b in s["swaps"]:
                assert (a < nL) != (b < nL)
                for q in range(n):
                    if lay[q] == a:
                        lay[q] = b
                    elif lay[q] == b:
                        lay[q] = a
            continue
        T, O = s["tile_bits"], s["tile_bits_out"]
        assert T == sorted(T) and sorted(O) == T and len(T) == d["tile_k"]
        assert set(range(min(c, d["tile_k"]))) <= set(T)
        assert max(T) < nL
        for gi in order[o:o + s["gates"]]:
            for q in circ.gates[gi][1]:
                assert lay[q] in T, (gi, q, lay[q], T)
        o += s["gates"]
        where = {p: q for q, p in enumerate(lay)}
        moved = [where[t] for t in T]
        for j, q in enumerate(moved):
            lay[q] = O[j]
    assert o == len(circ.gates)
    assert sorted(order) == list(range(len(circ.gates)))
    assert lay == d["pos_after"]


@pytest.mark.parametrize("relayout", ["1", "0"])
@pytest.mark.parametrize("c", [3, 4, 6])
@pytest.mark.parametrize("k", [10, 12, 13])
@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("sched", [0, 1])
def test_plan_replays(P, monkeypatch, name, k, c, sched, relayout):
    monkeypatch.setenv("SVQ_LOW_BITS", str(c))
    monkeypatch.setenv("SVQ_RELAYOUT", relayout)
    make, g = CASES[name]
    circ = make()
    k = min(k, circ.n - g)
    d = P.sv_plan_circuit_json(circ.n, g, circ.gates, sched, k)
    assert d["tile_k"] == k and d["low_bits"] == min(c, k)
    _replay(d, circ, c)
    if relayout == "0":
        assert all(s["tile_bits"] == s["tile_bits_out"] for s in d["steps"] if s["type"] != "qr")


@pytest.mark.parametrize("c", [4, 6])
@pytest.mark.parametrize("k", [12, 13])
def test_relabelling_saves_passes_at_30_qubits(P, monkeypatch, k, c):
    circ = W.config("fabric30")["circuit"]
    monkeypatch.setenv("SVQ_LOW_BITS", str(c))
    monkeypatch.setenv("SVQ_RELAYOUT", "0")
    plain = P.sv_plan_circuit_json(30, 5, circ.gates, 1, k)
    monkeypatch.setenv("SVQ_RELAYOUT", "1")
    rel = P.sv_plan_circuit_json(30, 5, circ.gates, 1, k)
    assert rel["n_qr"] == plain["n_qr"] == 2
    assert rel["n_passes"] < plain["n_passes"]
