"""Host-only checks of the LDS slot map the planner gives each gate pass.

Every transpose writes the tile to LDS with one phase's lane mapping and reads
it back with the next phase's; tile index t lives in slot XOR_j(swz[j] for the
set bits j of t).  Checked on the plans of several workloads, tile widths and
low-bit counts:

* the map is a bijection of the tile (swz[0..5] independent six-bit values,
  swz[j] = 2^j ^ six low bits above that), checked exhaustively on the tile;
* the load and store phases keep the tile bits on the lowest physical
  positions (before and after the store's relabelling) as their first lanes;
* every phase's first 3, 4 and 5 lanes have slot values independent modulo 8,
  16 and 32 (the condition for conflict-free 8- and 16-byte LDS accesses);
* no phase lists a register or wave bit as a lane twice."""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def P():
    import paper_2410_04252_amd as P
    return P


def _rank(vals, nbits):
    piv = {}
    r = 0
    for x in vals:
        x &= (1 << nbits) - 1
        while x:
            hb = x.bit_length() - 1
            if hb not in piv:
                piv[hb] = x
                r += 1
                break
            x ^= piv[hb]
    return r


def _slots(swz, k):
    t = np.arange(1 << k, dtype=np.int64)
    s = np.zeros_like(t)
    for j in range(k):
        s ^= np.where((t >> j) & 1, swz[j], 0)
    return s


# name: (qubits, global qubits, circuit)
CASES = {
    "fabric30": (30, 5, lambda: W.config("fabric30")["circuit"]),
    "fabric20": (20, 3, lambda: W.fabric(20, 12, 5)),
    "random16": (16, 3, lambda: W.random_circuit(16, 400, 7)),
    "hea14": (14, 2, lambda: W.hea(14, 6, 8)),
}
PARAMS = [(name, k, c) for name, (n, g, _) in CASES.items() for k in (10, 12, 13) if k <= n - g
          for c in (3, 4, 6)]


@pytest.mark.parametrize("name,k,c", PARAMS)
def test_slot_map(P, name, k, c, monkeypatch):
    n, g, make = CASES[name]
    circ = make()
    assert circ.n == n
    monkeypatch.setenv("SVQ_LOW_BITS", str(c))
    d = P.sv_plan_circuit_json(circ.n, g, circ.gates, P.LAZY, k)
    K, cl = d["tile_k"], min(d["low_bits"], 6)
    assert K == k
    multi = 0
    for s in d["steps"]:
        if s["type"] != "gate_pass":
            continue
        swz = s["swz"]
        assert _rank(swz[:6], 6) == 6
        for j in range(6, K):
            assert swz[j] >> 6 == 1 << (j - 6), (j, swz[j])
        slots = _slots(swz, K)
        assert slots.min() == 0 and slots.max() == (1 << K) - 1
        assert np.unique(slots).size == 1 << K
        lanes = s["lanes"]
        assert len(lanes) == s["phases"]
        for ph, l in enumerate(lanes):
            assert len(set(l)) == 6 and all(0 <= t < K for t in l)
            assert not set(l) & set(s["regs"][ph])
        ld = {j for j in range(K) if s["tile_bits"][j] < cl}
        st = {j for j in range(K) if s["tile_bits_out"][j] < cl}
        assert set(lanes[0][:len(ld)]) == ld
        assert set(lanes[-1][:len(st)]) == st
        if len(lanes) < 2:
            continue
        multi += 1
        for l in lanes:
            v = [swz[t] for t in l]
            assert _rank(v[:3], 3) == 3 and _rank(v[:4], 4) == 4 and _rank(v[:5], 5) == 5, (l, v)
    assert multi > 0
