"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (lazy schedule, default tile widths), through properties and closed
forms that the oracle can afford at 28-30 qubits."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import ENERGY_REL, energy_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2410_04252_amd as P
    torch.cuda.set_device(0)
    return P


def _print(*a):
    print(*a, flush=True)


def _inverse(circ):
    """U^dagger as a gate list: reversed order, negated angles (every
    parametric kind here is exp(-i t K)); the remaining fabric kinds are
    self-inverse."""
    gates = []
    for kind, qs, p in reversed(circ.gates):
        assert kind in ("GIVENS", "CPHASE", "RY", "RZ", "RX")
        gates.append((kind, qs, -1, -float(circ.theta[p])))
    return gates


def test_fabric30_roundtrip_and_particle_number(P):
    """U then U^dagger returns psi0; U keeps the Hamming-weight sector (the
    fabric block conserves particle number), so every amplitude outside the
    sector is exactly zero."""
    import torch
    cfg = W.config("fabric30")
    circ, g = cfg["circuit"], cfg["g"]
    n = circ.n
    _print("fabric30 round trip")
    buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    st = P.State(n, g, "c64", buf=buf)
    st.set_basis(circ.psi0_index)
    stats = st.apply(circ, sched=P.LAZY)
    assert stats.n_qr == 2
    # sector check on the device: the buffer is in physical order; popcount
    # of the physical index equals that of the logical one
    ne = bin(circ.psi0_index).count("1")
    idx = torch.arange(1 << n, device="cuda", dtype=torch.int64)
    pc = torch.zeros_like(idx)
    for b in range(n):
        pc += (idx >> b) & 1
    inside = pc == ne
    amp2 = buf.real.double() ** 2 + buf.imag.double() ** 2
    outside = float(amp2[~inside].sum())
    norm = float(amp2.sum())
    del idx, pc, inside, amp2
    assert outside == 0.0
    assert abs(norm - 1.0) < 1e-5
    st.apply_gates(_inverse(circ), theta=[], sched=P.LAZY)
    v = buf.to("cpu")
    # the layout may be permuted; the basis state's physical index follows pos
    pos = st.layout()
    phys = sum(1 << pos[q] for q in range(n) if (circ.psi0_index >> q) & 1)
    top = complex(v[phys])
    assert abs(top - 1.0) < 1e-4
    rest = float((v.abs() ** 2).sum()) - abs(top) ** 2
    assert rest < 1e-8
    st.close()


def test_fabric30_evc_product_state_closed_form(P):
    """EVC of the 2000-term JW Hamiltonian on a 30-qubit product state
    prod_q RZ(f_q) RY(t_q)|0>: every <P> is a product of single-site factors."""
    cfg = W.config("fabric30")
    ham, g = cfg["ham"], cfg["g"]
    n = ham.n
    circ, t, f = W.product_state_circuit(n, 3030)
    _print("fabric30 product-state EVC")
    want = 0.0
    for k in range(len(ham.coef)):
        x, z = int(ham.x[k]), int(ham.z[k])
        v = 1.0
        for q in range(n):
            xb, zb = (x >> q) & 1, (z >> q) & 1
            if xb and zb:
                v *= math.sin(t[q]) * math.sin(f[q])
            elif xb:
                v *= math.sin(t[q]) * math.cos(f[q])
            elif zb:
                v *= math.cos(t[q])
        want += ham.coef[k] * v
    for sched in (P.LAZY, P.EAGER):
        st = P.State(n, g, "c64")
        st.set_basis(0)
        st.apply(circ, sched=sched)
        e, stats = st.expectation(ham, sched=sched)
        assert abs(e - want) <= ENERGY_REL["c64"] * energy_scale(want, ham), (e, want)
        st.close()


def test_fabric28_evc_random_state_sampled_terms(P):
    """A seeded dense random 28-qubit state; the GPU evaluates a sample of the
    2000 Pauli strings that the oracle computes term by term."""
    cfg = W.config("fabric28")
    ham, g = cfg["ham"], cfg["g"]
    n = ham.n
    _print("fabric28 random-state EVC")
    v = W.random_state(n, 2828, np.complex64)
    rng = np.random.default_rng(28)
    pick = np.sort(rng.choice(len(ham.coef), size=24, replace=False))
    sub = W.Hamiltonian(n, ham.x[pick], ham.z[pick], ham.coef[pick])
    st = P.State(n, g, "c64")
    st.set_amplitudes(v)
    e, _ = st.expectation(sub, sched=P.LAZY)
    st.close()
    ref = oracle.expectation(v.astype(np.complex128), sub)
    assert abs(e - ref) <= ENERGY_REL["c64"] * energy_scale(ref, sub), (e, ref)


def test_grad24_adjoint_equals_gpu_parameter_shift(P):
    """At the full 24-qubit, 400-parameter size: the adjoint gradient equals
    the exact parameter-shift gradient (two-term rule for CPHASE, two-frequency
    four-term rule for GIVENS) on a sample of parameters."""
    import torch
    cfg = W.config("grad24")
    circ, ham = cfg["circuit"], cfg["ham"]
    n, g = circ.n, 5
    _print("grad24 adjoint vs parameter shift")
    st = P.State(n, g, "c64")
    st.set_basis(circ.psi0_index)
    _, grad, _ = st.grad(circ, ham)
    kind_of = {p: kind for kind, _, p in circ.gates}
    rng = np.random.default_rng(24)
    sample = rng.choice(len(circ.theta), size=12, replace=False)
    for p in sample:
        acc = 0.0
        for shift, w in oracle.SHIFT_RULES[kind_of[p]]:
            for sgn in (+1, -1):
                th = circ.theta.copy()
                th[p] += sgn * shift
                st.set_basis(circ.psi0_index)
                st.apply(circ, theta=th)
                e, _ = st.expectation(ham)
                acc += sgn * w * e
        assert abs(acc - grad[p]) <= 1e-5 * max(1e-3, np.abs(grad).max()), (p, acc, grad[p])
    st.close()


def test_wide_chunk_round_trip_64bit_offsets(P):
    """31 qubits with one global qubit: chunks of 2^30 amplitudes (8 GiB), so
    passes whose tiles reach physical bit 29 take the 64-bit in-tile offset
    path and the others the 32-bit one.  U then U^dagger must return the
    basis state; every amplitude outside its particle-number sector stays
    exactly zero after U."""
    import torch
    n, g = 31, 1
    circ = W.fabric(n, 4, 3131)
    _print("31-qubit round trip (64-bit offsets)")
    buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    st = P.State(n, g, "c64", buf=buf)
    st.set_basis(circ.psi0_index)
    stats = st.apply(circ, sched=P.LAZY)
    assert stats.n_gate_passes >= 1
    amp2 = (buf.real.double() ** 2 + buf.imag.double() ** 2)
    assert abs(float(amp2.sum()) - 1.0) < 1e-5
    del amp2
    st.apply_gates(_inverse(circ), theta=[], sched=P.LAZY)
    pos = st.layout()
    phys = sum(1 << pos[q] for q in range(n) if (circ.psi0_index >> q) & 1)
    top = complex(buf[phys].item())
    assert abs(top - 1.0) < 1e-4
    st.close()


def _product_expectation(ham, t, f):
    want = 0.0
    for k in range(len(ham.coef)):
        x, z = int(ham.x[k]), int(ham.z[k])
        v = 1.0
        for q in range(ham.n):
            xb, zb = (x >> q) & 1, (z >> q) & 1
            if xb and zb:
                v *= math.sin(t[q]) * math.sin(f[q])
            elif xb:
                v *= math.sin(t[q]) * math.cos(f[q])
            elif zb:
                v *= math.cos(t[q])
            if v == 0.0:
                break
        want += ham.coef[k] * v
    return want


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_fabric32_evc_product_state_and_round_trip(P, dtype):
    """The 32-qubit configuration (g = 6, 10^4 JW-like strings), c64 (32 GiB)
    and c128 (64 GiB): EVC of a product state against its closed form, then
    the 360-gate fabric circuit and its inverse return the basis state."""
    cfg = W.config("fabric32")
    circ, ham, g = cfg["circuit"], cfg["ham"], cfg["g"]
    n = ham.n
    pc, t, f = W.product_state_circuit(n, 3232)
    want = _product_expectation(ham, t, f)
    _print(f"fabric32 {dtype} product-state EVC")
    import torch
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    buf = torch.empty(1 << n, dtype=tdt, device="cuda")
    st = P.State(n, g, dtype, buf=buf)
    st.set_basis(0)
    st.apply(pc)
    e, stats = st.expectation(ham)
    assert stats.n_qr <= 8
    assert abs(e - want) <= ENERGY_REL[dtype] * energy_scale(want, ham), (e, want)
    _print(f"fabric32 {dtype} round trip")
    st.set_basis(circ.psi0_index)
    s1 = st.apply(circ)
    assert s1.n_qr <= 4
    st.apply_gates(_inverse(circ), theta=[], sched=P.LAZY)
    pos = st.layout()
    phys = sum(1 << pos[q] for q in range(n) if (circ.psi0_index >> q) & 1)
    top = complex(buf[phys].item())
    assert abs(top - 1.0) < (1e-4 if dtype == "c64" else 1e-10), top
    st.close()
    del buf
    torch.cuda.empty_cache()
