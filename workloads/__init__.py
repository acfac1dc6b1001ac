"""Seeded synthetic inputs for the state-vector hot path and for its CPU checker.

This module only *draws* data: gate lists (kind name, qubits, parameter
index), angles, Pauli strings as (x_mask, z_mask, coefficient) and dense
random states.  It holds none of the simulation arithmetic (no gate matrices,
no Pauli action, no schedules), so the HIP path and the oracle can both use it
without sharing any of the method's code.

Conventions (fixed here so both sides read the data the same way):

* qubit q is bit q of the amplitude index (qubit 0 = least significant bit),
  as in the paper's state-vector layout (Section "Preliminaries", eq. sv);
* a gate is ``(kind, qubits, param)``: ``kind`` is one of ``GATE_KINDS``,
  ``qubits`` a tuple (controlled gates list the control first), ``param`` an
  index into the angle vector ``theta`` or -1 for a fixed gate;
* a Pauli string is ``(x, z, coef)``: qubit q carries X if only bit q of x is
  set, Z if only bit q of z is set, Y if both are set; ``coef`` is real
  (Pauli strings are Hermitian, so the Hamiltonian of eq. hamiltonian is real
  when its coefficients are).

Random generator: ``numpy.random.default_rng(seed)`` (PCG64).  Draw order:
angles in gate order, then Pauli terms in emission order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GATE_KINDS = ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ",
              "CNOT", "CZ", "CPHASE", "GIVENS", "SWAP")
#: number of qubits each gate kind acts on
GATE_ARITY = {"H": 1, "X": 1, "Y": 1, "Z": 1, "S": 1, "T": 1, "RX": 1, "RY": 1,
              "RZ": 1, "CNOT": 2, "CZ": 2, "CPHASE": 2, "GIVENS": 2, "SWAP": 2}
#: gate kinds that take an angle
PARAM_KINDS = ("RX", "RY", "RZ", "CPHASE", "GIVENS")

SEED_BASE = 4252


@dataclass
class Circuit:
    n: int
    gates: list = field(default_factory=list)   # [(kind, (q0, q1?), param)]
    theta: np.ndarray = field(default_factory=lambda: np.zeros(0))
    psi0_index: int = 0                          # initial computational basis state

    @property
    def n_params(self) -> int:
        return int(self.theta.shape[0])


@dataclass
class Hamiltonian:
    n: int
    x: np.ndarray      # uint64 flip masks
    z: np.ndarray      # uint64 phase masks
    coef: np.ndarray   # float64

    def __len__(self) -> int:
        return int(self.x.shape[0])

    def n_groups(self) -> int:
        return int(np.unique(self.x).shape[0])


# --------------------------------------------------------------------------
# circuits
# --------------------------------------------------------------------------

def hea(n: int, layers: int, seed: int) -> Circuit:
    """Hardware-efficient ansatz: per layer an RY then an RZ on every qubit,
    then a linear CNOT ladder 0->1->...->n-1.  Angles uniform in [0, 2pi)."""
    rng = np.random.default_rng(seed)
    gates, p = [], 0
    for _ in range(layers):
        for q in range(n):
            gates.append(("RY", (q,), p)); p += 1
        for q in range(n):
            gates.append(("RZ", (q,), p)); p += 1
        for q in range(n - 1):
            gates.append(("CNOT", (q, q + 1), -1))
    theta = rng.uniform(0.0, 2.0 * math.pi, size=p)
    return Circuit(n, gates, theta, 0)


def fabric(n: int, layers: int, seed: int, max_params: int | None = None,
           n_electrons: int | None = None) -> Circuit:
    """Fabric-style particle-conserving ansatz (the paper's GateFabric is only
    cited, so its block is fixed here): spin-orbital pairs P_j = (2j, 2j+1);
    a block on P_j u P_{j+1} is GIVENS(2j, 2j+2), GIVENS(2j+1, 2j+3) and
    CPHASE(2j+1, 2j+2).  Layer l places blocks at j = l (mod 2), j+1 < n//2.
    Angles uniform in [-pi, pi).  With ``max_params`` the brick order is cut
    after that many parameters.  Initial state: the lowest ``n_electrons``
    qubits set (Hartree-Fock-like), default min(10, n//2)."""
    rng = np.random.default_rng(seed)
    npairs = n // 2
    gates, p = [], 0
    done = False
    for layer in range(layers):
        for j in range(layer % 2, npairs - 1, 2):
            for kind, qs in (("GIVENS", (2 * j, 2 * j + 2)),
                             ("GIVENS", (2 * j + 1, 2 * j + 3)),
                             ("CPHASE", (2 * j + 1, 2 * j + 2))):
                if max_params is not None and p >= max_params:
                    done = True
                    break
                gates.append((kind, qs, p)); p += 1
            if done:
                break
        if done:
            break
    theta = rng.uniform(-math.pi, math.pi, size=p)
    ne = min(10, n // 2) if n_electrons is None else n_electrons
    return Circuit(n, gates, theta, (1 << ne) - 1)


def block_ops(n: int, layers: int) -> list:
    """The fabric circuit as one operator per 4-qubit block (the operator
    granularity the paper schedules GateFabric at); each entry is a qubit
    tuple.  Used for paper-style QR counts only."""
    ops = []
    for layer in range(layers):
        for j in range(layer % 2, n // 2 - 1, 2):
            ops.append((2 * j, 2 * j + 1, 2 * j + 2, 2 * j + 3))
    return ops


def random_circuit(n: int, m: int, seed: int) -> Circuit:
    """Random mix of every gate kind on random qubits (parity stress input)."""
    rng = np.random.default_rng(seed)
    gates, p = [], 0
    kinds = GATE_KINDS
    draws = []
    for _ in range(m):
        kind = kinds[int(rng.integers(len(kinds)))]
        a = GATE_ARITY[kind]
        qs = tuple(int(v) for v in rng.choice(n, size=a, replace=False))
        if kind in PARAM_KINDS:
            gates.append((kind, qs, p)); p += 1
        else:
            gates.append((kind, qs, -1))
        draws.append(kind)
    theta = rng.uniform(-math.pi, math.pi, size=p)
    return Circuit(n, gates, theta, 0)


# --------------------------------------------------------------------------
# Hamiltonians
# --------------------------------------------------------------------------

def _mask(qs) -> int:
    v = 0
    for q in qs:
        v |= 1 << int(q)
    return v


def random_pauli(n: int, n_terms: int, seed: int, sigma: float = 1.0) -> Hamiltonian:
    """Each qubit's letter uniform in {I, X, Y, Z}; coefficients N(0, sigma)."""
    rng = np.random.default_rng(seed)
    xs, zs = [], []
    for _ in range(n_terms):
        letters = rng.integers(0, 4, size=n)       # 0=I 1=X 2=Y 3=Z
        x = _mask([q for q in range(n) if letters[q] in (1, 2)])
        z = _mask([q for q in range(n) if letters[q] in (2, 3)])
        xs.append(x); zs.append(z)
    coef = rng.normal(0.0, sigma, size=n_terms)
    return Hamiltonian(n, np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64), coef)


_TWO_SITE = (("X", "X"), ("Y", "Y"))
_FOUR_SITE = tuple(c for c in
                   ((a, b, cc, d) for a in "XY" for b in "XY" for cc in "XY" for d in "XY")
                   if sum(ch == "Y" for ch in c) % 2 == 0)   # 8 combos with even #Y


def _letters_to_xz(sites, letters, zchain):
    x = z = 0
    for q, ch in zip(sites, letters):
        x |= 1 << q
        if ch == "Y":
            z |= 1 << q
    for q in zchain:
        z |= 1 << q
    return x, z


def jw_terms(n: int, n_terms: int, seed: int, sigma: float = 0.1,
             frac_diag: float = 0.05, frac_two: float = 0.15) -> Hamiltonian:
    """Jordan-Wigner-like Hamiltonian (real-orbital molecular structure).

    * diagonal: Z_p or Z_p Z_q;
    * two-site hopping: {XX, YY} at p < q with a Z chain on (p, q) - both
      letter combos are emitted for each drawn (p, q);
    * four-site: p < q < r < s, the 8 X/Y combos with an even number of Y,
      Z chains on (p, q) and (r, s) - all 8 emitted per drawn tuple.

    Strings are distinct; a kind that runs out of distinct strings passes its
    share to the four-site kind.  Coefficients N(0, sigma)."""
    rng = np.random.default_rng(seed)
    want_diag = int(round(frac_diag * n_terms))
    want_two = int(round(frac_two * n_terms))
    seen = set()
    out = []

    def add(x, z):
        if (x, z) in seen:
            return False
        seen.add((x, z)); out.append((x, z))
        return True

    # diagonal
    n_diag_avail = n + n * (n - 1) // 2
    want_diag = min(want_diag, n_diag_avail)
    while len(out) < want_diag:
        if rng.random() < 0.3:
            p = int(rng.integers(n)); add(0, 1 << p)
        else:
            p, q = sorted(int(v) for v in rng.choice(n, size=2, replace=False))
            add(0, (1 << p) | (1 << q))
    # two-site hopping
    n_two_avail = 2 * (n * (n - 1) // 2)
    want_two = min(want_two, n_two_avail)
    target = len(out) + want_two
    while len(out) < target:
        p, q = sorted(int(v) for v in rng.choice(n, size=2, replace=False))
        for letters in _TWO_SITE:
            if len(out) >= target:
                break
            add(*_letters_to_xz((p, q), letters, range(p + 1, q)))
    # four-site
    while len(out) < n_terms:
        p, q, r, s = sorted(int(v) for v in rng.choice(n, size=4, replace=False))
        chain = list(range(p + 1, q)) + list(range(r + 1, s))
        for letters in _FOUR_SITE:
            if len(out) >= n_terms:
                break
            add(*_letters_to_xz((p, q, r, s), letters, chain))
    coef = rng.normal(0.0, sigma, size=len(out))
    x = np.array([a for a, _ in out], dtype=np.uint64)
    z = np.array([b for _, b in out], dtype=np.uint64)
    return Hamiltonian(n, x, z, coef)


def product_state_circuit(n: int, seed: int):
    """Per-qubit RY(t_q) then RZ(f_q) from |0...0>: a product state whose
    Pauli expectations have a closed form at any n.  Returns the circuit and
    the (t, f) angle arrays."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, math.pi, size=n)
    f = rng.uniform(-math.pi, math.pi, size=n)
    gates, theta = [], []
    for q in range(n):
        gates.append(("RY", (q,), len(theta))); theta.append(t[q])
        gates.append(("RZ", (q,), len(theta))); theta.append(f[q])
    return Circuit(n, gates, np.array(theta), 0), t, f


def random_state(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Dense random state (complex Gaussian entries, unit norm)."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    v /= np.sqrt(np.vdot(v, v).real)
    return v.astype(dtype)


# --------------------------------------------------------------------------
# the five workload configurations and the 30-qubit headline
# --------------------------------------------------------------------------

def config(name: str) -> dict:
    """Workload by name: 'hea12', 'fabric28', 'fabric30', 'fabric32',
    'grad24', and 'batch' (the latter via :func:`batch_instances`)."""
    if name == "hea12":
        c = hea(12, 4, SEED_BASE + 1)
        h = random_pauli(12, 64, SEED_BASE + 1 + 1000)
        return dict(name=name, circuit=c, ham=h, g=2, k=8, dtype="c128")
    if name == "fabric28":
        c = fabric(28, 8, SEED_BASE + 2)
        h = jw_terms(28, 2000, SEED_BASE + 2 + 1000)
        return dict(name=name, circuit=c, ham=h, g=5, k=0, dtype="c64")
    if name == "fabric30":
        c = fabric(30, 16, SEED_BASE + 30)
        h = jw_terms(30, 2000, SEED_BASE + 30 + 1000)
        return dict(name=name, circuit=c, ham=h, g=5, k=0, dtype="c64")
    if name == "fabric32":
        c = fabric(32, 16, SEED_BASE + 3)
        h = jw_terms(32, 10000, SEED_BASE + 3 + 1000)
        return dict(name=name, circuit=c, ham=h, g=6, k=0, dtype="c64")
    if name == "grad24":
        c = fabric(24, 1000, SEED_BASE + 4, max_params=400)
        h = jw_terms(24, 1000, SEED_BASE + 4 + 1000)
        return dict(name=name, circuit=c, ham=h, g=5, k=0, dtype="c64")
    raise KeyError(name)


def batch_instances(n_inst: int = 256, seed: int = SEED_BASE * 1000,
                    n_lo: int = 10, n_hi: int = 22, layers: int = 6, n_terms: int = 200):
    """Independent VQE instances with uneven qubit counts (uniform in
    [n_lo, n_hi]); instance i uses seed ``seed + i``."""
    out = []
    for i in range(n_inst):
        rng = np.random.default_rng(seed + i)
        n = int(rng.integers(n_lo, n_hi + 1))
        c = fabric(n, layers, seed + i)
        h = jw_terms(n, n_terms, seed + i + 7919)
        out.append(dict(circuit=c, ham=h))
    return out
