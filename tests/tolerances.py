"""Tolerances of the parity tests.

Amplitudes: max |delta psi| <= 1e-5 (complex64) / 1e-12 (complex128), and the
relative L2 error ||psi - psi_ref|| / ||psi_ref|| under the same bounds (for a
normalised state the L2 bound is the stricter of the two).

Energy: "1e-6 relative" (complex64) / 1e-12 (complex128), taken relative to
max(|E|, 1e-2 * sum_t |a_t|).  Gradient: ||g - g_ref||_2 <= 1e-6 (complex64) /
1e-11 (complex128) times max(||g_ref||_2, 1e-2 * sum_t |a_t|).

Why the floor: a rounding error delta in a complex64 state moves each <P_t>
(and each 2 Im <lambda|K_j|psi>) by an amount set by ||delta|| and the
Hamiltonian's 1-norm, not by the size of the result, so a purely relative
bound fails whenever the terms cancel to a small energy or gradient.  The
smallest decade that clears the error of complex64 arithmetic itself is
1e-2: test_complex64_noise.py evaluates circuits in plain complex64 numpy
arithmetic (no GPU) and finds energies that miss 1e-6 relative to
max(|E|, 1e-3 sum |a_t|) and gradients that miss 1e-6 relative to ||g||,
while every one of them meets the bounds above.
"""
import numpy as np


AMP = {"c64": 1e-5, "c128": 1e-12}
AMP_REL_L2 = {"c64": 1e-5, "c128": 1e-12}
ENERGY_REL = {"c64": 1e-6, "c128": 1e-12}
GRAD_REL = {"c64": 1e-6, "c128": 1e-11}
FLOOR = 1e-2


def energy_scale(e_ref, ham):
    return max(abs(e_ref), FLOOR * float(np.abs(ham.coef).sum()))


def energy_ok(e, e_ref, psi_ref, ham, dtype):
    """psi_ref is accepted for call-site symmetry; the scale needs only E and H."""
    scale = energy_scale(e_ref, ham)
    return abs(e - e_ref) <= ENERGY_REL[dtype] * scale, abs(e - e_ref) / scale


def grad_scale(g_ref, ham):
    return max(float(np.linalg.norm(g_ref)), FLOOR * float(np.abs(ham.coef).sum()))


def grad_ok(grad, g_ref, ham, dtype):
    """(ok, ||g - g_ref|| / scale)."""
    rel = float(np.linalg.norm(np.asarray(grad) - np.asarray(g_ref))) / grad_scale(g_ref, ham)
    return rel <= GRAD_REL[dtype], rel


def amp_errors(psi, ref, block=1 << 24):
    """(max |psi - ref|, ||psi - ref||_2 / ||ref||_2), in blocks so that a
    2^30-amplitude comparison needs no full-size temporaries."""
    psi = np.asarray(psi).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    assert psi.shape == ref.shape
    mx, d2, r2 = 0.0, 0.0, 0.0
    for i in range(0, ref.size, block):
        r = ref[i:i + block].astype(np.complex128)
        d = psi[i:i + block].astype(np.complex128) - r
        a = np.abs(d)
        if a.size:
            mx = max(mx, float(a.max()))
        d2 += float(np.vdot(d, d).real)
        r2 += float(np.vdot(r, r).real)
    return mx, (d2 ** 0.5) / max(r2 ** 0.5, 1e-300)


def amp_ok(psi, ref, dtype):
    mx, rl2 = amp_errors(psi, ref)
    return mx <= AMP[dtype] and rl2 <= AMP_REL_L2[dtype], mx, rl2
