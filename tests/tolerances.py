"""Tolerances of the parity tests.

Energy: the bound "1e-6 relative" (complex64) / 1e-12 (complex128) is taken
relative to max(|E|, 1e-2 * sum_t |a_t|).  Rounding of a complex64 state moves
every <P_t> by O(eps * gates) in absolute terms however small <P_t> is, so the
error scales with the Hamiltonian's 1-norm; the floor keeps the relative
bound meaningful when the terms cancel to an energy near zero.
Amplitudes: max |delta psi| <= 1e-5 (complex64) / 1e-12 (complex128).
Gradient: ||g - g_ref||_2 <= 1e-5 (complex64) / 1e-11 (complex128) relative.
"""
import numpy as np


AMP = {"c64": 1e-5, "c128": 1e-12}
ENERGY_REL = {"c64": 1e-6, "c128": 1e-12}
GRAD_REL = {"c64": 1e-5, "c128": 1e-11}


def energy_scale(e_ref, ham):
    return max(abs(e_ref), 1e-2 * float(np.abs(ham.coef).sum()))


def energy_ok(e, e_ref, psi_ref, ham, dtype):
    """psi_ref is accepted for call-site symmetry; the scale needs only E and H."""
    scale = energy_scale(e_ref, ham)
    return abs(e - e_ref) <= ENERGY_REL[dtype] * scale, abs(e - e_ref) / scale
