"""VQE energy as a differentiable torch function.

``VQEEnergy.apply(theta, problem)`` returns E(theta) = <psi0|U(theta)^dag H
U(theta)|psi0> as a 0-d float64 CUDA tensor.  The forward call runs the
library's adjoint sweep (sv_grad): one forward pass, lambda = H psi, then a
reverse sweep that un-applies the circuit on psi and lambda while summing the
FP64 gradient.  The gradient stays on the device and ``backward`` only scales
it by the incoming gradient.  No 2^n state is checkpointed per layer.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import (LAZY, State, _check, _dptr, gates_array, lib, paulis_array, svq_stats)


class Problem:
    """A fixed circuit and Hamiltonian bound to one state handle."""

    def __init__(self, circuit, ham, g=0, dtype="c64", sched=LAZY, psi0_index=None):
        self.circuit = circuit
        self.ham = ham
        self.sched = sched
        self.state = State(circuit.n, g, dtype)
        self.psi0 = circuit.psi0_index if psi0_index is None else psi0_index
        self.gates_c = gates_array(circuit.gates)
        self.terms_c = paulis_array(ham)
        self.m = len(circuit.gates)
        self.nt = len(ham.coef)
        self.npar = circuit.n_params
        self.stats = svq_stats()

    def close(self):
        self.state.close()


class VQEEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, prob: Problem):
        th = np.ascontiguousarray(theta.detach().to("cpu", torch.float64).numpy())
        if th.shape[0] != prob.npar:
            raise ValueError(f"theta has {th.shape[0]} entries, the circuit {prob.npar}")
        dev = torch.device("cuda", torch.cuda.current_device())
        energy = torch.empty((), dtype=torch.float64, device=dev)
        grad = torch.empty(max(1, prob.npar), dtype=torch.float64, device=dev)
        h = prob.state.h
        _check(lib.sv_set_basis(h, int(prob.psi0)))
        _check(lib.sv_grad(h, prob.gates_c, prob.m, _dptr(th), prob.npar, prob.terms_c, prob.nt,
                           prob.sched, None,
                           ctypes.cast(energy.data_ptr(), ctypes.POINTER(ctypes.c_double)),
                           None, ctypes.cast(grad.data_ptr(), ctypes.POINTER(ctypes.c_double)),
                           ctypes.byref(prob.stats)))
        ctx.save_for_backward(grad[:prob.npar])
        ctx.theta_device = theta.device
        ctx.theta_dtype = theta.dtype
        return energy

    @staticmethod
    def backward(ctx, g_out):
        (grad,) = ctx.saved_tensors
        gt = (g_out * grad).to(ctx.theta_device, ctx.theta_dtype)
        return gt, None


def vqe_energy(theta: torch.Tensor, prob: Problem) -> torch.Tensor:
    return VQEEnergy.apply(theta, prob)
