"""The ansatz energy E(theta) = <psi(theta)|H|psi(theta)> / <psi(theta)|psi(theta)>
as a torch.autograd.Function whose backward is the library's adjoint sweep
(fock_energy_grad_adjoint: forward gates, H psi, one reverse sweep giving all
dE/dtheta_k = 2 Re <lambda_k|A_k phi_k> / <psi|psi>, Sec. IV.B gradient
identity applied to every parameter).

    energy = AnsatzEnergy(ham, ops, psi0)      # owns two work states and the workspace
    theta = torch.zeros(len(ops), dtype=torch.float64, requires_grad=True)
    E = energy(theta)                           # 0-dim float64 tensor (host)
    E.backward()                                # theta.grad = dE/dtheta

theta lives on the host (float64): the library stages angles to the device
itself.  When theta requires a gradient the forward call already runs the
reverse sweep (one library call computes E and dE/dtheta together) and the
backward only scales the stored gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lib


class _AdjointEnergyFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, runner):
        want = theta.requires_grad
        E, n2, g = runner._eval(theta.detach().cpu().numpy().astype(np.float64), want)
        ctx.save_for_backward(torch.from_numpy(g) if want else torch.zeros(0, dtype=torch.float64))
        ctx.n2 = n2
        return torch.tensor(E, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gE):
        (g,) = ctx.saved_tensors
        return gE * g, None


class AnsatzEnergy:
    """Callable E(theta) for a fixed Hamiltonian, operator list and initial
    state (a complex64 CUDA tensor of d^L amplitudes)."""

    def __init__(self, ham: lib.Ham, ops, psi0, stream=None):
        self.ham, self.ops, self.psi0, self.stream = ham, list(ops), psi0, stream
        self.phi = torch.empty_like(psi0)
        self.lam = torch.empty_like(psi0)
        self.ws = lib.workspace(ham, 0, len(self.ops))
        self.last_norm2 = None

    def _eval(self, theta, grad):
        if theta.shape != (len(self.ops),):
            raise lib.FockError(-1, f"theta must have shape ({len(self.ops)},), got {theta.shape}")
        E, n2, g = lib.energy_grad_adjoint(self.ham, self.ops, theta, self.psi0, self.phi, self.lam, self.ws,
                                           grad=grad, stream=self.stream)
        self.last_norm2 = n2
        return E, n2, g

    def __call__(self, theta: torch.Tensor) -> torch.Tensor:
        return _AdjointEnergyFn.apply(theta, self)
