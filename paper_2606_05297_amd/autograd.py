"""The ansatz energy E(theta) = <psi(theta)|H|psi(theta)> / <psi(theta)|psi(theta)>
as a torch.autograd.Function whose backward is the library's hand-written
adjoint sweep (the gradient identity of Sec. IV.B applied to every parameter:
dE/dtheta_k = 2 Re <lambda_k|A_k phi_k> / <psi|psi>).

    energy = AnsatzEnergy(ham, ops, psi0)      # owns two work states and the workspace
    theta = torch.zeros(len(ops), dtype=torch.float64, requires_grad=True)
    E = energy(theta)                           # 0-dim tensor on theta's device
    E.backward()                                # theta.grad = dE/dtheta

Forward runs the circuit and H psi only (fock_energy_grad_adjoint without
gradient), leaving psi_n and H psi_n in the two work states; backward runs the
reverse sweep from them (fock_adjoint_sweep).  The angles themselves cross to
the library as host doubles (8 bytes per gate).  If the work states were
reused or consumed since this forward (another forward, or an earlier backward
with retain_graph), backward recomputes them first.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lib


class _AdjointEnergyFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, runner):
        th = theta.detach().to("cpu", torch.float64).numpy().copy()
        E, n2 = runner._energy(th)
        ctx.runner, ctx.theta, ctx.n2, ctx.token = runner, th, n2, runner._token
        return torch.tensor(E, dtype=theta.dtype if theta.dtype.is_floating_point else torch.float64,
                            device=theta.device)

    @staticmethod
    def backward(ctx, gE):
        g = ctx.runner._gradient(ctx.theta, ctx.n2, ctx.token)
        gt = torch.from_numpy(g).to(device=gE.device, dtype=gE.dtype)
        return gE * gt, None


class AnsatzEnergy:
    """Callable E(theta) for a fixed Hamiltonian, operator list and initial
    state (a complex64 CUDA tensor of d^L amplitudes)."""

    def __init__(self, ham: lib.Ham, ops, psi0, stream=None):
        lib._state_arg(psi0, ham.L, ham.d, "psi0")
        self.ham, self.ops, self.psi0, self.stream = ham, list(ops), psi0, stream
        self.phi = torch.empty_like(psi0)
        self.lam = torch.empty_like(psi0)
        self.ws = lib.workspace(ham, 0, len(self.ops))
        self.last_norm2 = None
        self._token = 0      # bumped by every forward: identifies what phi/lam hold
        self._fresh = False  # phi/lam still hold psi_n and H psi_n of the last forward

    def _check_theta(self, th):
        if th.shape != (len(self.ops),):
            raise lib.FockError(-1, f"theta must have shape ({len(self.ops)},), got {th.shape}")

    def _energy(self, th):
        self._check_theta(th)
        E, n2, _ = lib.energy_grad_adjoint(self.ham, self.ops, th, self.psi0, self.phi, self.lam, self.ws,
                                           grad=False, stream=self.stream)
        self._token += 1
        self._fresh = True
        self.last_norm2 = n2
        return E, n2

    def _gradient(self, th, n2, token):
        if not (self._fresh and token == self._token):
            _, n2 = self._energy(th)  # the work states no longer hold this forward's psi_n, H psi_n
        self._fresh = False
        return lib.adjoint_sweep(self.ham, self.ops, th, self.phi, self.lam, n2, self.ws, stream=self.stream)

    def __call__(self, theta: torch.Tensor) -> torch.Tensor:
        return _AdjointEnergyFn.apply(theta, self)
