"""PyTorch autograd entry for the probe-energy objective.

J(eps) = sum_n dt sum_{T in probes} ||e^n||^2_{L2(T)} along the RK4 trajectory
of a fixed initial field, with dJ/deps computed by the library's checkpointed
discrete adjoint (mdg_adjoint_probe_energy). The binding only marshals
arguments; the forward steps, the adjoint sweep and the reductions run in
the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from .mdg import Solver


class ProbeEnergyProblem:
    """Mesh, initial state, sources and run length of the objective; eps is
    the differentiable input. E0/H0 are covariant coefficients [nt][3][N]
    (they do not depend on eps). dipoles = (pos[n][3], dir[n][3], wave[n][3])
    or None; omega[nt][3] per-axis PML damping or None (the PML starts at
    rest); mixed pairs e at order+1 with h at order (H0 then has the modes of
    h's order); flux is "central" or "upwind"; sip_alpha > 0 adds the SIP
    surface unknown (central flux, starting at zero)."""

    def __init__(self, verts, tets, order, E0, H0, dt, nsteps, every, probes, mu=None, dipoles=None,
                 precision="fp64", omega=None, mixed=False, flux="central", sip_alpha=0.0):
        self.verts, self.tets, self.order = verts, tets, order
        self.E0, self.H0, self.mu, self.dipoles = E0, H0, mu, dipoles
        self.omega, self.mixed = omega, mixed
        self.flux, self.sip_alpha = flux, sip_alpha
        self.dt, self.nsteps, self.every = dt, nsteps, every
        self.probes = np.asarray(probes, dtype=np.int64)
        self.precision = precision

    def _solver(self, eps):
        """The problem's solver with permittivity eps and the initial state:
        built once (mesh setup, device workspace), re-bound for a new eps."""
        if getattr(self, "_s", None) is None:
            s = Solver(self.order, self.precision, self.flux, dt=self.dt, mixed=self.mixed,
                       sip_alpha=self.sip_alpha)
            s.set_mesh(self.verts, self.tets)
            s.set_material(eps, self.mu)
            if self.omega is not None:
                s.set_pml(self.omega)
            if self.dipoles is not None:
                s.set_dipoles(*self.dipoles)
            self._ws = s.bind_torch_workspace()
            self._s = s
        else:
            s = self._s
            s.set_material(eps, self.mu)
            s.bind_workspace(self._ws, torch.cuda.current_stream(self._ws.device).cuda_stream)
        s.set_state(self.E0, self.H0)
        return s

    def run(self, eps):
        """(J, dJ/deps) by the library's checkpointed discrete adjoint."""
        return self._solver(eps).adjoint_probe_energy(self.nsteps, self.every, self.probes)

    def objective(self, eps):
        """J alone (the forward steps only)."""
        return self._solver(eps).probe_energy(self.nsteps, self.probes)

    def close(self):
        if getattr(self, "_s", None) is not None:
            self._s.close()
            self._s = None
            self._ws = None

    def __call__(self, eps: torch.Tensor) -> torch.Tensor:
        return ProbeEnergy.apply(eps, self)


class ProbeEnergy(torch.autograd.Function):
    """J(eps); the adjoint sweep runs only when a gradient is requested."""

    @staticmethod
    def forward(ctx, eps, problem):
        e = eps.detach().cpu().double().numpy()
        if ctx.needs_input_grad[0]:
            J, g = problem.run(e)
            ctx.save_for_backward(torch.as_tensor(g, dtype=eps.dtype, device=eps.device))
        else:
            J = problem.objective(e)
        return eps.new_tensor(J)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        return gJ * g, None
