"""ADER-DG time stepping on a mesh through the C ABI: predictor (stp_predict)
then corrector (stp_correct) every step.

Orchestration and argument marshalling only: the per-face Godunov operators
and the reference tables come from the library's host functions, every step
runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np

from . import api
from . import workload as wl


class AderSolver:
    """Global time stepping of one degree N on a mesh (``mesh.Mesh``) with
    per-element physical Jacobians ABC [n, 3, nq, nq] and sources E [n, nq, nq]
    (host arrays); state Q [n, nq, B] on the device."""

    def __init__(self, N, mesh, ABC, E, device="cuda"):
        import torch
        self.N, self.mesh = N, mesh
        ABC = np.ascontiguousarray(ABC, dtype=np.float64)
        n, nq = ABC.shape[0], ABC.shape[-1]
        self.n, self.nq, self.B = n, nq, wl.n_modes(N)
        star = wl.star_matrices(ABC[:, 0], ABC[:, 1], ABC[:, 2], mesh.vertices)
        Gp, Gm = api.face_operators(ABC, mesh.vertices)
        dev = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        self.star, self.E = dev(star), dev(E)
        self.Gp, self.Gm = dev(Gp), dev(Gm)
        self.neighbor = dev(mesh.neighbor, torch.int32)
        self.nb_code = dev(mesh.nb_code, torch.int32)
        self.tables = dev(api.corrector_tables(N))
        self.Qst = torch.empty((n, nq, self.B, N + 1), dtype=torch.float64, device=device)
        self.Qint = torch.empty((n, nq, self.B), dtype=torch.float64, device=device)

    def predict(self, Q, dt, **kw):
        api.predict(Q, self.star, self.E, dt, self.N, Q=self.Qst, Qint=self.Qint, **kw)
        return self.Qint

    def correct(self, Q, Qint=None):
        api.correct(self.N, self.tables, self.star, self.E, self.Gp, self.Gm, self.neighbor, self.nb_code,
                    self.Qint if Qint is None else Qint, Q)
        return Q

    def step(self, Q, dt, **kw):
        """One ADER-DG step in place: Q^{n+1} from Q^n."""
        self.predict(Q, dt, **kw)
        return self.correct(Q)

    def cfl_dt(self, vmax, c=0.5):
        """Global time step of the CFL condition dt = c / (2N+1) min d / v."""
        return c / (2 * self.N + 1) * float(wl.insphere_diameter(self.mesh.vertices).min()) / vmax
