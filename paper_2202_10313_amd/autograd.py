"""torch.autograd bridge to the library's discrete adjoint.

`Simulation.seismograms(rho, vp, vs)` runs the forward solve for per-element
materials given as torch tensors and returns the receiver seismograms as a
tensor; calling backward on any scalar built from them runs edg_adjoint (the
checkpointed reverse sweep of the GPU kernels) and returns d/d rho, d/d vp,
d/d vs.  Argument marshalling only: both directions run in libedge_lts.so.

Clusters and time steps are those of the context's edg_upload_clusters call
and stay fixed for every material passed in (the adjoint differentiates the
discrete scheme at fixed steps), as do omega and the anelastic weights.  Each
backward must follow its own forward: a later forward on the same context
replaces the checkpoints (a stale backward fails with EDG_ESTATE).
"""
from __future__ import annotations

import numpy as np
import torch


def _host(t):
    return t.detach().to("cpu", torch.float64).numpy()


class _Seismograms(torch.autograd.Function):
    @staticmethod
    def forward(fctx, rho, vp, vs, sim):
        sim._forward(_host(rho), _host(vp), _host(vs))
        fctx.sim = sim
        fctx.device = rho.device
        return torch.as_tensor(sim.context.read_receivers(), dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(fctx, grad_seis):
        res = fctx.sim.context.adjoint(dj_dseis=_host(grad_seis), want_q0=False)
        to = lambda a: torch.as_tensor(a, dtype=torch.float64, device=fctx.device)  # noqa: E731
        return to(res["g_rho"]), to(res["g_vp"]), to(res["g_vs"]), None


class Simulation:
    """A context prepared for gradient runs: mesh, clusters, sources and
    receivers already uploaded (the clusters fix the time steps).

    omega, yp, ys: anelastic inputs (None for an elastic context); q0: initial
    DOFs [K][Nq][B] (None = at rest); t_end: simulated time of every forward
    solve (a multiple of the coarsest step); checkpoint_every: cycles per
    checkpoint segment of the forward (the final segment records its level
    states and is not replayed by the backward, so an interval that covers
    t_end needs no replay, at (levels per segment) states of device memory)."""

    def __init__(self, context, t_end, omega=None, yp=None, ys=None, q0=None, checkpoint_every=1):
        self.context = context
        self.t_end = float(t_end)
        self.attn = None if omega is None else (omega, yp, ys)
        self.q0 = np.zeros((context.K, context.nq, context.B)) if q0 is None else np.asarray(q0, dtype=np.float64)
        self.every = int(checkpoint_every)

    def _forward(self, rho, vp, vs):
        c = self.context
        if self.attn is None:
            c.upload_materials(rho, vp, vs)
        else:
            c.upload_materials(rho, vp, vs, *self.attn)
        c.rewind()
        c.set_checkpointing(self.every)
        c.set_initial(self.q0)
        c.advance_to(self.t_end)

    def seismograms(self, rho, vp, vs):
        """Receiver samples [n_rec][n_samples][9] (float64 tensor on rho's
        device), differentiable with respect to rho, vp, vs."""
        return _Seismograms.apply(rho, vp, vs, self)
