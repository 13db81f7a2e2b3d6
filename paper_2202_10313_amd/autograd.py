"""torch.autograd bridge to the library's discrete adjoint.

`Simulation.seismograms(rho, vp, vs)` runs the forward solve for per-element
materials given as CUDA float64 tensors and returns the receiver seismograms
as a tensor on the same device; calling backward on any scalar built from
them runs edg_adjoint (the checkpointed reverse sweep of the GPU kernels) and
returns d/d rho, d/d vp, d/d vs.  Argument marshalling only: both directions
run in libedge_lts.so, and every array crosses the C-ABI as a device pointer
(edg_upload_materials, edg_read_receivers and edg_adjoint with on_device = 1),
so nothing is copied to the host.

Clusters and time steps are those of the context's edg_upload_clusters call
and stay fixed for every material passed in (the adjoint differentiates the
discrete scheme at fixed steps), as do omega and the anelastic weights.  Each
backward must follow its own forward: a later forward on the same Simulation
replaces the checkpoints, so the backward of an earlier graph raises
RuntimeError instead of returning the later model's gradient.
"""
from __future__ import annotations

import numpy as np
import torch


def _cuda64(t):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("Simulation.seismograms takes CUDA tensors")
    return t.detach().to(torch.float64).contiguous()


class _Seismograms(torch.autograd.Function):
    @staticmethod
    def forward(fctx, rho, vp, vs, sim):
        sim._forward(_cuda64(rho), _cuda64(vp), _cuda64(vs))
        fctx.sim = sim
        fctx.generation = sim.generation
        fctx.dtypes = (rho.dtype, vp.dtype, vs.dtype)
        return sim.context.read_receivers_device(rho.device)

    @staticmethod
    def backward(fctx, grad_seis):
        sim = fctx.sim
        if sim.generation != fctx.generation:
            raise RuntimeError("a later forward on this Simulation replaced the checkpoints of this graph: "
                               "run its backward before the next forward")
        torch.cuda.current_stream(grad_seis.device).synchronize()
        res = sim.context.adjoint_device(grad_seis.to(torch.float64).contiguous())
        g = [res[k].to(dt) for k, dt in zip(("g_rho", "g_vp", "g_vs"), fctx.dtypes)]
        return g[0], g[1], g[2], None


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
        self.generation = 0          # forwards run so far (a backward checks it is still its own)

    def _forward(self, rho, vp, vs):
        c = self.context
        torch.cuda.current_stream(rho.device).synchronize()
        if self.attn is None:
            c.upload_materials(rho, vp, vs)
        else:
            c.upload_materials(rho, vp, vs, *self.attn)
        c.rewind()
        c.set_checkpointing(self.every)
        c.set_initial(self.q0)
        c.advance_to(self.t_end)
        self.generation += 1

    def seismograms(self, rho, vp, vs):
        """Receiver samples [n_rec][n_samples][9] (float64 tensor on rho's
        device), differentiable with respect to rho, vp, vs."""
        return _Seismograms.apply(rho, vp, vs, self)
