"""Receiver seismograms as a differentiable function of the per-element
material (lambda, mu, rho), for full-waveform-inversion style misfits.

Forward: the implicit scheme from rest with point sources, the velocity
sampled at the receivers after every step.  Backward: the discrete adjoint
of the time stepping (sdg_adjoint_step, run step by step backwards), with
the forward slabs recomputed segment by segment from checkpoints of the
state taken every `checkpoint_every` steps, so the memory held is one
segment of velocity slabs plus the checkpoints.

All arithmetic runs in the library's kernels; this module only sequences
the calls and holds the device buffers.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (Context, SDG_PREC_F64, SDG_PRECOND_MASS, SDG_SOLVER_AUTO, SolveOpts, sdg_set_material,
               sdg_assemble, sdg_query)


class Seismograms:
    """Seismogram simulator bound to one mesh and discretisation.

    mesh: object with xyz, elem, period (see synth.Mesh); p, p_gamma, scheme
    (SDG_SCHEME_*), dt; src_pos (n_src, dim), src_dir (n_src, dim);
    amps (n_steps, n_src, N_gamma) source amplitudes at the slab time nodes;
    receivers (n_rec, dim).
    """

    def __init__(self, mesh, p, p_gamma, scheme, dt, lam, mu, rho, src_pos, src_dir, amps, receivers,
                 checkpoint_every=20, opts: SolveOpts | None = None, device=0, precisions=None):
        self.ctx = Context(device)
        self.mesh = mesh
        precisions = precisions or SDG_PREC_F64
        self.device = torch.device("cuda", device)
        self.sizes = self.ctx.setup(mesh.xyz, mesh.elem, mesh.period, p, p_gamma, scheme, dt,
                                    np.asarray(lam, float), np.asarray(mu, float), np.asarray(rho, float),
                                    precisions)
        self.precisions = precisions
        self.ctx.set_sources(src_pos, src_dir)
        self.amps = np.asarray(amps, float)
        self.receivers = np.asarray(receivers, float)
        self.n_steps = self.amps.shape[0]
        self.K = int(checkpoint_every)
        if self.K < 1:
            raise ValueError("checkpoint_every must be >= 1")
        self.opts = opts or SolveOpts(SDG_SOLVER_AUTO, SDG_PREC_F64, 1e-12, 4000, 30, 5, 10, 1e-4, SDG_PRECOND_MASS)
        self._material = self._key(lam, mu, rho)
        self.stats = {"forward_steps": 0, "adjoint_steps": 0, "krylov_iterations": 0}

    # --------------------------------------------------------------- helpers
    @staticmethod
    def _key(lam, mu, rho):
        return tuple(np.ascontiguousarray(x, float).tobytes() for x in (lam, mu, rho))

    def set_material(self, lam, mu, rho):
        key = self._key(lam, mu, rho)
        if key == self._material:
            return
        sdg_set_material(self.ctx.h, np.asarray(lam, float), np.asarray(mu, float), np.asarray(rho, float))
        sdg_assemble(self.ctx.h, self.precisions)
        self.ctx.sizes = sdg_query(self.ctx.h)
        self._material = key

    def _zeros_state(self):
        v = torch.zeros(self.sizes["n_vel_state"], dtype=torch.float64, device=self.device)
        s = torch.zeros(self.sizes["n_stress_state"], dtype=torch.float64, device=self.device)
        return v, s

    def _step(self, v, s, n, v_slab=None):
        info = self.ctx.step(v, s, self.amps[n].ravel(), opts=self.opts, v_slab=v_slab)
        self.stats["forward_steps"] += 1
        self.stats["krylov_iterations"] += info["iterations"]

    def _sample(self, v, out):
        from . import sdg_sample_velocity
        sdg_sample_velocity(self.ctx.h, v, self.receivers, out)

    # --------------------------------------------------------------- API
    def run(self, lam, mu, rho, keep_checkpoints=False):
        """Forward only: seismograms (n_steps, n_rec, dim) on the device."""
        self.set_material(lam, mu, rho)
        v, s = self._zeros_state()
        d = self.sizes["dim"]
        obs = torch.empty((self.n_steps, len(self.receivers), d), dtype=torch.float64, device=self.device)
        ckpt = []
        for n in range(self.n_steps):
            if keep_checkpoints and n % self.K == 0:
                ckpt.append((v.clone(), s.clone()))
            self._step(v, s, n)
            self._sample(v, obs[n])
        return obs, ckpt

    def gradient(self, lam, mu, rho, obs_bar, checkpoints):
        """Adjoint sweep: given dJ/d(obs) (n_steps, n_rec, dim) on the
        device, return dJ/d(lambda, mu, rho) as a (3, n_elem) device tensor."""
        self.set_material(lam, mu, rho)
        ne = self.sizes["n_elem"]
        grad = torch.zeros(3 * ne, dtype=torch.float64, device=self.device)
        vbar, sbar = self._zeros_state()
        nslab = self.sizes["n_vel_slab"]
        seg_len = min(self.K, self.n_steps)
        slabs = torch.empty((seg_len, nslab), dtype=torch.float64, device=self.device)
        olds = torch.empty((seg_len, self.sizes["n_vel_state"]), dtype=torch.float64, device=self.device)
        obs_bar = obs_bar.to(dtype=torch.float64).contiguous()
        n_seg = (self.n_steps + self.K - 1) // self.K
        for seg in range(n_seg - 1, -1, -1):
            n0, n1 = seg * self.K, min(self.n_steps, (seg + 1) * self.K)
            v, s = (t.clone() for t in checkpoints[seg])
            for n in range(n0, n1):
                olds[n - n0].copy_(v)
                self._step(v, s, n, v_slab=slabs[n - n0])
            for n in range(n1 - 1, n0 - 1, -1):
                # misfit terms at t^{n+1,-} act on the state the step produced
                self.ctx.sample_adjoint(self.receivers, obs_bar[n].reshape(-1).contiguous(), vbar)
                info = self.ctx.adjoint_step(olds[n - n0], slabs[n - n0], vbar, sbar, grad, opts=self.opts)
                self.stats["adjoint_steps"] += 1
                self.stats["krylov_iterations"] += info["iterations"]
        return grad.view(3, ne)

    def __call__(self, lam: torch.Tensor, mu: torch.Tensor, rho: torch.Tensor) -> torch.Tensor:
        return _SeismogramFn.apply(lam, mu, rho, self)

    def close(self):
        self.ctx.close()


class _SeismogramFn(torch.autograd.Function):
    """obs = F(lambda, mu, rho); backward runs the checkpointed discrete adjoint."""

    @staticmethod
    def forward(fctx, lam, mu, rho, sim: Seismograms):
        host = [t.detach().to("cpu", torch.float64).numpy() for t in (lam, mu, rho)]
        obs, ckpt = sim.run(*host, keep_checkpoints=True)
        fctx.sim = sim
        fctx.host = host
        fctx.ckpt = ckpt
        fctx.dev = lam.device
        return obs

    @staticmethod
    def backward(fctx, obs_bar):
        sim = fctx.sim
        g = sim.gradient(*fctx.host, obs_bar, fctx.ckpt)
        fctx.ckpt = None
        out = g.to(fctx.dev)
        return out[0], out[1], out[2], None
