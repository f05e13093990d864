"""Gradients of a final-state objective through many lattice-Boltzmann steps.

``final_density(rho_a0, G, rho_b0, spec)`` returns rho_A after ``spec.steps``
steps as a torch tensor that autograd can differentiate with respect to the
initial density rho_A(0) (and rho_B(0)) of a fluid at rest and the Shan-Chen
coupling G.  Every step and every adjoint step runs in liblb's HIP kernels;
this module only drives them:

* forward: lb_set_fields, then the steps, saving a raw state snapshot every
  ``spec.every`` steps (device memory, one grid per checkpoint);
* backward: seed lam(T) = dJ/drho(T) (lb_adjoint_begin); for each segment,
  last first, restore its checkpoint and recompute its steps with
  lb_step_record, which writes the moment record (rho, m, psi: 10 values per
  node) the adjoint needs instead of the whole state, then run the adjoint
  steps in reverse over the records (lb_adjoint_step_record); finally read
  dJ/drho(0) and dJ/dG (lb_adjoint_result).

Memory: one state snapshot per checkpoint plus ``spec.every`` moment records
for the segment being recomputed.
"""

from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import torch

from . import lb as L


@dataclasses.dataclass(frozen=True)
class Spec:
    shape: Tuple[int, int, int]           # (nz, ny, nx)
    tau: Tuple[float, float] = (1.0, 1.0)
    steps: int = 1
    every: int = 50                       # checkpoint interval
    storage: str = "f32"
    psi_ref: float = 1.0
    solid: Optional[torch.Tensor] = None  # uint8 [nz, ny, nx] on the device, or None
    kernel: str = "auto"


class _Timings:
    """Device-time split of the last forward/backward (for the benchmark):
    forward_ms covers the steps and the checkpoint saves (not the context's
    creation, the initial state or the final read-out); backward_ms covers
    seeding the adjoint, every restore, recomputation and adjoint step, and
    reading the gradients out."""

    forward_ms = 0.0
    backward_ms = 0.0


timings = _Timings()


def _event():
    return torch.cuda.Event(enable_timing=True)


class FinalDensity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho_a0: torch.Tensor, G: torch.Tensor, rho_b0: torch.Tensor, spec: Spec):
        dev = rho_a0.device
        n = rho_a0.numel()
        e0, e1 = _event(), _event()
        lat = L.Lattice(spec.shape, tau=spec.tau, G=float(G), psi_ref=spec.psi_ref, storage=spec.storage,
                        device=dev.index or 0, kernel=spec.kernel)
        solid = None if spec.solid is None else spec.solid.contiguous().view(-1)
        lat.set_fields(rho_a0.detach().contiguous().view(-1).to(torch.float64),
                       rho_b0.detach().contiguous().view(-1).to(torch.float64), None, solid)
        nbytes = L.lb_state_bytes(lat.ctx)
        nck = (spec.steps + spec.every - 1) // spec.every
        ckpts = [torch.empty(nbytes, dtype=torch.uint8, device=dev) for _ in range(nck)]
        e0.record()
        for k, s0 in enumerate(range(0, spec.steps, spec.every)):
            L.lb_save_state(lat.ctx, ckpts[k])
            lat.step(min(spec.every, spec.steps - s0))
        e1.record()
        out = torch.empty(n, dtype=torch.float64, device=dev)
        lat.moments(rho_a=out)
        torch.cuda.synchronize(dev)
        timings.forward_ms = e0.elapsed_time(e1)
        ctx.lat, ctx.ckpts, ctx.spec, ctx.nbytes = lat, ckpts, spec, nbytes
        return out.view(rho_a0.shape)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        lat, ckpts, spec, nbytes = ctx.lat, ctx.ckpts, ctx.spec, ctx.nbytes
        dev = grad_out.device
        n = grad_out.numel()
        e0, e1 = _event(), _event()
        seed = grad_out.detach().contiguous().view(-1).to(torch.float64)
        rbytes = L.lb_record_bytes(lat.ctx)
        recs = [torch.empty(rbytes, dtype=torch.uint8, device=dev) for _ in range(min(spec.every, spec.steps))]
        ga = torch.empty(n, dtype=torch.float64, device=dev)
        gb = torch.empty(n, dtype=torch.float64, device=dev)
        e0.record()
        L.lb_adjoint_begin(lat.ctx, n, seed, None)
        for seg in range(len(ckpts) - 1, -1, -1):
            s0 = seg * spec.every
            length = min(spec.every, spec.steps - s0)
            L.lb_restore_state(lat.ctx, ckpts[seg])
            for t in range(length):
                L.lb_step_record(lat.ctx, recs[t])
            for t in range(length - 1, -1, -1):
                L.lb_adjoint_step_record(lat.ctx, recs[t])
        dG = L.lb_adjoint_result(lat.ctx, n, ga, gb)
        e1.record()
        torch.cuda.synchronize(dev)
        timings.backward_ms = e0.elapsed_time(e1)
        lat.close()
        ctx.lat = None
        ctx.ckpts = None
        shape = grad_out.shape
        return ga.view(shape), torch.tensor(dG, dtype=torch.float64, device=dev), gb.view(shape), None


def final_density(rho_a0: torch.Tensor, G: torch.Tensor, rho_b0: torch.Tensor, spec: Spec) -> torch.Tensor:
    """rho_A after spec.steps steps from a fluid at rest with densities (rho_a0, rho_b0)."""
    return FinalDensity.apply(rho_a0, G, rho_b0, spec)
