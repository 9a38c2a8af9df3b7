"""``msm_energy``: the MSM energy as a differentiable function of positions
and charges.

The paper's problem statement (Section 2) asks for the energy and the forces
F_i = -dU/dr_i; U is also a quadratic form in the charges, so dU/dq_i is the
per-atom potential phi_i. Both gradients come from the library's own kernels
(the interpolation kernel returns the force and potential of every atom in
the same pass), so the backward pass is two scalings of saved tensors.
"""
from __future__ import annotations

import torch


class _MsmEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, msm, offsets):
        xyzq = torch.cat([pos.detach(), q.detach().unsqueeze(-1)], dim=1).contiguous()
        energy, forces, pots = msm.energy_forces(xyzq, offsets)
        ctx.save_for_backward(forces, pots)
        ctx.offsets = offsets
        return energy

    @staticmethod
    def backward(ctx, g):
        forces, pots = ctx.saved_tensors
        offsets = ctx.offsets
        if offsets is None:
            scale = g.to(forces.dtype).reshape(1)[0]
            gpos = -scale * forces
            gq = scale * pots
        else:
            counts = torch.as_tensor([offsets[i + 1] - offsets[i] for i in range(len(offsets) - 1)],
                                     device=forces.device)
            per_atom = torch.repeat_interleave(g.to(forces.dtype), counts)
            gpos = -per_atom[:, None] * forces
            gq = per_atom * pots
        return gpos, gq, None, None


def msm_energy(pos: torch.Tensor, q: torch.Tensor, msm, offsets=None) -> torch.Tensor:
    """Energy of each system (float64 tensor of length nsys) with gradients
    dU/dpos = -F and dU/dq = phi. ``pos`` (N, 3) and ``q`` (N,) must be device
    tensors in the context's precision."""
    return _MsmEnergy.apply(pos, q, msm, offsets)
