"""torch.autograd.Function around the SBR radio map.

forward  -> rt_radio_map with a tape (hit slots, crossed cells, directions,
            bases and per-bounce transfer matrices of every segment)
backward -> rt_radio_map_backward: replays the tape (no re-tracing) and
            returns dLoss/d eps_r, dLoss/d sigma per material and
            dLoss/d (yaw, pitch, roll) of the transmitter

Tensors are used for device memory and the current stream only; all
arithmetic runs in the HIP kernels behind the C ABI.
"""
from __future__ import annotations

import dataclasses

import torch

from . import rt_build_scene  # noqa: F401  (re-exported for convenience)
from . import RtScene, make_params, rt_radio_map, rt_radio_map_backward, rt_tape_create


class RadioMapFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_r, sigma, orient, scene: RtScene, tx, plane, params, thickness=None, scattering=None,
                xpd=None, scatter_pattern=None):
        """eps_r, sigma: device f32 [n_mat]; orient: (yaw, pitch, roll), any
        device; thickness: optional device f32 [n_mat] slab thickness;
        scattering, xpd (and scatter_pattern): optional diffuse reflection
        (none of these four is differentiated)."""
        ypr = [float(v) for v in orient.detach().cpu().tolist()]
        txo = dataclasses.replace(tx, yaw=ypr[0], pitch=ypr[1], roll=ypr[2])
        npol = 2 if int(tx.pol) == 2 else 1
        out = torch.empty((npol, plane.H, plane.W), dtype=torch.float32, device=eps_r.device)
        p = make_params(params)
        need_grad = any(ctx.needs_input_grad[:3])
        tape = rt_tape_create(p) if need_grad else None
        diffuse = dict(scattering=scattering, xpd=xpd, scatter_pattern=scatter_pattern)
        rt_radio_map(scene, eps_r.contiguous(), sigma.contiguous(), txo, plane, p, out, tape=tape,
                     thickness=thickness, **diffuse)
        ctx.save_for_backward(eps_r, sigma)
        ctx.state = (scene, txo, plane, p, tape, orient.device, orient.dtype, thickness, diffuse)
        return out

    @staticmethod
    def backward(ctx, grad_map):
        eps_r, sigma = ctx.saved_tensors
        scene, txo, plane, p, tape, odev, odt, thickness, diffuse = ctx.state
        n_mat = eps_r.shape[0]
        ge = torch.empty(n_mat, dtype=torch.float32, device=eps_r.device)
        gs = torch.empty(n_mat, dtype=torch.float32, device=eps_r.device)
        go = torch.empty(3, dtype=torch.float32, device=eps_r.device)
        rt_radio_map_backward(scene, eps_r.contiguous(), sigma.contiguous(), txo, plane, p, tape,
                              grad_map.contiguous().to(torch.float32), ge, gs, go, thickness=thickness,
                              **diffuse)
        return (ge, gs, go.to(device=odev, dtype=odt)) + (None,) * 8


def radio_map(eps_r, sigma, orient, scene, tx, plane, params, thickness=None, scattering=None, xpd=None,
              scatter_pattern=None):
    """Differentiable radio map [npol][H][W] (slab walls and refraction with a
    thickness tensor, diffuse reflection with scattering and xpd tensors)."""
    return RadioMapFn.apply(eps_r, sigma, orient, scene, tx, plane, params, thickness, scattering, xpd,
                            scatter_pattern)
