"""Differentiable closest hit: ``(t, u, v)`` of the nearest accepted hit as a
function of the rays and of the mesh's vertex positions.

Forward: host BVH build over ``vertices[faces]`` (rt_bvh_build) -- or, given
a ``rtx.RefitScene`` built once from the mesh, a device refit of that tree to
the current vertices (rt_bvh_refit) -- and one rt_trace_closest launch with
the chosen intersector.  Backward: one
rt_hit_backward launch (implicit differentiation of o + t d = P(u, v) for the
fixed hit triangle).  The hit triangle and the intersector's decision are
discrete and are not differentiated; misses return zeros with zero gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rtx


def _same_cuda_device(**tensors):
    """Raises ValueError unless every tensor lives on one CUDA device: the
    backward kernel dereferences their data pointers on that device."""
    devs = {name: t.device for name, t in tensors.items() if t is not None}
    bad = [name for name, d in devs.items() if d.type != "cuda"]
    if bad:
        raise ValueError(f"{', '.join(bad)} must be CUDA tensors (got {[str(devs[b]) for b in bad]})")
    if len(set(devs.values())) > 1:
        raise ValueError(f"tensors on different devices: { {k: str(v) for k, v in devs.items()} }")


class DifferentiableHit(torch.autograd.Function):
    """``tuv, prim, hit = DifferentiableHit.apply(rays, vertices, faces, geom_ids,
    texcoords, textures, intersector, alpha_min, checker_n, max_leaf, image_width,
    refit, shape)``

    rays float32 [N, 8] and vertices float32 [nv, 3] on one GPU (both may
    require grad; anything else raises ValueError before a launch); faces
    uint32/int32 [n, 3] on any device (copied to the vertices' device);
    geom_ids, texcoords, textures as
    numpy arrays (alpha intersector) or None; max_leaf: leaf size limit of the
    forward's BVH build (1..7); image_width: the rays form an image of that
    width in scanline order, traced in 8 x 8 tiles (same results); refit: a
    ``rtx.RefitScene`` of this mesh (its faces, texture data and leaf limit
    replace the arguments'), refitted on the device to ``vertices`` instead
    of a host rebuild; shape: the forward's launch shape (one of
    ``rtx.rt_launch_shapes()``, None for the default; results do not depend
    on it -- a launch with fewer rays than resident lanes runs faster without
    the persistent queue).  Returns tuv float32 [N, 3]
    (zeros for misses), prim int32 [N] (-1 for misses) and hit bool [N]."""

    @staticmethod
    def forward(ctx, rays, vertices, faces, geom_ids, texcoords, textures, intersector="default",
                alpha_min=128, checker_n=8, max_leaf=4, image_width=None, refit=None,
                shape=None):
        _same_cuda_device(rays=rays, vertices=vertices)
        v = vertices.detach()
        if refit is not None:
            scene = refit.update(v.contiguous())
            f = refit.faces
        else:
            f = faces.detach().to(torch.int64)
            tris = v.cpu().numpy()[f.cpu().numpy()]
            scene = rtx.upload_scene(tris, geom_ids, texcoords, textures, device=rays.device,
                                     max_leaf=max_leaf)
        hits = rtx.trace(scene, rays.detach().contiguous(), intersector, alpha_min=alpha_min,
                         checker_n=checker_n, image_width=image_width, shape=shape)
        prim = hits[:, 1].view(torch.int32).clone()
        hit = prim != -1
        tuv = hits[:, [0, 2, 3]].clone()
        tuv[~hit] = 0.0
        # the backward kernel reads the faces on the vertices' device
        faces_u32 = f.to(device=v.device, dtype=torch.int32).contiguous()
        ctx.save_for_backward(rays.detach().contiguous(), hits, v.contiguous(), faces_u32)
        ctx.mark_non_differentiable(prim, hit)
        return tuv, prim, hit

    @staticmethod
    def backward(ctx, grad_tuv, grad_prim=None, grad_hit=None):
        rays, hits, vertices, faces = ctx.saved_tensors
        n = rays.shape[0]
        g = grad_tuv.contiguous().to(torch.float32)
        _same_cuda_device(rays=rays, hits=hits, vertices=vertices, faces=faces, grad_tuv=g)
        grad_vertices = torch.zeros_like(vertices)
        grad_rays = torch.empty_like(rays)
        stream = torch.cuda.current_stream(rays.device).cuda_stream
        rtx.rt_hit_backward(rays.data_ptr(), hits.data_ptr(), g.data_ptr(), n,
                            vertices.data_ptr(), vertices.shape[0], faces.data_ptr(),
                            faces.shape[0], grad_vertices.data_ptr(), grad_rays.data_ptr(),
                            stream)
        return (grad_rays, grad_vertices, None, None, None, None, None, None, None, None, None,
                None, None)


def hit_backward(rays, hits, grad_tuv, vertices, faces, grad_vertices=None, grad_rays=True):
    """Direct call of rt_hit_backward on device tensors.  Returns
    (grad_vertices, grad_rays or None); grad_vertices is zeroed here unless
    given (then accumulated)."""
    _same_cuda_device(rays=rays, hits=hits, vertices=vertices, grad_tuv=grad_tuv,
                      grad_vertices=grad_vertices)
    if grad_vertices is None:
        grad_vertices = torch.zeros_like(vertices)
    gr = torch.empty_like(rays) if grad_rays else None
    # faces given on the host are copied to the vertices' device
    faces_i = faces.to(device=vertices.device, dtype=torch.int32).contiguous()
    g = grad_tuv.contiguous().to(torch.float32)
    stream = torch.cuda.current_stream(rays.device).cuda_stream
    rtx.rt_hit_backward(rays.data_ptr(), hits.data_ptr(), g.data_ptr(), rays.shape[0],
                        vertices.data_ptr(), vertices.shape[0], faces_i.data_ptr(),
                        faces_i.shape[0], grad_vertices.data_ptr(),
                        None if gr is None else gr.data_ptr(), stream)
    return grad_vertices, gr


def as_numpy_u32(faces) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(faces), np.uint32)
