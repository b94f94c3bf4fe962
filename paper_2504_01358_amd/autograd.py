"""torch.autograd binding of the shading: the forward runs ssr_shade and keeps
its per-sample hit codes; the backward runs ssr_shade_backward with those
codes replayed (the hit selection is held fixed, as the paper treats its
screen-space tracing)."""

import torch

from . import ssr


class _Shade(torch.autograd.Function):
    @staticmethod
    def forward(fctx, context, camera, params, depth, normal_rough, albedo_metal, radiance, env):
        cam = ssr.make_camera(camera) if not isinstance(camera, ssr.Camera) else camera
        prm = ssr.make_params(params) if not isinstance(params, ssr.Params) else params
        hits = torch.empty((cam.height, cam.width, prm.spp), dtype=torch.int32, device=depth.device)
        out = context.shade(cam, depth, normal_rough.detach(), albedo_metal.detach(),
                            radiance.detach(), env.detach(), prm, hits=hits)
        fctx.save_for_backward(depth, normal_rough, albedo_metal, radiance, env, hits)
        fctx.context, fctx.cam, fctx.prm = context, cam, prm
        return out

    @staticmethod
    def backward(fctx, grad_out):
        depth, nr, am, rad, env, hits = fctx.saved_tensors
        need = fctx.needs_input_grad
        dev = depth.device
        H, W = fctx.cam.height, fctx.cam.width
        g_nr = torch.empty((H, W, 4), dtype=torch.float32, device=dev) if need[4] else None
        g_am = torch.empty((H, W, 4), dtype=torch.float32, device=dev) if need[5] else None
        g_rad = torch.zeros((H, W, 4), dtype=torch.float32, device=dev) if need[6] else None
        g_env = torch.zeros(tuple(env.shape), dtype=torch.float32, device=dev) if need[7] else None
        fctx.context.shade_backward(fctx.cam, depth, nr.detach(), am.detach(), rad.detach(),
                                    env.detach(), fctx.prm, hits,
                                    grad_out.contiguous().to(torch.float32), g_normal_rough=g_nr,
                                    g_albedo_metal=g_am, g_env=g_env, g_radiance=g_rad)
        cast = (lambda g, like: None if g is None else g.to(like.dtype))
        return (None, None, None, None, cast(g_nr, nr), cast(g_am, am), cast(g_rad, rad),
                cast(g_env, env))


def shade(context, camera, params, depth, normal_rough, albedo_metal, radiance, env):
    """Differentiable ssr_shade: the image [H][W][3], with gradients for
    normal_rough, albedo_metal, radiance and env (depth is not differentiated)."""
    return _Shade.apply(context, camera, params, depth, normal_rough, albedo_metal, radiance, env)
