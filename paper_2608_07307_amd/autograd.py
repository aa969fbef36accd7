"""torch.autograd.Function over srp_eval_grad_batch.

SrpEval.apply(rho_s, rho_d, theta, scene, sun_dirs, n, bounces, pressure)
returns the SRP forces (E, 3) of a batch of attitudes (sun_dirs (E, 3), body
frame) for optical coefficients rho_s, rho_d (M,) and hinge angles theta (J,)
or (E, J).  The forward pass runs the batched evaluation with the
hand-written adjoint on the GPU and keeps the per-item Jacobians dF/drho_s,
dF/drho_d, dF/dtheta and dF/dd (d = -s/|s| the photon direction; fixed
visibility: the hit sets of the forward pass are held, and each primary ray
keeps its share of its triangle's visible area) on the device; the backward
pass contracts them with the incoming gradient, and for sun_dirs chains
dF/dd with dd/ds = -(I - s_hat s_hat^T)/|s|.  An attitude enters through the
body-frame Sun direction, so attitude gradients follow by composing with the
rotation in torch (F_inertial = R F(R^T s)).  For coefficient estimation and
variational equations.
"""
from __future__ import annotations

import numpy as np
import torch

from . import RESULT_DTYPE, Scene, eval_grad_batch, params

_REC = RESULT_DTYPE.itemsize // 8   # doubles per result record


class SrpEval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho_s, rho_d, theta, scene: Scene, sun_dirs, n, bounces, pressure):
        M, J = scene.n_mats, scene.n_dof
        if rho_s.shape != (M,) or rho_d.shape != (M,):
            raise ValueError("rho_s and rho_d need shape (n_mats,)")
        sun_t = torch.as_tensor(sun_dirs)
        sun = np.asarray(sun_t.detach().cpu(), dtype=np.float64).reshape(-1, 3)
        E = sun.shape[0]
        th = theta.detach().cpu().double().numpy()
        th = np.broadcast_to(th.reshape(-1, J) if th.ndim == 2 else th.reshape(1, J), (E, J))
        scene.set_materials(np.stack([rho_s.detach().cpu().double().numpy(),
                                      rho_d.detach().cpu().double().numpy()], 1))
        want_dir = bool(getattr(sun_dirs, "requires_grad", False))
        entries = [(scene, th[k], params(sun[k], n, bounces, float(pressure), grad_dir=want_dir)) for k in range(E)]
        res, grad = eval_grad_batch(entries)
        F = res.view(torch.float64).view(E, _REC)[:, :3].clone()
        ctx.save_for_backward(grad, torch.as_tensor(sun, dtype=torch.float64, device=grad.device))
        ctx.dims = (E, M, J, theta.dim() == 2)
        ctx.sun_shape = tuple(sun_t.shape)
        ctx.sun_device, ctx.sun_dtype = sun_t.device, sun_t.dtype
        out_dev = rho_s.device if rho_s.is_cuda else F.device
        return F.to(device=out_dev, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gF):
        grad, sun = ctx.saved_tensors
        E, M, J, per_item_theta = ctx.dims
        g = gF.to(device=grad.device, dtype=torch.float64).reshape(E, 1, 3)
        Js = grad[:, : 3 * M].reshape(E, M, 3)
        Jd = grad[:, 3 * M: 6 * M].reshape(E, M, 3)
        Jt = grad[:, 6 * M: 6 * M + 3 * J].reshape(E, J, 3)
        g_s = (Js * g).sum((0, 2))
        g_d = (Jd * g).sum((0, 2))
        g_t = (Jt * g).sum(2)
        if not per_item_theta:
            g_t = g_t.sum(0)
        g_sun = None
        if ctx.needs_input_grad[4]:
            Jd = grad[:, 6 * M + 3 * J: 6 * M + 3 * J + 9].reshape(E, 3, 3)   # dF_i/dd_j
            gdir = (g.reshape(E, 3, 1) * Jd).sum(1)                               # dL/dd
            norm = sun.norm(dim=1, keepdim=True)
            sh = sun / norm
            g_sun = -(gdir - (gdir * sh).sum(1, keepdim=True) * sh) / norm
            g_sun = g_sun.reshape(ctx.sun_shape).to(device=ctx.sun_device, dtype=ctx.sun_dtype)
        return g_s, g_d, g_t, None, g_sun, None, None, None


def srp_forces(rho_s, rho_d, theta, scene, sun_dirs, n, bounces=0, pressure=1.0):
    """Differentiable SRP forces (E, 3) of a batch of attitudes."""
    return SrpEval.apply(rho_s, rho_d, theta, scene, sun_dirs, n, bounces, pressure)
