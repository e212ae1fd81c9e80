"""torch.autograd.Function around the library's adjoint (twa_adjoint).

Forward builds the pump of Eq. (2) for (w, alpha), runs the checkpointed
forward and the reverse sweep in one call and returns the steady-state
<S+S-> and g2; backward contracts the incoming gradients with the pathwise
(fixed-noise) derivatives the sweep produced.  All arithmetic happens in the
HIP library; this module only moves scalars.
"""
from __future__ import annotations

import torch


class TWAObservables(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, alpha, cfg: dict):
        from . import adjoint, build_pump
        wv, av = float(w.detach()), float(alpha.detach())
        pump = build_pump(int(cfg["N"]), wv, av)
        try:
            obs, g = adjoint(pump, int(cfg["n_traj"]), float(cfg["dt"]), int(cfg["n_steps"]),
                             int(cfg.get("seed", 0)), ckpt_every=int(cfg.get("ckpt_every", 256)),
                             gamma=float(cfg.get("gamma", 1.0)), s0z=float(cfg.get("s0z", 1.0)),
                             burnin=int(cfg.get("burnin", -1)), precision=cfg.get("precision", "fp32"),
                             norm_tol=float(cfg.get("norm_tol", 0.0)))
        finally:
            pump.close()
        ctx.save_for_backward(torch.tensor([[g["d_SpSm_dw"], g["d_SpSm_dalpha"]],
                                            [g["d_g2_dw"], g["d_g2_dalpha"]]], dtype=torch.float64))
        ctx.obs = obs
        return (torch.tensor(obs["SpSm"], dtype=torch.float64), torch.tensor(obs["g2"], dtype=torch.float64))

    @staticmethod
    def backward(ctx, g_spsm, g_g2):
        (jac,) = ctx.saved_tensors
        gw = g_spsm * jac[0, 0] + g_g2 * jac[1, 0]
        ga = g_spsm * jac[0, 1] + g_g2 * jac[1, 1]
        return gw, ga, None
