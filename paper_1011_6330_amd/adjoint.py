"""torch.autograd.Function around the hand-written adjoint of the PIC step.

``exit_gamma_loss(knots, kappa, rate, cfg, x, u, n_steps)`` builds a tube whose
Goldreich-Julian amplitude is the piecewise-linear profile ``knots`` (eqs. 6-7
with frame dragging kappa), loads the particles (x, u), runs n_steps and returns
the mean Lorentz factor of the electrons that leave the tube.  The forward runs
only the checkpointed forward (``pic_adjoint_forward``); the reverse sweep
(``pic_backward``) runs when autograd asks for the gradient, and returns
dL/d knots, dL/d kappa and dL/d rate (the charge factor of electrons injected
during the run) with every discrete decision of the run held fixed, scaled by
the incoming gradient.  The library evaluates the forward at rate = 1 (the
gradient with respect to rate is the derivative there).
"""
import torch

from . import _binding


class ExitGammaLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, knots, kappa, rate, cfg, x, u, n_steps, checkpoint_every=50):
        if float(rate) != 1.0:
            raise ValueError("the forward step is evaluated at an injected charge factor of 1")
        c = dict(cfg)
        c["knots"] = knots.detach().to("cpu", torch.float64).numpy()
        c["kappa"] = float(kappa)
        c["rho_kind"] = _binding.RHO_KNOTS
        c["sort_every"] = 0
        c["precision"] = _binding.FP64
        tube = _binding.Tube(c)
        if len(x):
            tube.inject(x, u)
        r = tube.adjoint_forward(int(n_steps), int(checkpoint_every))
        ctx.tube = tube                       # holds the recorded run and its tape until backward
        ctx.info = r
        ctx.device = knots.device
        return torch.tensor(r["loss"], dtype=torch.float64, device=knots.device)

    @staticmethod
    def backward(ctx, g):
        tube = ctx.tube
        r = tube.backward(float(g))
        tube.close()
        ctx.tube = None
        ctx.info.update(r)
        dev = ctx.device
        return (torch.as_tensor(r["g_knots"], dtype=torch.float64, device=dev),
                torch.tensor(r["g_kappa"], dtype=torch.float64, device=dev),
                torch.tensor(r["g_rate"], dtype=torch.float64, device=dev), None, None, None, None, None)


def exit_gamma_loss(knots, kappa, rate, cfg, x, u, n_steps, checkpoint_every=50):
    return ExitGammaLoss.apply(knots, kappa, rate, cfg, x, u, n_steps, checkpoint_every)
