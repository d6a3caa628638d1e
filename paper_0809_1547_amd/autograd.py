"""torch.autograd binding of the loss-box adjoint (argument marshalling only:
the forward run and the reverse sweep are mbf_adjoint_run in the HIP
library)."""
from __future__ import annotations

import numpy as np
import torch

from . import mbf


class LossBoxObjective(torch.autograd.Function):
    """L(eps_r, N_a) = sum over steps n = 1..nsteps of sum over the interior
    E-sites of the loss box of (E^n)^2, for a run that starts from the pump.

    forward(eps, Na, setup): eps is the per-cell eps_r map (nz, ny, nx), Na a
    scalar tensor in m^-3; setup is a dict with the grid and run description:
      n, gain (uint8 map), box ((i0, j0, k0), (i1, j1, k1)), nsteps, K,
      init ("prepumped" or "ground"), source (optional (comp, i, j, k, amp)),
      and any mbf.make_config keyword (boundary, precision, seed, ...).
    backward returns dL/d eps (same shape, dtype and device as eps) and dL/dNa.
    """

    @staticmethod
    def forward(ctx, eps, Na, setup):
        kw = {k: v for k, v in setup.items()
              if k not in ("n", "gain", "box", "nsteps", "K", "init", "source")}
        sim = mbf.Sim(setup["n"], **kw)
        try:
            sim.set_material(np.ascontiguousarray(eps.detach().cpu().numpy(), dtype=np.float32),
                             np.ascontiguousarray(setup["gain"], dtype=np.uint8))
            sim.set_pump(float(Na), setup.get("init", "prepumped"))
            if setup.get("source") is not None:
                comp, i, j, k, amp = setup["source"]
                sim.set_source(comp, i, j, k, amp=amp)
            sim.set_loss_box(*setup["box"])
            L, g, gna = sim.adjoint_run(setup["nsteps"], K=setup.get("K", 50))
        finally:
            sim.close()
        ctx.save_for_backward(torch.from_numpy(g).to(device=eps.device, dtype=eps.dtype),
                              torch.tensor(gna, dtype=torch.float64))
        return torch.tensor(L, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gL):
        g, gna = ctx.saved_tensors
        return gL.to(g.dtype).to(g.device) * g, (gL.cpu() * gna).to(torch.float64), None


def loss_box_objective(eps, Na, setup):
    return LossBoxObjective.apply(eps, Na, setup)
