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

    A device eps stays on the device: the library reads it and writes the
    FP64 gradient into a device tensor through device pointers, on torch's
    current stream (the handle is created on that stream).  A host eps goes
    through host buffers.
    """

    @staticmethod
    def forward(ctx, eps, Na, setup):
        kw = {k: v for k, v in setup.items()
              if k not in ("n", "gain", "box", "nsteps", "K", "init", "source")}
        dev = eps.is_cuda
        stream = torch.cuda.current_stream(eps.device).cuda_stream if dev else None
        sim = mbf.Sim(setup["n"], stream=stream, **kw)
        try:
            if dev:
                e = eps.detach().to(torch.float32).contiguous()
                g8 = torch.as_tensor(np.ascontiguousarray(setup["gain"], dtype=np.uint8), device=eps.device)
                sim.set_material(e, g8)
                grad = torch.empty(tuple(e.shape), dtype=torch.float64, device=eps.device)
            else:
                sim.set_material(np.ascontiguousarray(eps.detach().numpy(), dtype=np.float32),
                                 np.ascontiguousarray(setup["gain"], dtype=np.uint8))
                grad = np.zeros(tuple(eps.shape), dtype=np.float64)
            sim.set_pump(float(Na.detach()) if torch.is_tensor(Na) else float(Na), setup.get("init", "prepumped"))
            if setup.get("source") is not None:
                comp, i, j, k, amp = setup["source"]
                sim.set_source(comp, i, j, k, amp=amp)
            sim.set_loss_box(*setup["box"])
            L, gna = mbf.mbf_adjoint_run(sim.h, setup["nsteps"], setup.get("K", 50), grad)
        finally:
            sim.close()
        g = grad.to(eps.dtype) if dev else torch.from_numpy(grad).to(dtype=eps.dtype)
        ctx.save_for_backward(g, torch.tensor(gna, dtype=torch.float64))
        return torch.tensor(L, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gL):
        g, gna = ctx.saved_tensors
        return gL.to(g.dtype).to(g.device) * g, (gL.cpu() * gna).to(torch.float64), None


def loss_box_objective(eps, Na, setup):
    return LossBoxObjective.apply(eps, Na, setup)
