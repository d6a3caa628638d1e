"""Lasing threshold of each packing from a batched pump sweep (Results
section, Fig. 5b, where the linewidth collapses above threshold; the
operational reading: the energy of the least-damped mode grows or decays
exponentially in the linear interval at a rate that is close to linear in
N_a near threshold, and N_th is the root of that line).

Orchestration only: the runs are one batched launch sequence of the HIP
library, and the growth rates and the line fit are mbf_growth_threshold.
This module chooses the pump levels and reads the histories back.

Each member starts from the prepumped state with no noise and is excited by
one soft pulse at the gain centre in the middle of the box.  A pulse with no
DC content leaves no static field, whose undamped energy would otherwise hide
the decay of the lasing mode below threshold.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np

from . import mbf

# pass 1: a geometric ladder of pump densities [m^-3]; pass 2: REFINE levels
# spread evenly over the bracket that pass 1 finds
LADDER = tuple(4e24 * 2.0 ** j for j in range(5))
REFINE = 3


MAX_MEMBERS = 255        # members of one batch


def _run(mats, sizes, levels, *, boundary, steps, window, amp, lambda_s, stream, phys):
    """Growth rates (R, L) and fits [(a, b, N_th)] of R packings at levels
    (R, L): R*L members, in batches of at most MAX_MEMBERS."""
    R, L = len(sizes), len(levels[0])
    per = max(1, MAX_MEMBERS // L)
    rates = np.zeros((R, L))
    fits = []
    for r0 in range(0, R, per):
        rr = range(r0, min(R, r0 + per))
        cfgs = [mbf.make_config(sizes[r], boundary=boundary, noise=False, seed=0, realization=r,
                                energy_history=steps, **phys)
                for r in rr for _ in range(L)]
        b = mbf.Batch(cfgs, stream=stream)
        try:
            for q, r in enumerate(rr):
                c = sizes[r] // 2
                for j in range(L):
                    s = b[q * L + j]
                    s.set_material(*mats[r])
                    s.set_pump(float(levels[r][j]), "prepumped")
                    s.set_source(2, c, c, c, amp=amp, lambda_s=lambda_s)
            b.step(steps)
            b.sync()
            for q, r in enumerate(rr):
                hist = np.stack([b[q * L + j].energy_history() for j in range(L)])
                rates[r], fit = mbf.mbf_growth_threshold(hist, np.asarray(levels[r], dtype=np.float64), *window)
                fits.append(fit)
        finally:
            b.close()
    return rates, fits


def packing_thresholds(mats: Sequence[Tuple[np.ndarray, np.ndarray]], sizes: Sequence[int], *,
                       boundary="absorb", steps: int = 3000, window=(1500, 3000), amp: float = 1e-3,
                       lambda_s: float = 590e-9, ladder=LADDER, stream=None, **phys):
    """N_th of each packing (mats[r] = (eps, gain) on a sizes[r]^3 grid).

    Pass 1 runs every packing at each density of `ladder` and takes the first
    density with a positive growth rate and the one below it (0 below the
    first) as a bracket; pass 2 runs REFINE densities spread evenly over the
    bracket, fits the line and takes its root, kept inside the bracket (the
    bracket's midpoint when the line is flat).
    Returns (N_th per packing, details dict).  Raises ValueError when a
    packing grows at no density of the ladder."""
    R = len(sizes)
    lad = np.asarray(ladder, dtype=np.float64)
    r1, _ = _run(mats, sizes, [lad] * R, boundary=boundary, steps=steps, window=window, amp=amp,
                 lambda_s=lambda_s, stream=stream, phys=phys)
    brackets = []
    for r in range(R):
        up = np.nonzero(r1[r] > 0)[0]
        if up.size == 0:
            raise ValueError(f"packing {r} ({sizes[r]}^3) does not grow up to N_a = {lad[-1]:.3g}")
        j = int(up[0])
        brackets.append((lad[j - 1] if j else 0.0, lad[j]))
    lv2 = [np.linspace(lo if lo > 0 else 0.25 * hi, hi, REFINE) for lo, hi in brackets]
    r2, fits = _run(mats, sizes, lv2, boundary=boundary, steps=steps, window=window, amp=amp,
                    lambda_s=lambda_s, stream=stream, phys=phys)
    # the root, kept inside the bracket (its midpoint if the line is flat)
    nth = np.array([min(max(f[2], lo), hi) if np.isfinite(f[2]) else 0.5 * (lo + hi)
                    for f, (lo, hi) in zip(fits, brackets)])
    return nth, {"ladder": lad, "ladder_rates": r1, "brackets": brackets, "levels": lv2, "rates": r2,
                 "fits": fits}
