"""Writes pulse128_oracle.json: the oracle's passive-pulse run of the 128^3
sample, the reference of the 128^3 passive-pulse parity test.

Test infrastructure: calls only the oracle (FP64 arithmetic, coefficients
rounded once to binary32 as the FP32 library forms them) and the seeded input
generators.  About 3 minutes on 8 cores:

    python tests/golden/make_pulse128.py

The run (the passive spectrum of the Simulations section, Fig. 1, on the
128^3 workload): RSA spheres (d = 300 nm, eps_r = 8.41, fill 0.4, seed 0) in
a background of eps_r = 1 without gain, the graded absorbing layer on every
wall, the single-cycle 532 nm soft pulse (tau_p = 1 fs) on E_z at the void
site nearest the centre, 5000 steps (0.19 ps); running DFT of E at 64 seeded
void probe sites over 450-800 nm at the run's resolution.  Stored: the probe
spectra, the energy every 100 steps, and E at 1024 seeded sites after 1000,
2500 and 5000 steps.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O                                   # noqa: E402
from paper_0809_1547_amd import inputs as I          # noqa: E402

N, STEPS = 128, 5000
CHECKPOINTS = (1000, 2500, 5000)
N_PROBES, N_SAMPLES = 64, 1024
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pulse128_oracle.json")


def setup():
    eps, void = I.voxelize(I.packing_for("c2", N, 0))
    src = I.nearest_void_site(void)
    probes = I.select_probes(eps, void, N_PROBES, seed=1)
    return eps, np.zeros_like(void), src, probes


def r12(x):
    # 12 significant digits: far below the parity tolerance, a third of the
    # file of full precision
    return float(f"{x:.12g}")


def sample_sites():
    # interior E-sites (comp, i, j, k), seeded
    g = np.random.Generator(np.random.PCG64([0, 128, 7]))
    return [[int(g.integers(0, 3))] + [int(v) for v in g.integers(1, N, size=3)] for _ in range(N_SAMPLES)]


def main():
    eps, gain, src, probes = setup()
    o = O.Oracle(O.default_params(N, bc=(O.ABSORB,) * 3, round_f32=True, noise=False))
    o.set_material(eps, gain)
    o.set_pump(0.0, O.GROUND)
    o.set_source(*[int(v) for v in src], amp=1.0)
    dt = o.coefficients()[O.C_DT]
    om = I.dft_omegas(450e-9, 800e-9, STEPS, dt)
    o.set_probes(probes, om)
    sites = sample_sites()
    energy, samples = [], {}
    for s in range(STEPS // 100):
        o.step(100)
        energy.append(o.energy()[0])
        if o.step_index in CHECKPOINTS:
            E = [o.field(c) for c in range(3)]
            samples[str(o.step_index)] = [r12(E[c][k, j, i]) for c, i, j, k in sites]
            print(f"step {o.step_index}: W = {energy[-1]:.6e}", flush=True)
    F = o.spectrum()
    o.close()
    doc = {
        "run": {"n": N, "steps": STEPS, "boundary": "absorb", "source": [int(v) for v in src],
                "packing": "c2 seed 0", "probes": N_PROBES, "band_m": [450e-9, 800e-9]},
        "omega": [float(w) for w in om],
        "spectrum_re": [[r12(v) for v in row] for row in F.real],
        "spectrum_im": [[r12(v) for v in row] for row in F.imag],
        "energy_every_100": [r12(v) for v in energy],
        "sample_sites": sites,
        "sample_E": samples,
    }
    with open(OUT, "w") as fh:
        json.dump(doc, fh, separators=(",", ":"))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
