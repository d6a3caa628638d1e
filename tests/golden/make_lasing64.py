"""Writes lasing64_oracle.json: the oracle's lasing run of a 64^3 random
laser, the reference of the 64^3 lasing-regime parity test; with --hot,
lasing64_hot_oracle.json, the same sample pre-pumped at N_a = 3.2e26 m^-3
(about 26 times its threshold).

Test infrastructure: calls only the oracle (FP64 arithmetic, coefficients
rounded once to binary32 as the FP32 library forms them) and the seeded input
generators.  About 16 minutes on 8 cores each:

    python tests/golden/make_lasing64.py
    python tests/golden/make_lasing64.py --hot

The run: 64^3 cells of 20 nm, RSA spheres (d = 300 nm, eps_r = 8.41, fill
0.4, seed 0) in the gain medium, the graded absorbing layer on every wall,
ground-state start at N_a = 2.5e25 m^-3 (about twice the threshold of this
packing), spontaneous-emission noise at the default
amplitude (seed 0, realization 0), 78675 steps (3 ps, the length of the paper's
runs); running DFT of E at
64 seeded probe sites over 450-800 nm at the run's resolution.  Stored: the
probe-summed power spectrum, its statistics, the energy every 1000 steps and
E at 1024 seeded sites after the last step.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O                                   # noqa: E402
from oracle import spectra as OS                     # noqa: E402
from paper_0809_1547_amd import inputs as I          # noqa: E402

N, STEPS = 64, 78675
N_PROBES, N_SAMPLES = 64, 1024
HOT = "--hot" in sys.argv[1:]
# (N_a, start): twice the packing's threshold from the ground state, or 26
# times it pre-pumped
NA, INIT = (3.2e26, "prepumped") if HOT else (2.5e25, "ground")
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                   "lasing64_hot_oracle.json" if HOT else "lasing64_oracle.json")


def setup():
    eps, gain = I.voxelize(I.rsa_pack(N, seed=0, fill=0.4))
    probes = I.select_probes(eps, gain, N_PROBES, seed=0)
    return eps, gain, probes


def sample_sites():
    # interior E-sites (comp, i, j, k), seeded
    g = np.random.Generator(np.random.PCG64([0, 64, 7]))
    out = []
    while len(out) < N_SAMPLES:
        c = int(g.integers(0, 3))
        ijk = [int(v) for v in g.integers(1, N, size=3)]
        out.append([c] + ijk)
    return out


def main():
    eps, gain, probes = setup()
    o = O.Oracle(O.default_params(N, bc=(O.ABSORB,) * 3, round_f32=True, seed=0, realization=0))
    o.set_material(eps, gain)
    o.set_pump(NA, O.PREPUMPED if INIT == "prepumped" else O.GROUND)
    dt = o.coefficients()[O.C_DT]
    om = I.dft_omegas(450e-9, 800e-9, STEPS, dt)
    o.set_probes(probes, om)
    energy = []
    for c in range(STEPS // 1000):
        o.step(1000)
        energy.append(o.energy()[0])
        print(f"step {(c + 1) * 1000}: W = {energy[-1]:.6e}", flush=True)
    o.step(STEPS % 1000)
    F = o.spectrum()
    stats = OS.spectral_stats(F, om, 0.5)
    sites = sample_sites()
    E = [o.field(c) for c in range(3)]
    values = [float(E[c][k, j, i]) for c, i, j, k in sites]
    o.close()
    doc = {
        "run": {"n": N, "steps": STEPS, "Na": NA, "init": INIT, "boundary": "absorb", "seed": 0,
                "realization": 0, "packing": "rsa seed 0 fill 0.4", "probes": N_PROBES,
                "band_m": [450e-9, 800e-9]},
        "omega": [float(w) for w in om],
        "power_spectrum": [float(s) for s in OS.power_spectrum(F)],
        "stats": {k: float(v) for k, v in stats.items()},
        "energy_every_1000": energy,
        "sample_sites": sites,
        "sample_E": values,
    }
    with open(OUT, "w") as fh:
        json.dump(doc, fh, separators=(",", ":"))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
