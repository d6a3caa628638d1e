"""GPU: the passive spectrum of the 128^3 workload (Simulations section,
Fig. 1: a single-cycle 532 nm pulse in the passive sample) over 5000 steps,
FP32, against the oracle's run stored by tests/golden/make_pulse128.py.

RSA spheres at fill 0.4 in a background without gain, the graded absorbing
layer on every wall, the soft pulse on E_z at the void site nearest the
centre, 64 void probes.  The pulse spreads through the sample and leaves
through the layer, so E is compared against the largest norm its samples
reached (the field's own norm goes to zero), the spectra against their own
norm, and the energy against the largest energy of the run."""
import json
import os

import numpy as np
import pytest

from paper_0809_1547_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "pulse128_oracle.json")
TOL32 = 1e-5


def test_pulse128_fp32_matches_the_oracle():
    from paper_0809_1547_amd import mbf
    with open(GOLD) as fh:
        gold = json.load(fh)
    r = gold["run"]
    n, steps = r["n"], r["steps"]
    eps, void = I.voxelize(I.packing_for("c2", n, 0))
    src = I.nearest_void_site(void)
    assert list(src) == r["source"]
    probes = I.select_probes(eps, void, r["probes"], seed=1)
    s = mbf.Sim(n, boundary="absorb", precision="fp32", noise=False)
    s.set_material(eps, np.zeros_like(void))
    s.set_pump(0.0, "ground")
    s.set_source(*src, amp=1.0)
    om = I.dft_omegas(*r["band_m"], steps, s.coefficients()[mbf.MBF_C_DT])
    assert np.allclose(om, gold["omega"], rtol=1e-12, atol=0.0)
    s.set_probes(probes, om, decim=32)
    sites = gold["sample_sites"]
    energy, errs, peak = [], {}, 0.0
    for q in range(steps // 100):
        s.step(100)
        energy.append(s.energy()[0])
        key = str(s.step_index)
        if key in gold["sample_E"]:
            E = [s.field(c) for c in range(3)]
            v = np.array([float(E[c][k, j, i]) for c, i, j, k in sites])
            ref = np.array(gold["sample_E"][key])
            peak = max(peak, float(np.linalg.norm(ref)))
            errs[key] = float(np.linalg.norm(v - ref)) / peak
    F = s.spectrum()
    s.close()
    Fo = np.array(gold["spectrum_re"]) + 1j * np.array(gold["spectrum_im"])
    rel_F = float(np.linalg.norm(F - Fo) / np.linalg.norm(Fo))
    eo = np.array(gold["energy_every_100"])
    rel_W = float(np.max(np.abs(np.array(energy) - eo)) / np.max(eo))
    print(f"128^3 pulse: sampled E / peak norm {errs}; spectra {rel_F:.2e}; energy {rel_W:.2e}")
    assert eo.argmax() < len(eo) - 1 and eo[-1] < 0.1 * eo.max()      # the pulse leaves the box
    assert max(errs.values()) <= TOL32
    assert rel_F <= TOL32
    assert rel_W <= TOL32
