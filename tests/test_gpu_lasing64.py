"""GPU: a 64^3 random laser in the lasing regime over 78675 steps (3 ps, the
length of the paper's runs), FP32, against the oracle's run of the same
member (FP64 arithmetic, binary32 coefficients), stored by
tests/golden/make_lasing64.py.

The physics of the large batched workload at a size the oracle can run: RSA
spheres at fill 0.4 in the gain medium, the graded absorbing layer on every
wall, ground-state start at about twice the packing's threshold,
spontaneous-emission noise, 64 probes.  The field grows from the noise by
fourteen orders of magnitude, saturates and lases.  Compared: the probe-summed
emission spectrum (peak bin, standard deviation, Gaussian-fit width: the
linewidths of the Results section, Fig. 5b), the energy every 1000 steps, and
E at 1024 seeded sites.  In this model FP32 does not decorrelate from FP64
within the run (the sampled E stays within 1e-2); a second member with
another noise realization does decorrelate (E differs by more than 10%) and
must still lase in the same spectral bin.

The same sample pre-pumped at 3.2e26 m^-3, about 26 times its threshold
(tests/golden/make_lasing64.py --hot), is the strongest drive compared: the
field lases from the first steps, and FP32 still tracks the oracle over the
whole run (E within 2e-2; the same spectral criteria).  Against the library's
own FP64 path the FP32 run stays within 9e-3 there, so the model is driven by
its noise, not chaotic: no pump level tried makes rounding differences grow
exponentially."""
import json
import math
import os

import numpy as np
import pytest

from paper_0809_1547_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "lasing64_oracle.json")
GOLD_HOT = os.path.join(os.path.dirname(__file__), "golden", "lasing64_hot_oracle.json")


def _mbf():
    from paper_0809_1547_amd import mbf
    return mbf


def _run(mbf, gold, realization):
    r = gold["run"]
    n, steps = r["n"], r["steps"]
    eps, gain = I.voxelize(I.rsa_pack(n, seed=0, fill=0.4))
    probes = I.select_probes(eps, gain, r["probes"], seed=0)
    s = mbf.Sim(n, boundary="absorb", precision="fp32", seed=r["seed"], realization=realization,
                energy_history=steps)
    s.set_material(eps, gain)
    s.set_pump(r["Na"], r["init"])
    om = I.dft_omegas(*r["band_m"], steps, s.coefficients()[mbf.MBF_C_DT])
    assert np.allclose(om, gold["omega"], rtol=1e-12, atol=0.0)
    s.set_probes(probes, om, decim=32)
    s.step(steps)
    h = s.energy_history()
    E = [s.field(c) for c in range(3)]
    vals = np.array([float(E[c][k, j, i]) for c, i, j, k in gold["sample_sites"]])
    S = np.sum(np.abs(s.spectrum()) ** 2, axis=0)
    st = s.spectrum_stats(0.5)
    s.close()
    return h, vals, S, st


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as fh:
        return json.load(fh)


def test_lasing64_fp32_tracks_the_oracle(gold):
    mbf = _mbf()
    h, vals, S, st = _run(mbf, gold, 0)
    ref_vals = np.array(gold["sample_E"])
    ref_S = np.array(gold["power_spectrum"])
    ref = gold["stats"]
    W = h[999::1000]
    assert W[-1] > 1e12 * h[999]                       # grown from the noise and lasing
    rel_E = np.linalg.norm(vals - ref_vals) / np.linalg.norm(ref_vals)
    rel_S = np.linalg.norm(S - ref_S) / np.linalg.norm(ref_S)
    print(f"64^3 lasing: sampled E rel {rel_E:.2e}, spectrum rel {rel_S:.2e}; peak {st['peak_bin']} / "
          f"{int(ref['peak_bin'])}; std {st['std_omega']:.6e} / {ref['std_omega']:.6e}; "
          f"sigma {st['fit_sigma']:.5e} / {ref['fit_sigma']:.5e}")
    assert np.allclose(W, gold["energy_every_1000"], rtol=1e-2)
    assert rel_E < 1e-2
    assert rel_S < 1e-2
    assert abs(st["peak_bin"] - int(ref["peak_bin"])) <= 1
    assert st["std_omega"] == pytest.approx(ref["std_omega"], rel=0.02)
    assert st["fit_ok"] == int(ref["fit_ok"])
    if st["fit_ok"]:
        assert st["fit_sigma"] == pytest.approx(ref["fit_sigma"], rel=0.02)


def test_lasing64_another_realization_decorrelates_and_lases_in_the_same_bin(gold):
    mbf = _mbf()
    h, vals, S, st = _run(mbf, gold, 1)
    ref_vals = np.array(gold["sample_E"])
    rel_E = np.linalg.norm(vals - ref_vals) / np.linalg.norm(ref_vals)
    print(f"realization 1: sampled E rel {rel_E:.2e}; peak {st['peak_bin']} / {int(gold['stats']['peak_bin'])}; "
          f"std {st['std_omega']:.6e} / {gold['stats']['std_omega']:.6e}")
    assert h[-1] > 1e12 * h[999]
    assert rel_E > 0.1
    assert abs(st["peak_bin"] - int(gold["stats"]["peak_bin"])) <= 1


def test_lasing64_far_above_threshold_fp32_tracks_the_oracle():
    mbf = _mbf()
    with open(GOLD_HOT) as fh:
        gold = json.load(fh)
    assert gold["run"]["init"] == "prepumped" and gold["run"]["Na"] == 3.2e26
    h, vals, S, st = _run(mbf, gold, 0)
    ref_vals = np.array(gold["sample_E"])
    ref_S = np.array(gold["power_spectrum"])
    ref = gold["stats"]
    W = h[999::1000]
    rel_E = np.linalg.norm(vals - ref_vals) / np.linalg.norm(ref_vals)
    rel_S = np.linalg.norm(S - ref_S) / np.linalg.norm(ref_S)
    rel_W = float(np.max(np.abs(W - np.array(gold["energy_every_1000"])) / np.array(gold["energy_every_1000"])))
    print(f"64^3 at 3.2e26: sampled E rel {rel_E:.2e}, spectrum rel {rel_S:.2e}, energy rel {rel_W:.2e}; "
          f"peak {st['peak_bin']} / {int(ref['peak_bin'])}; std {st['std_omega']:.6e} / {ref['std_omega']:.6e}")
    assert rel_W < 1e-2
    assert rel_E < 2e-2
    assert rel_S < 1e-2
    assert abs(st["peak_bin"] - int(ref["peak_bin"])) <= 1
    assert st["std_omega"] == pytest.approx(ref["std_omega"], rel=0.02)
    assert st["fit_ok"] == int(ref["fit_ok"])
    if st["fit_ok"]:
        assert st["fit_sigma"] == pytest.approx(ref["fit_sigma"], rel=0.02)
