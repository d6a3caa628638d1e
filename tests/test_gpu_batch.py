"""GPU: batched stepping of realizations of different sizes (one launch per
kernel for all members) against the same members stepped alone, and one
member against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from paper_0809_1547_amd import inputs as I

pytestmark = pytest.mark.gpu

MEMBERS = [
    dict(n=(24, 20, 18), boundary="pec", seed=1, realization=0, Na=2e24, src=True, probes=True),
    dict(n=(33, 17, 29), boundary="absorb", seed=1, realization=1, Na=3e24, src=False, probes=True),
    dict(n=(16, 16, 16), boundary=("mur", "pec", "mur"), seed=5, realization=2, Na=1e24, src=True, probes=False),
    dict(n=(70, 12, 9), boundary="absorb", seed=2, realization=7, Na=5e24, src=False, probes=False),
]


def _mbf():
    from paper_0809_1547_amd import mbf
    return mbf


def _setup(sim, spec, r):
    mbf = _mbf()
    eps, gain = I.voxelize(I.rsa_pack(spec["n"], seed=10 + r, fill=0.35))
    sim.set_material(eps, gain)
    sim.set_pump(spec["Na"])
    if spec["src"]:
        sim.set_source(*I.nearest_void_site(gain), amp=0.2)
    if spec["probes"]:
        probes = I.select_probes(eps, gain, 6, seed=r)
        dt = sim.coefficients()[mbf.MBF_C_DT]
        sim.set_probes(probes, I.dft_omegas(450e-9, 800e-9, 400, dt), decim=16)
    sim.set_loss_box((1, 1, 1), (5, 6, 7))


def _cfg(spec, hist):
    mbf = _mbf()
    return mbf.make_config(spec["n"], boundary=spec["boundary"], seed=spec["seed"],
                           realization=spec["realization"], energy_history=hist, E_sp=1e-3)


def _snapshot(sim, probes):
    out = [sim.field(f) for f in range(21)]
    out.append(np.array(sim.energy()))
    out.append(sim.energy_history())
    out.append(np.array([sim.loss()]))
    if probes:
        out.append(sim.spectrum())
    return out


@pytest.mark.parametrize("variant,group_mb,remap", [("two_pass", 0, 2), ("fused", 0, 2), ("two_pass", 1, 2),
                                                     ("fused", 2, 1), ("two_pass", 0, 0), ("two_pass_split", 0, 2),
                                                     ("two_pass_split", 1, 1), ("fused_lds", 0, 2),
                                                     ("fused_lds", 1, 1), ("fused_persistent", 0, 2),
                                                     ("fused_persistent", 1, 1)])
def test_batch_members_equal_solo_runs(variant, group_mb, remap):
    # group_mb 1 and 2 split the members into groups that run whole graph
    # chunks one after the other
    mbf = _mbf()
    hist = 120
    batch = mbf.Batch([_cfg(s, hist) for s in MEMBERS])
    batch.set_tuning(variant, tile_y=4, zseg=4, xcd_remap=remap, group_mb=group_mb)
    for r, s in enumerate(MEMBERS):
        _setup(batch[r], s, r)
    batch.step(3)          # unaligned start: single batched steps
    batch.step(100)        # then graph chunks of 16 (the shared probe decimation)
    got = [_snapshot(batch[r], s["probes"]) for r, s in enumerate(MEMBERS)]
    assert all(batch[r].step_index == 103 for r in range(len(MEMBERS)))
    for r, s in enumerate(MEMBERS):
        solo = mbf.Sim(None, _cfg=_cfg(s, hist))
        solo.set_tuning(variant, tile_y=4, zseg=4, xcd_remap=remap)
        _setup(solo, s, r)
        solo.step(103)
        ref = _snapshot(solo, s["probes"])
        for q, (a, b) in enumerate(zip(got[r], ref)):
            assert np.array_equal(a, b), (r, q)
        solo.close()
    batch.close()


def test_batch_member_matches_oracle():
    mbf = _mbf()
    spec = MEMBERS[1]
    batch = mbf.Batch([_cfg(s, 0) for s in MEMBERS[:2]])
    for r, s in enumerate(MEMBERS[:2]):
        _setup(batch[r], s, r)
    ora = O.Oracle(O.default_params(spec["n"], bc=(O.ABSORB,) * 3, round_f32=True, seed=spec["seed"],
                                    realization=spec["realization"], E_sp=1e-3))
    eps, gain = I.voxelize(I.rsa_pack(spec["n"], seed=11, fill=0.35))
    ora.set_material(eps, gain)
    ora.set_pump(spec["Na"], O.PREPUMPED)
    for _ in range(3):
        batch.step(40)
        ora.step(40)
        m = batch[1]
        for grp in ((0, 1, 2), (3, 4, 5), (6, 7, 8)):
            num = sum(float(np.sum((m.field(f).astype(np.float64) - ora.field(f)) ** 2)) for f in grp)
            den = sum(float(np.sum(ora.field(f) ** 2)) for f in grp)
            assert np.sqrt(num / den) <= 1e-5, grp
    batch.close()


def test_batch_with_different_probe_decimations_and_errors():
    mbf = _mbf()
    specs = MEMBERS[:2]
    batch = mbf.Batch([_cfg(s, 0) for s in specs])
    with pytest.raises(mbf.MbfError) as err:
        batch.step(1)                       # no material yet
    assert err.value.code == mbf.MBF_ESTATE
    for r, s in enumerate(specs):
        _setup(batch[r], s, r)
    dt = batch[1].coefficients()[mbf.MBF_C_DT]
    eps, gain = I.voxelize(I.rsa_pack(specs[1]["n"], seed=11, fill=0.35))
    batch[1].set_probes(I.select_probes(eps, gain, 6, seed=1), I.dft_omegas(450e-9, 800e-9, 400, dt), decim=8)
    batch.step(40)                          # decimations differ: single batched steps
    for r, s in enumerate(specs):
        solo = mbf.Sim(None, _cfg=_cfg(s, 0))
        _setup(solo, s, r)
        if r == 1:
            solo.set_probes(I.select_probes(eps, gain, 6, seed=1), I.dft_omegas(450e-9, 800e-9, 400, dt), decim=8)
        solo.step(40)
        assert np.array_equal(solo.spectrum(), batch[r].spectrum())
        assert np.array_equal(solo.field(0), batch[r].field(0))
        solo.close()
    batch.close()


def test_autotune_keeps_the_trajectory():
    # trials run on the live state, which is restored afterwards: the run
    # continues exactly as a run that was given the chosen schedule directly
    mbf = _mbf()
    spec = MEMBERS[0]
    a = mbf.Sim(None, _cfg=_cfg(spec, 80))
    _setup(a, spec, 0)
    a.step(13)
    chosen = a.autotune(budget_ms=300)
    assert a.step_index == 13
    a.step(60)
    b = mbf.Sim(None, _cfg=_cfg(spec, 80))
    _setup(b, spec, 0)
    b.step(13)                 # energy sums follow the schedule: switch at the same step
    b.set_tuning(**chosen)
    b.step(60)
    for x, y in zip(_snapshot(a, True), _snapshot(b, True)):
        assert np.array_equal(x, y)
    a.close()
    b.close()
    batch = mbf.Batch([_cfg(s, 40) for s in MEMBERS])
    for r, s in enumerate(MEMBERS):
        _setup(batch[r], s, r)
    batch.step(5)
    first = batch.tuning()
    chosen = batch.autotune(budget_ms=300)
    assert batch.tuning() == chosen
    batch.step(35)
    for r, s in enumerate(MEMBERS):
        solo = mbf.Sim(None, _cfg=_cfg(s, 40))
        _setup(solo, s, r)
        solo.set_tuning(**first)   # a single grid's own default may cut it finer than a batch's
        solo.step(5)
        solo.set_tuning(**chosen)
        solo.step(35)
        for x, y in zip(_snapshot(batch[r], s["probes"]), _snapshot(solo, s["probes"])):
            assert np.array_equal(x, y), r
        solo.close()
    batch.close()


def test_member_schedule_change_does_not_break_batched_steps():
    # a member whose own schedule differs from the batch's is still stepped
    # whole by the batched kernels (geometry follows the batch's schedule)
    mbf = _mbf()
    batch = mbf.Batch([_cfg(s, 0) for s in MEMBERS])
    batch.set_tuning("two_pass", tile_y=4, zseg=4)
    for r, s in enumerate(MEMBERS):
        _setup(batch[r], s, r)
    batch[1].set_tuning("fused", tile_y=16, zseg=2)
    batch.step(40)
    for r, s in enumerate(MEMBERS):
        solo = mbf.Sim(None, _cfg=_cfg(s, 0))
        _setup(solo, s, r)
        solo.step(40)
        for f in range(21):
            assert np.array_equal(batch[r].field(f), solo.field(f)), (r, f)
        solo.close()
    batch.close()


def test_default_schedule_follows_grid_size():
    # the split two-pass variant over 2-plane segments from 4 Mi cells on,
    # the whole-plane two-pass variant below, over the longest of 4, 2 and 1
    # planes that still makes 1024 work items of 64 x 4 columns (the tuning
    # reads back the segment length in effect); a batch goes by its largest
    # member
    mbf = _mbf()
    for n, want, zs in (((32, 32, 32), "two_pass", 1), ((64, 64, 64), "two_pass", 1),
                        ((64, 64, 128), "two_pass", 2), ((80, 80, 80), "two_pass", 2),
                        ((96, 96, 96), "two_pass", 4), ((65, 64, 256), "two_pass", 4),
                        ((160, 160, 163), "two_pass", 4),
                        ((160, 160, 164), "two_pass_split", 2), ((320, 320, 320), "two_pass_split", 2)):
        s = mbf.Sim(n)
        t = s.tuning()
        assert (t["variant"], t["tile_y"], t["zseg"], t["xcd_remap"]) == (want, 4, zs, 2), (n, t)
        s.close()
    b = mbf.Batch([mbf.make_config(m) for m in ((48, 48, 48), (160, 160, 164), (64, 64, 64))])
    assert b.tuning()["variant"] == "two_pass_split" and all(b[r].tuning()["variant"] == "two_pass_split"
                                                               for r in range(3))
    b.close()


def test_autotune_choice_is_persisted(tmp_path, monkeypatch):
    # with MBF_TUNE_CACHE set, the first autotune of a shape times the
    # candidates and appends its choice; a second handle of the same shape
    # (and architecture, precision, walls) takes it from the file without
    # timing; another shape gets a line of its own; batches likewise
    mbf = _mbf()
    cache = tmp_path / "tuning.txt"
    monkeypatch.setenv("MBF_TUNE_CACHE", str(cache))

    def sim(n):
        s = mbf.Sim(n, boundary="absorb")
        eps, gain = I.voxelize(I.rsa_pack(n, seed=3, fill=0.3))
        s.set_material(eps, gain)
        s.set_pump(2e24)
        return s
    a = sim((40, 36, 28))
    ta = a.autotune(budget_ms=200)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and "40x36x28" in lines[0] and "single" in lines[0]
    # plant another schedule for this key: the next handle must take it
    planted = {**ta, "variant": "fused" if ta["variant"] != "fused" else "two_pass", "tile_y": 8, "zseg": 3}
    vid = {"two_pass": 0, "fused": 1, "two_pass_split": 2, "fused_lds": 3}[planted["variant"]]
    key = lines[0].split("\t")[0]
    with open(cache, "a") as f:
        f.write(f"{key}\t{vid} 8 3 {ta['xcd_remap']} {ta['group_mb']}\n")
    b = sim((40, 36, 28))
    tb = b.autotune(budget_ms=200)
    assert (tb["variant"], tb["tile_y"], tb["zseg"]) == (planted["variant"], 8, 3)
    assert len(cache.read_text().splitlines()) == 2               # nothing timed, nothing added
    c = sim((36, 36, 28))
    c.autotune(budget_ms=200)
    assert len(cache.read_text().splitlines()) == 3
    for s in (a, b, c):
        s.close()
    cfgs = [mbf.make_config(n, boundary="absorb") for n in ((24, 20, 16), (32, 20, 16))]
    bt = mbf.Batch(cfgs)
    for r, s in enumerate(bt.members):
        eps, gain = I.voxelize(I.rsa_pack(s.n, seed=r, fill=0.3))
        s.set_material(eps, gain)
        s.set_pump(2e24)
    t1 = bt.autotune(budget_ms=200)
    assert len(cache.read_text().splitlines()) == 4 and "batch" in cache.read_text().splitlines()[-1]
    assert bt.autotune(budget_ms=200) == t1
    assert len(cache.read_text().splitlines()) == 4
    bt.close()
