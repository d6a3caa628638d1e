"""Host logic of the per-packing threshold sweep (no GPU): the bracket taken
from the ladder's growth rates, the refined densities, the root kept inside
the bracket, and the error when a packing grows nowhere on the ladder.  The
batched runs are replaced by a linear rate law per packing."""
import numpy as np
import pytest

from paper_0809_1547_amd import sweep


def _fake_run(slopes, roots, calls):
    # rates b (N_a - root) at every level; the fit is that line
    def run(mats, sizes, levels, **kw):
        calls.append([np.array(lv, dtype=float) for lv in levels])
        rates = np.array([[b * (na - r0) for na in lv] for b, r0, lv in zip(slopes, roots, levels)])
        fits = [(-b * r0, b, r0) for b, r0 in zip(slopes, roots)]
        return rates, fits
    return run


def test_bracket_refine_and_root(monkeypatch):
    roots = [5e24, 3.3e25, 1e23]
    calls = []
    monkeypatch.setattr(sweep, "_run", _fake_run([1e-28] * 3, roots, calls))
    nth, d = sweep.packing_thresholds([None] * 3, [48, 64, 80])
    lad = np.array(sweep.LADDER)
    assert np.array_equal(calls[0][0], lad) and len(calls) == 2
    # first ladder density that grows, and the one below it (0 below the first)
    assert d["brackets"][0] == (4e24, 8e24)
    assert d["brackets"][1] == (32e24, 64e24)
    assert d["brackets"][2] == (0.0, 4e24)
    # three densities over the bracket (from a quarter of its top when it starts at 0)
    assert np.allclose(calls[1][0], [4e24, 6e24, 8e24])
    assert np.allclose(calls[1][2], [1e24, 2.5e24, 4e24])
    # the root, clamped into the bracket: the third packing's 1e23 sits below
    # its bracket's refined range but inside [0, 4e24]
    assert np.allclose(nth, roots)


def test_root_outside_the_bracket_is_clamped_and_a_flat_line_takes_the_midpoint(monkeypatch):
    calls = []

    def run(mats, sizes, levels, **kw):
        calls.append(levels)
        if len(calls) == 1:      # the ladder: grows from 16e24 on
            return np.array([[-1.0, -1.0, -1.0, 1.0, 1.0]] * 2), [(0.0, 1.0, 0.0)] * 2
        return np.zeros((2, 3)), [(1.0, 1e-30, -1e30), (0.0, 0.0, float("nan"))]
    monkeypatch.setattr(sweep, "_run", run)
    nth, d = sweep.packing_thresholds([None] * 2, [48, 48])
    assert d["brackets"] == [(16e24, 32e24)] * 2
    assert nth[0] == 16e24                   # a root far below: the bracket's bottom
    assert nth[1] == 24e24                   # no root: the bracket's midpoint


def test_no_growth_on_the_ladder_raises(monkeypatch):
    monkeypatch.setattr(sweep, "_run", _fake_run([1e-28], [1e27], []))
    with pytest.raises(ValueError, match="does not grow"):
        sweep.packing_thresholds([None], [48])
