"""GPU: the Gross-Pitaevskii bound states of the random laser (Gross-
Pitaevskii section, Eqs. g5, ee, s1) through the C ABI against the oracle's
solution of the same discrete problem."""
import math

import numpy as np
import pytest

from oracle import gp as OG

pytestmark = pytest.mark.gpu

ES = [1.001, 1.01, 1.1, 1.5, 2.0, 3.0, 5.0, 10.0, 30.0]


def _mbf():
    from paper_0809_1547_amd import mbf
    return mbf


@pytest.mark.parametrize("M,L", [(1023, 12.0), (255, 10.0), (100, 9.0)])
def test_bound_states_match_oracle(M, L):
    mbf = _mbf()
    g = mbf.mbf_gp_solve(ES, M=M, L=L, n_nu=300, dnu=0.03)
    for q, E in enumerate(ES):
        o = OG.gp_solve(E, M, L, 300, 0.03)
        assert g["converged"][q] == 1.0, E
        scale = float(np.max(o["phi"]))
        assert np.max(np.abs(g["phi"][q] - o["phi"])) <= 1e-9 * scale, E
        for key in ("N", "w", "peak", "phi_max"):
            assert g[key][q] == pytest.approx(o[key], rel=1e-9), (E, key)
        assert g["residual"][q] <= 1e-8 * (4.0 * scale * (M + 1) ** 2 / (2 * L) ** 2 + 1.0)
        assert np.max(np.abs(g["spec"][q] - o["spec"])) <= 1e-9 * float(np.max(o["spec"]))


def test_threshold_and_eigenvalue_closed_forms():
    mbf = _mbf()
    for kappa in (1e-3, 0.1, 0.14, 1.0):
        p = mbf.mbf_gp_threshold(kappa)
        assert p == pytest.approx(OG.threshold(kappa), rel=1e-15)
        assert mbf.mbf_gp_eigenvalue(p, kappa) == pytest.approx(1.0, rel=1e-13)


def test_linewidth_against_pump():
    # the waist W ~ w(E(p)) sqrt(kappa) / p^{1/4} narrows above threshold
    mbf = _mbf()
    kappa = 0.14
    ps = mbf.mbf_gp_threshold(kappa) * np.array([1.02, 1.1, 1.3, 2.0, 4.0])
    E = np.array([mbf.mbf_gp_eigenvalue(p, kappa) for p in ps])
    g = mbf.mbf_gp_solve(E, M=1023, L=14.0, n_nu=600, dnu=0.02)
    W = g["w"] * math.sqrt(kappa) / ps ** 0.25
    assert np.all(np.diff(W) < 0.0) and np.all(g["converged"] == 1.0)


def test_bad_arguments():
    mbf = _mbf()
    for kw in (dict(E=[1.0]), dict(E=[0.5]), dict(E=[2.0], M=2), dict(E=[2.0], M=2000),
               dict(E=[2.0], L=-1.0), dict(E=[2.0], n_nu=0), dict(E=[float("nan")])):
        E = kw.pop("E")
        with pytest.raises(mbf.MbfError):
            mbf.mbf_gp_solve(E, **kw)
