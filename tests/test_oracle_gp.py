"""Pins of the oracle's Gross-Pitaevskii solver (Gross-Pitaevskii section,
Eqs. g5, ee, s1, wth) against the bifurcation from the linear ground state,
the paper's near-threshold closed form, the virial identity, the
Thomas-Fermi limit and the threshold root."""
import math

import numpy as np
import pytest

from oracle import gp as G

M, L = 1023, 10.0


@pytest.mark.parametrize("eps", [1e-4, 1e-3])
def test_bifurcation_from_the_linear_ground_state(eps):
    # just above the discrete linear eigenvalue lambda0 the bound state is
    # a psi0 with a^2 = (E - lambda0) / (h sum psi0^4), to first order
    lam0, psi0 = G.linear_ground_state(M, L)
    tau, h = G.grid(M, L)
    r = G.gp_solve(lam0 + eps, M, L, 8, 0.1)
    a = math.sqrt(eps / (h * float(np.sum(psi0 ** 4))))
    assert r["converged"] and r["residual"] < 1e-9
    assert np.max(np.abs(r["phi"] - a * psi0)) <= 3.0 * eps * a


def test_paper_near_threshold_closed_form():
    # phi ~ 2^{1/4} sqrt(E - 1) exp(-tau^2/2): phi(0)^2 = sqrt(2) (E - 1); the
    # discrete linear threshold is 1 up to the discretisation
    lam0, _ = G.linear_ground_state(M, L)
    assert abs(lam0 - 1.0) < 1e-4
    E = 1.01
    r = G.gp_solve(E, M, L, 8, 0.1)
    assert r["phi_max"] ** 2 / (math.sqrt(2.0) * (E - 1.0)) == pytest.approx(1.0, rel=0.03)
    # and the spectral waist of a Gaussian phi: w = 1/(2 sqrt(2) pi)
    r = G.gp_solve(lam0 + 1e-5, M, L, 400, 0.02)
    assert r["w"] == pytest.approx(1.0 / (2.0 * math.sqrt(2.0) * math.pi), rel=1e-3)


@pytest.mark.parametrize("E", [1.5, 3.0, 10.0])
def test_virial_identity(E):
    # scaling phi -> sqrt(l) phi(l tau) keeps the norm; stationarity of the
    # energy int(phi'^2 + tau^2 phi^2 + phi^4/2) gives 2K - 2V + I/2 = 0
    r = G.gp_solve(E, M, 12.0, 8, 0.1)
    phi, tau, h = r["phi"], r["tau"], r["h"]
    ext = np.concatenate(([0.0], phi, [0.0]))
    K = float(np.sum(np.diff(ext) ** 2)) / h
    V = h * float(np.sum(tau * tau * phi * phi))
    I = h * float(np.sum(phi ** 4))
    assert abs(2 * K - 2 * V + 0.5 * I) <= 1e-3 * (K + V)


def test_thomas_fermi_limit():
    # far above threshold phi^2 ~ E - tau^2; at the centre E - 1/E
    E = 200.0
    r = G.gp_solve(E, M, 20.0, 8, 0.1)
    assert abs(r["phi_max"] ** 2 - (E - 1.0 / E)) <= 0.5 / E


@pytest.mark.parametrize("kappa", [1e-3, 0.1, 0.14, 1.0, 5.0])
def test_threshold_is_the_root_of_E_equals_one(kappa):
    p = G.threshold(kappa)
    assert G.eigenvalue(p, kappa) == pytest.approx(1.0, rel=1e-13)
    assert G.eigenvalue(1.0, kappa) == 0.0
    assert p > 1.0 and G.eigenvalue(p * 1.01, kappa) > 1.0


def test_line_narrows_above_threshold():
    # N grows with E while the spectral waist shrinks (the line narrows)
    rs = [G.gp_solve(E, M, 12.0, 600, 0.02) for E in (1.01, 1.1, 1.5, 3.0, 10.0)]
    N = [r["N"] for r in rs]
    w = [r["w"] for r in rs]
    assert all(a < b for a, b in zip(N, N[1:]))
    assert all(a > b for a, b in zip(w, w[1:]))
