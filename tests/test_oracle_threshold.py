"""Pins of the oracle's threshold and linewidth fits (Results section, Fig. 5b;
Gross-Pitaevskii section, Eqs. ee, s1, wth): exact recovery of exponential
growth and of a linear rate law, the growth rate and threshold of a single
cavity mode against the discrete dispersion relation, and the kappa fit
against data generated with a known kappa and against the paper's
threshold waist."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import gp as G
from oracle import threshold as T
from paper_0809_1547_amd import inputs as I

from test_oracle_bloch import _newton_root, physics  # the P5 dispersion root


def test_growth_rate_is_exact_for_exponentials():
    n = np.arange(4000)
    for g in (-3e-4, 1e-5, 2.5e-3):
        W = 7.5e-9 * np.exp(g * n)
        assert T.growth_rate(W, 1000, 4000) == pytest.approx(g, rel=1e-10, abs=1e-15)
    # the window matters: a history that bends at step 2000
    W = np.exp(np.where(n < 2000, 1e-3 * n, 2.0 + 3e-3 * (n - 2000)))
    assert T.growth_rate(W, 2000, 4000) == pytest.approx(3e-3, rel=1e-10)
    assert T.growth_rate(W, 0, 2000) == pytest.approx(1e-3, rel=1e-10)


def test_threshold_is_the_root_of_a_linear_rate_law():
    Na = np.array([0.5, 1.0, 2.0, 3.5, 6.0]) * 1e24
    b, Nth = 3.2e-28, 1.7e24
    a_, b_, r = T.threshold(Na, b * (Na - Nth))
    assert r == pytest.approx(Nth, rel=1e-12)
    assert b_ == pytest.approx(b, rel=1e-12) and a_ == pytest.approx(-b * Nth, rel=1e-12)
    # order of the runs does not matter; two runs suffice
    assert T.threshold(Na[::-1], b * (Na[::-1] - Nth))[2] == pytest.approx(Nth, rel=1e-12)
    assert T.threshold(Na[:2], b * (Na[:2] - Nth))[2] == pytest.approx(Nth, rel=1e-12)


def test_threshold_of_a_cavity_mode_follows_the_dispersion_relation():
    # one TM(1,1,0) mode of a closed cavity filled with a gain medium whose
    # inversion is frozen at N1 - N2 = dN: the energy grows at 2 Im theta(dN)
    # per step (theta the root of the coupled discrete dispersion relation);
    # rates measured on the oracle's energy history give the same line, and
    # its root lies at the loss-free threshold dN = 0 to the curvature of
    # Im theta(dN)
    n = (20, 20, 2)
    ph = physics()
    kx, ky = math.pi / n[0], math.pi / n[1]
    dns = np.array([-0.6, -0.2, 0.25, 0.7])
    meas, exact = [], []
    for dn in dns:
        o = O.Oracle(O.default_params(n, noise=False, frozen_pop=True))
        o.set_material(*I.homogeneous(n, 1.0, 1))
        o.set_pump(2e24, O.PREPUMPED)
        for c in range(3):
            m = I.interior_e_mask(n, c)
            a1 = np.zeros(o.shape); a1[m] = 1.0 + dn
            a2 = np.zeros(o.shape); a2[m] = 1.0
            o.set_field(12 + c, a1)
            o.set_field(15 + c, a2)
        kk, jj, ii = np.meshgrid(np.arange(n[2] + 1), np.arange(n[1] + 1), np.arange(n[0] + 1), indexing="ij")
        ez = np.sin(kx * ii) * np.sin(ky * jj)
        ez[~I.interior_e_mask(n, 2)] = 0.0
        o.set_field(2, 1e-6 * ez)
        o.step(3000)
        meas.append(T.growth_rate(o.energy_history(), 1000, 3000))
        exact.append(2.0 * _newton_root(kx, ky, dn, ph).imag)
        o.close()
    meas, exact = np.array(meas), np.array(exact)
    # gain where N2 > N1 (dN < 0), loss where N1 > N2
    assert np.all(np.sign(exact) == -np.sign(dns))
    assert np.max(np.abs(meas - exact)) < 2e-3 * np.max(np.abs(exact))
    r_meas = T.threshold(dns, meas)[2]
    r_exact = T.threshold(dns, exact)[2]
    assert abs(r_meas - r_exact) < 2e-3 * np.ptp(dns)
    assert abs(r_exact) < 0.05 * np.ptp(dns)


M, L, NNU, DNU = 255, 14.0, 512, 0.02
T_G = 1.0 / 1.24458e15


def test_model_waist_at_threshold_is_the_papers_closed_form():
    # just above threshold the waist is W_th = sqrt(kappa/2) / (2 pi t_g)
    # (Eq. wth): E -> 1, w -> 1/(2 sqrt(2) pi), p -> p_th
    for kappa in (0.05, 0.14, 0.5):
        W = T.model_waist([1.0 + 1e-6], kappa, 1.0, T_G, 1023, 12.0, 400, 0.02)[0]
        Wth = math.sqrt(kappa / 2.0) / (2.0 * math.pi * T_G) / G.threshold(kappa) ** 0.25
        assert W == pytest.approx(Wth, rel=2e-3)


@pytest.mark.parametrize("kappa", [0.02, 0.14, 1.1])
def test_kappa_fit_recovers_the_kappa_of_its_data(kappa):
    Nth = 2.0e24
    Na = Nth * np.array([1.15, 1.4, 1.9, 2.6])
    W = T.model_waist(Na, kappa, Nth, T_G, M, L, NNU, DNU)
    k, Wf = T.kappa_fit(Na, W, Nth, T_G, M, L, NNU, DNU)
    assert k == pytest.approx(kappa, rel=1e-7)
    assert np.max(np.abs(Wf / W - 1)) < 1e-7
    # widths that do not depend on kappa's sign of error: a 2% wider line
    # asks for a larger kappa
    k2, _ = T.kappa_fit(Na, 1.02 * W, Nth, T_G, M, L, NNU, DNU)
    assert k2 > k


def test_kappa_fit_of_near_threshold_widths_follows_eq_wth():
    # pumps barely above threshold: the widths are the closed form W_th
    # divided by p^{1/4}; the fit returns the kappa they were made with
    kappa, Nth = 0.3, 1.0e24
    Na = Nth * (1.0 + np.array([2e-4, 5e-4, 1e-3]))
    pth = G.threshold(kappa)
    W = np.array([math.sqrt(kappa) / (2.0 * math.sqrt(2.0) * math.pi * T_G) / (pth * x / Nth) ** 0.25 for x in Na])
    k, _ = T.kappa_fit(Na, W, Nth, T_G, 1023, 12.0, 400, 0.02)
    assert k == pytest.approx(kappa, rel=5e-3)


# ------------------------------------------------------------------ knee

def test_knee_of_two_exact_lines_is_their_crossing():
    # a broad width below threshold falling linearly, a narrow one above: the
    # split between the last point of the first line and the first of the
    # second leaves no residual, and the knee is the lines' crossing
    x = np.array([1.0, 1.5, 2.0, 2.5, 3.1, 3.6, 4.2, 5.0])
    xk = 2.8
    y = np.where(x < xk, 10.0 - 0.5 * (x - xk), 10.0 - 6.0 * (x - xk))
    k, s, (aL, bL), (aR, bR), sse = T.knee(x, y)
    assert s == 4 and sse < 1e-24
    assert k == pytest.approx(xk, abs=1e-12)
    assert bL == pytest.approx(-0.5) and bR == pytest.approx(-6.0)
    # shifting y or scaling x moves nothing but the knee's scale
    assert T.knee(x, y + 3.0)[0] == pytest.approx(xk, abs=1e-12)
    assert T.knee(2.0 * x, y)[0] == pytest.approx(2.0 * xk, abs=1e-12)


def test_knee_is_kept_between_the_split_points():
    # noisy points: whatever the crossing of the two fitted lines, the knee
    # lies between the two points either side of the chosen split
    g = np.random.default_rng(3)
    for trial in range(20):
        x = np.sort(g.uniform(0, 10, 12))
        y = np.where(x < 5, 1.0, 1.0 - (x - 5)) + 0.3 * g.standard_normal(12)
        k, s, *_ = T.knee(x, y)
        assert 2 <= s <= len(x) - 2
        assert x[s - 1] <= k <= x[s]


def test_knee_of_a_straight_line_takes_the_first_split():
    x = np.arange(6.0)
    k, s, _, _, sse = T.knee(x, 2.0 * x + 1.0)
    assert s == 2 and sse < 1e-24 and x[1] <= k <= x[2]
