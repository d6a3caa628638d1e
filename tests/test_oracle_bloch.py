"""Pins of the oracle's Bloch part (rows a2 and a4) and of the coupled step.

* P3: the polarisation recurrence driven by a harmonic field settles on the
  closed-form discrete Lorentz susceptibility
  Omega_p^2 dN / (w_a^2 - (4/dt^2) sin^2(w dt/2) - i dw_a sin(w dt)/dt),
  which approaches the continuous Lorentzian to O((w dt)^2).
* P4: the four-level rates conserve N0+N1+N2+N3 = N_a at every site; with
  E = 0 the recurrence is the matrix power of (I + dt A); its fixed point is
  the null space of the continuous rate matrix A.
* P5: a cavity mode of a homogeneous pre-pumped gain medium grows at twice
  the imaginary part of the complex root of the coupled discrete dispersion
  relation (2/(c dt))^2 sin^2(w dt/2) (1 + chi_d(w)) = K^2; with absorbing
  populations (N1 > N2) the same mode decays.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as O
from paper_0809_1547_amd import inputs as I

C0 = 299792458.0
EPS0 = 8.8541878128e-12
HBAR = 1.054571817e-34


def physics():
    """Independent evaluation of the model constants from their definitions:
    gain centre lambda0 = 590 nm, bandwidth 230 nm, coupling from the
    radiative lifetime tau21 (classical oscillator), N_ref = 1e24 m^-3."""
    dx, S3 = 20e-9, 0.99
    dt = S3 * dx / (C0 * math.sqrt(3))
    wa = 2 * math.pi * C0 / 590e-9
    dwa = 2 * math.pi * C0 * 230e-9 / 590e-9 ** 2
    tau21 = 1e-9
    kappa = 6 * math.pi * EPS0 * C0 ** 3 / (wa ** 2 * tau21)
    omp2 = kappa * 1e24 / EPS0
    return dict(dt=dt, wa=wa, dwa=dwa, omp2=omp2, S=C0 * dt / dx)


def chi_discrete(theta, dN, ph):
    """Discrete susceptibility at complex or real w dt = theta (e^{-i w t})."""
    dt = ph["dt"]
    return ph["omp2"] * dt ** 2 * dN / (
        (ph["wa"] * dt) ** 2 - 4 * np.sin(theta / 2) ** 2 - 1j * ph["dwa"] * dt * np.sin(theta))


def test_coefficients_match_stated_constants():
    o = O.Oracle(O.default_params(4))
    c = o.coefficients()
    ph = physics()
    assert c[O.C_DT] == pytest.approx(3.81315e-17, rel=1e-5)
    assert c[O.C_S] == pytest.approx(0.99 / math.sqrt(3), rel=1e-15)
    assert c[O.C_WA] == pytest.approx(3.19263e15, rel=1e-5)
    assert c[O.C_DWA] == pytest.approx(1.24458e15, rel=1e-5)
    assert c[O.C_OMP2] == pytest.approx(ph["omp2"], rel=1e-14)
    # beta = eps0 E_ref^2 / (hbar w_a N_ref)
    assert c[O.C_BETA] == pytest.approx(0.26298, rel=1e-4)


@pytest.mark.parametrize("lam_nm", [400, 520, 590, 650, 800])
@pytest.mark.parametrize("dN", [-2.0, 0.7])
def test_p3_lorentz_susceptibility(lam_nm, dN):
    o = O.Oracle(O.default_params(4))
    coef = o.coefficients()
    ph = physics()
    theta = 2 * math.pi * C0 / (lam_nm * 1e-9) * ph["dt"]
    n = 6000
    t = np.arange(n)
    P = O.p_series(coef, np.cos(theta * t), np.full(n, dN))
    # P^n (stored at index n-1) against A cos(theta n) + B sin(theta n) late in the run
    w = slice(3000, n)
    tt = t[w] + 1
    M = np.stack([np.cos(theta * tt), np.sin(theta * tt)], axis=1)
    (A, B), *_ = np.linalg.lstsq(M, P[w], rcond=None)
    got = A + 1j * B
    expect = chi_discrete(theta, dN, ph)
    assert abs(got - expect) < 1e-10 * abs(expect)
    # the continuous Lorentzian, to O((w dt)^2)
    wv = theta / ph["dt"]
    cont = ph["omp2"] * dN / (ph["wa"] ** 2 - wv ** 2 - 1j * wv * ph["dwa"])
    assert abs(got - cont) < 0.03 * abs(cont)


def test_p3_gain_sign():
    # an inverted medium (N2 > N1, dN < 0) has Im chi < 0: amplification for e^{-i w t}
    ph = physics()
    th = ph["wa"] * ph["dt"]
    assert chi_discrete(th, -1.0, ph).imag < 0 < chi_discrete(th, 1.0, ph).imag


def _rate_matrix(c):
    """Continuous-time rate matrix A (per step) on (N0, N1, N2, N3)."""
    d32, d21, d10, dwp = c[O.C_DT32], c[O.C_DT21], c[O.C_DT10], c[O.C_DTWP]
    return np.array([[-dwp, d10, 0.0, 0.0],
                     [0.0, -d10, d21, 0.0],
                     [0.0, 0.0, -d21, d32],
                     [dwp, 0.0, 0.0, -d32]])


def test_p4_conservation_under_random_fields():
    o = O.Oracle(O.default_params(4))
    coef = o.coefficients()
    rng = np.random.default_rng(1)
    n = 10000
    N0 = np.array([2.0, 0.0, 0.0, 0.0])
    out = O.pop_series(coef, N0, rng.standard_normal(n), 1e-2 * rng.standard_normal(n))
    tot = out.sum(axis=1)
    assert np.max(np.abs(tot - 2.0)) / 2.0 < 1e-13
    assert np.ptp(out[:, 2]) > 1e-3          # the field work really moved N2


def test_p4_matrix_power_steady_state_and_expm():
    o = O.Oracle(O.default_params(4, Wp=3e13))
    coef = o.coefficients()
    A = _rate_matrix(coef)
    n = 20000
    N_init = np.array([2.0, 0.0, 0.0, 0.0])
    out = O.pop_series(coef, N_init, np.zeros(n), np.zeros(n))
    for k in (1, 7, 1000, n):
        expect = np.linalg.matrix_power(np.eye(4) + A, k) @ N_init
        assert np.allclose(out[k - 1], expect, rtol=1e-12, atol=1e-15)
    # continuous solution exp(A t): agreement to first order in dt/tau
    cont = scipy.linalg.expm(A * 500) @ N_init
    assert np.allclose(out[499], cont, rtol=0, atol=2.0 * 5 * coef[O.C_DT32])
    # fixed point: null space of A, normalised to N_a
    _, _, vh = np.linalg.svd(A)
    ns = vh[-1] / vh[-1].sum() * 2.0
    o.set_material(*I.homogeneous(4, 1.0, 1))
    o.set_pump(2e24, O.PREPUMPED)
    site = (slice(None), 1, 1, 1)
    got = np.array([o.field(21)[1, 1, 1], o.field(12)[1, 1, 1], o.field(15)[1, 1, 1],
                    o.field(18)[1, 1, 1]])
    assert np.allclose(got, ns, rtol=1e-12)
    # stationary under the recurrence
    res = O.pop_series(coef, got, np.zeros(50), np.zeros(50))
    assert np.allclose(res[-1], got, rtol=1e-13)


def test_p4_conservation_on_the_grid():
    n = (8, 7, 6)
    o = O.Oracle(O.default_params(n, E_sp=1e-2))
    pk = I.rsa_pack(n, seed=1, count=2, radius=2.0)
    o.set_material(*I.voxelize(pk))
    o.set_pump(3e24, O.GROUND)
    f = I.random_fields(n, seed=2, amplitude=3.0)
    for c in range(3):
        o.set_field(c, f[c])
    o.step(300)
    for c in range(3):
        tot = o.field(12 + c) + o.field(15 + c) + o.field(18 + c) + o.field(21 + c)
        m = I.interior_e_mask(n, c)
        m[:n[2], :n[1], :n[0]] &= I.voxelize(pk)[1].astype(bool)
        m[n[2]:, :, :] = False
        m[:, n[1]:, :] = False
        m[:, :, n[0]:] = False
        assert np.max(np.abs(tot[m] - 3.0)) < 1e-13 * 3.0
        assert np.ptp(o.field(15 + c)[m]) > 0     # populations did move


def _growth_setup(n, m_idx, *, frozen, dN_override=None):
    p = O.default_params(n, noise=False, frozen_pop=frozen)
    o = O.Oracle(p)
    o.set_material(*I.homogeneous(n, 1.0, 1))
    o.set_pump(2e24, O.PREPUMPED)
    if dN_override is not None:
        n1, n2 = dN_override
        for c in range(3):
            m = I.interior_e_mask(n, c)
            a1 = np.zeros(o.shape); a1[m] = n1
            a2 = np.zeros(o.shape); a2[m] = n2
            o.set_field(12 + c, a1)
            o.set_field(15 + c, a2)
    # TM mode (m, m', 0): E_z only, uniform along z
    nx, ny, nz = n
    kx, ky = m_idx[0] * math.pi / nx, m_idx[1] * math.pi / ny
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                             indexing="ij")
    ez = np.sin(kx * ii) * np.sin(ky * jj)
    ez[~I.interior_e_mask(n, 2)] = 0.0
    o.set_field(2, 1e-6 * ez)
    return o, ez, (kx, ky)


def _measured_growth(o, ez, steps=3000, start=1500):
    amps = []
    for _ in range(steps):
        o.step(1)
        amps.append(float(np.sum(o.field(2) * ez)))
    a = np.array(amps)
    # two-root linear prediction e_{n+1} = p e_n + q e_{n-1} on the late window
    y = a[start + 1:]
    X = np.stack([a[start:-1], a[start - 1:-2]], axis=1)
    (p, q), *_ = np.linalg.lstsq(X, y, rcond=None)
    z = np.roots([1.0, -p, -q])
    return math.log(abs(z[0])), abs(abs(z[0]) - abs(z[1]))


def _newton_root(kx, ky, dN, ph):
    K2 = 4 * math.sin(kx / 2) ** 2 + 4 * math.sin(ky / 2) ** 2
    S = ph["S"]

    def f(th):
        return 4 * np.sin(th / 2) ** 2 * (1 + chi_discrete(th, dN, ph)) - S ** 2 * K2

    th = complex(2 * math.asin(S * math.sqrt(K2) / 2))
    for _ in range(60):
        h = 1e-7
        d = (f(th + h) - f(th - h)) / (2 * h)
        th = th - f(th) / d
    return th


def test_p5_small_signal_growth_rate():
    n = (20, 20, 2)
    o, ez, (kx, ky) = _growth_setup(n, (1, 1), frozen=False)
    coef = o.coefficients()
    dN = o.field(12)[1, 1, 1] - o.field(15)[1, 1, 1]
    ph = physics()
    th = _newton_root(kx, ky, dN, ph)
    assert th.imag > 0                          # the pre-pumped medium amplifies
    rate, split = _measured_growth(o, ez)
    assert split < 1e-9                         # a complex pair: one oscillating mode
    assert abs(rate - th.imag) < 1e-6 * th.imag
    assert coef[O.C_DT21] > 0                   # populations were live (not frozen)


def test_p5_absorbing_populations_decay():
    n = (20, 20, 2)
    o, ez, (kx, ky) = _growth_setup(n, (1, 1), frozen=True, dN_override=(1.5, 0.2))
    th = _newton_root(kx, ky, 1.3, physics())
    assert th.imag < 0
    rate, _ = _measured_growth(o, ez)
    assert abs(rate - th.imag) < 1e-6 * abs(th.imag)


def test_p4_field_work_balances_field_energy():
    """Discrete Poynting theorem: with the Yee update the field invariant drops
    by sum Ebar.(P^{n+1}-P^n) per step, and the rate equations move exactly
    beta times that into N2 (out of N1).  With pump and the 3->2, 1->0 decays
    off, W_field + (1/beta)(sum N2 + accumulated 2->1 decay) is constant,
    whatever drives P.  (tau21 stays finite: it also fixes the coupling.)"""
    n = (8, 7, 6)
    o = O.Oracle(O.default_params(n, tau32=math.inf, tau10=math.inf, Wp=0.0, E_sp=0.3))
    coef = o.coefficients()
    beta, d21 = coef[O.C_BETA], coef[O.C_DT21]
    assert beta > 0 and coef[O.C_DT32] == 0.0 and coef[O.C_CK] > 0
    pk = I.rsa_pack(n, seed=2, count=2, radius=2.0)
    eps, gain = I.voxelize(pk)
    o.set_material(eps, gain)
    o.set_pump(2e24, O.GROUND)
    for c in range(3):
        m = np.zeros(o.shape, dtype=bool)
        m[:n[2], :n[1], :n[0]] = gain.astype(bool)
        m &= I.interior_e_mask(n, c)
        o.set_field(12 + c, np.where(m, 0.4, 0.0))
        o.set_field(15 + c, np.where(m, 1.6, 0.0))
        o.set_field(21 + c, np.zeros(o.shape))
    f = I.random_fields(n, seed=4)
    for c in range(3):
        o.set_field(c, f[c])
    vals, n2s = [], []
    decayed = 0.0
    for k in range(400):
        n2 = sum(float(np.sum(o.field(15 + c))) for c in range(3))
        n2s.append(n2)
        o.step(1)
        W = o.energy_history()[k]
        vals.append(W + (n2 + decayed) / beta)
        decayed += d21 * n2
    vals = np.array(vals)
    assert np.max(np.abs(vals - vals[0])) < 1e-12 * abs(vals[0])
    # the populations really exchanged energy with the field
    work = np.diff(n2s) + d21 * np.array(n2s[:-1])
    assert np.max(np.abs(work)) > 1e-9 * n2s[0]
