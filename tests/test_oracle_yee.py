"""Pins of the oracle's Maxwell part (rows a1 and a3 with PEC walls).

* P1: a cavity eigenmode of a vacuum PEC box keeps its shape, and its
  amplitude obeys the closed-form Yee dispersion relation
  sin^2(w dt/2)/(c dt)^2 = sum_a sin^2(m_a pi/(2 n_a))/dx^2.
* P2: with an arbitrary permittivity map and no gain, the discrete energy
  1/2 sum[eps |E^n|^2 + H^{n-1/2}.H^{n+1/2}] is invariant to rounding.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_0809_1547_amd import inputs as I


def cavity_mode(n, m, pol=(1.0, 0.3, -0.7)):
    """Sampled TE/TM cavity mode (E only) of a PEC box on the extended Yee
    index range; returns three (nz+1, ny+1, nx+1) arrays."""
    nx, ny, nz = n
    k = [m[a] * math.pi / n[a] for a in range(3)]
    K = np.array([2 * math.sin(k[a] / 2) for a in range(3)])
    A = np.cross(K, np.array(pol))            # A . K = 0: discretely divergence-free
    A /= np.linalg.norm(A)
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                             indexing="ij")
    ex = A[0] * np.cos(k[0] * (ii + 0.5)) * np.sin(k[1] * jj) * np.sin(k[2] * kk)
    ey = A[1] * np.sin(k[0] * ii) * np.cos(k[1] * (jj + 0.5)) * np.sin(k[2] * kk)
    ez = A[2] * np.sin(k[0] * ii) * np.sin(k[1] * jj) * np.cos(k[2] * (kk + 0.5))
    out = []
    for c, e in enumerate((ex, ey, ez)):
        e = e.copy()
        e[~I.interior_e_mask(n, c)] = 0.0
        out.append(e)
    return out


def vacuum_oracle(n, **kw):
    p = O.default_params(n, noise=False, **kw)
    o = O.Oracle(p)
    eps, gain = I.homogeneous(n, 1.0, 0)
    o.set_material(eps, gain)
    o.set_pump(2e24, O.GROUND)
    return o


@pytest.mark.parametrize("n,m", [((12, 10, 8), (1, 2, 1)), ((9, 9, 9), (2, 1, 3)),
                                 ((16, 6, 5), (3, 0, 1))])
def test_p1_yee_dispersion_and_mode_shape(n, m):
    o = vacuum_oracle(n)
    mode = cavity_mode(n, m)
    for c in range(3):
        o.set_field(c, mode[c])
    norm2 = sum(float(np.sum(e * e)) for e in mode)
    amps, resid = [], 0.0
    for _ in range(2000):
        o.step(1)
        E = [o.field(c) for c in range(3)]
        a = sum(float(np.sum(E[c] * mode[c])) for c in range(3)) / norm2
        amps.append(a)
        r = math.sqrt(sum(float(np.sum((E[c] - a * mode[c]) ** 2)) for c in range(3)))
        resid = max(resid, r / math.sqrt(norm2))
    amps = np.array([1.0] + amps)
    # e_{n+1} + e_{n-1} = 2 cos(theta) e_n for a single discrete mode
    lhs = amps[2:] + amps[:-2]
    cos_t = float(np.dot(lhs, amps[1:-1]) / (2 * np.dot(amps[1:-1], amps[1:-1])))
    theta = math.acos(cos_t)
    S = o.coefficients()[O.C_S]
    expect = 2 * math.asin(S * math.sqrt(sum(math.sin(m[a] * math.pi / (2 * n[a])) ** 2
                                              for a in range(3))))
    assert abs(theta - expect) < 1e-12 * expect
    assert resid < 1e-12
    # the physical frequency: sin^2(w dt/2)/(c dt)^2 = sum sin^2(.)/dx^2
    dt = o.coefficients()[O.C_DT]
    w = theta / dt
    c0, dx = 299792458.0, 20e-9
    lhs_phys = math.sin(w * dt / 2) ** 2 / (c0 * dt) ** 2
    rhs_phys = sum(math.sin(m[a] * math.pi / (2 * n[a])) ** 2 for a in range(3)) / dx ** 2
    assert abs(lhs_phys / rhs_phys - 1) < 1e-11


def test_p2_energy_invariant_with_dielectric_map():
    n = (10, 9, 8)
    o = O.Oracle(O.default_params(n, noise=False))
    pk = I.rsa_pack(n, seed=3, count=4, radius=2.5)
    eps, _ = I.voxelize(pk)
    assert 0 < (eps > 1).sum() < eps.size
    o.set_material(eps, np.zeros_like(eps, dtype=np.uint8))
    o.set_pump(2e24, O.GROUND)
    f = I.random_fields(n, seed=9)
    for c in range(3):
        o.set_field(c, f[c])
    naive = []
    for _ in range(20):
        o.step(500)
        eps_site = np.zeros(o.shape)
        eps_site[:n[2], :n[1], :n[0]] = eps
        W = 0.5 * sum(float(np.sum(eps_site * o.field(c) ** 2 + o.field(3 + c) ** 2))
                      for c in range(3))
        naive.append(W)
    hist = o.energy_history()
    assert hist.shape == (10000,)
    drift = np.max(np.abs(hist - hist[0])) / hist[0]
    assert drift < 1e-12
    # the naive energy is not invariant: the discrete invariant is non-trivial
    naive = np.array(naive)
    assert (naive.max() - naive.min()) / naive.mean() > 1e-6


def test_p2_energy_rises_with_a_source_in_a_closed_box():
    # sanity of the sign convention: injecting field raises the invariant
    n = (8, 8, 8)
    o = vacuum_oracle(n)
    o.set_source(2, 4, 4, 3, amp=1.0)
    o.step(400)
    h = o.energy_history()
    assert h[0] == 0.0 and h[-1] > 0.0
