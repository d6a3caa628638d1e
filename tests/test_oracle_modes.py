"""Pins of the oracle's passive mode-analysis pieces (Simulations section:
field distribution by continuous-wave excitation, energy density in the
middle section): the plane energy-density monitor against the exact
standing-wave solution of a cavity eigenmode, and the continuous-wave source
against the frequency it drives."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import spectra as OS
from paper_0809_1547_amd import inputs as I


def cavity_mode(n, m, pol=(1.0, 0.3, -0.7)):
    """E of a PEC-box eigenmode sampled on the extended Yee range (three
    (nz+1, ny+1, nx+1) arrays, zero off the interior E-sites) and the mode's
    wave numbers."""
    nx, ny, nz = n
    k = [m[a] * math.pi / n[a] for a in range(3)]
    K = np.array([2 * math.sin(k[a] / 2) for a in range(3)])
    A = np.cross(K, np.array(pol))
    A /= np.linalg.norm(A)
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    e = [A[0] * np.cos(k[0] * (ii + 0.5)) * np.sin(k[1] * jj) * np.sin(k[2] * kk),
         A[1] * np.sin(k[0] * ii) * np.cos(k[1] * (jj + 0.5)) * np.sin(k[2] * kk),
         A[2] * np.sin(k[0] * ii) * np.sin(k[1] * jj) * np.cos(k[2] * (kk + 0.5))]
    for c in range(3):
        e[c][~I.interior_e_mask(n, c)] = 0.0
    return e, k


def curl_plus(e, n):
    """Forward-difference curl of E on the H-sites of [0, n)^3."""
    nx, ny, nz = n
    ex, ey, ez = e
    g = [np.zeros_like(ex) for _ in range(3)]
    s = (slice(0, nz), slice(0, ny), slice(0, nx))
    dy = lambda a: a[0:nz, 1:ny + 1, 0:nx] - a[s]
    dz = lambda a: a[1:nz + 1, 0:ny, 0:nx] - a[s]
    dx = lambda a: a[0:nz, 0:ny, 1:nx + 1] - a[s]
    g[0][s] = dy(ez) - dz(ey)
    g[1][s] = dz(ex) - dx(ez)
    g[2][s] = dx(ey) - dy(ex)
    return g


@pytest.mark.parametrize("n,m,eps,plane", [((9, 8, 7), (1, 1, 1), 1.0, 3), ((10, 7, 9), (2, 1, 3), 2.25, 5),
                                           ((6, 6, 6), (1, 2, 0), 4.0, 0)])
def test_plane_monitor_on_a_standing_wave(n, m, eps, plane):
    # E^n = cos(n theta) e and H^{n+1/2} = beta sin((n+1/2) theta) curl+ e with
    # sin(theta/2) = (S/sqrt(eps)) sqrt(sum sin^2(k_a/2)), beta = -S/(2 sin(theta/2)),
    # solve the lossless step exactly when started from E^0 = e and
    # H^{-1/2} = (S/2) curl+ e; the monitor then sums, over steps 0..N-1,
    # 1/2 [eps cos^2(n theta) |e|^2 + beta^2 sin^2((n+1/2) theta) |curl+ e|^2]
    # at the cells (i, j, plane)
    p = O.default_params(n, noise=False)
    o = O.Oracle(p)
    epsm, gain = I.homogeneous(n, eps, 0)
    o.set_material(epsm, gain)
    o.set_pump(0.0, O.GROUND)
    S = o.coefficients()[O.C_S]
    e, k = cavity_mode(n, m)
    g = curl_plus(e, n)
    for c in range(3):
        o.set_field(c, e[c])
        o.set_field(3 + c, 0.5 * S * g[c])
    theta = 2.0 * math.asin(S / math.sqrt(eps) * math.sqrt(sum(math.sin(q / 2) ** 2 for q in k)))
    beta = -S / (2.0 * math.sin(theta / 2))
    o.set_plane_monitor(plane)
    N = 37
    o.step(N)
    got, cnt = o.plane_monitor()
    steps = np.arange(N)
    ce = float(np.sum(np.cos(steps * theta) ** 2))
    sh = float(np.sum(np.sin((steps + 0.5) * theta) ** 2))
    nx, ny, _ = n
    e2 = sum(e[c][plane, :ny, :nx] ** 2 for c in range(3))
    g2 = sum(g[c][plane, :ny, :nx] ** 2 for c in range(3))
    want = 0.5 * (eps * ce * e2 + beta * beta * sh * g2)
    assert cnt == N
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    # zeroed by a new pump, and off after k = -1
    o.set_pump(0.0, O.GROUND)
    got, cnt = o.plane_monitor()
    assert cnt == 0 and not np.any(got)
    o.set_plane_monitor(-1)
    with pytest.raises(ValueError):
        o.plane_monitor()


@pytest.mark.parametrize("lam", [560e-9, 610e-9])
def test_cw_source_drives_its_own_frequency(lam):
    # a continuous wave in an absorbing box: after the switch-on the field at
    # the source site oscillates at the drive frequency, so its spectrum over
    # a band around it peaks at the bin nearest w_s = 2 pi c / lambda
    n = (24, 24, 24)
    p = O.default_params(n, noise=False, bc=(O.ABSORB,) * 3)
    o = O.Oracle(p)
    epsm, gain = I.homogeneous(n, 1.0, 0)
    o.set_material(epsm, gain)
    o.set_pump(0.0, O.GROUND)
    o.set_cw_source(2, 12, 12, 12, amp=1.0, lambda_s=lam, t_ramp=10e-15)
    steps = 6000
    dt = o.coefficients()[O.C_DT]
    om = I.dft_omegas(500e-9, 700e-9, steps, dt)
    o.set_probes(np.array([[2, 12, 12, 12]]), om)
    o.step(steps)
    ws = 2.0 * math.pi * 299792458.0 / lam
    peaks = OS.spectral_peaks(o.spectrum(), 0.1, 1)
    assert peaks == [int(np.argmin(np.abs(om - ws)))]
    # the switch-on: the source value grows from zero like (t/t_ramp)^2
    v0 = o.source_value(0)
    assert abs(v0) < 1e-3 and o.source_value(100000) != 0.0
