"""Pins of the oracle's boundary, source and monitors (rows a6, a7).

* P7: the running DFT (sign e^{+i w t}, the Fourier convention of the
  Gross-Pitaevskii section) of a single discrete cavity mode equals the
  closed-form geometric sum; on a random series it equals numpy's FFT at the
  FFT bins.
* P8: the soft source's sampled spectrum equals the analytic Fourier
  transform of a Gaussian-modulated sinusoid; the first-order Mur wall
  reflects a guided TE10 wave with the exact discrete reflection coefficient
  of the Mur recurrence on the Yee grid.
* the loss-box monitor is the time sum of |E|^2 over the box.
* the graded lossy layer: a uniform loss decays a cavity mode by the closed
  form; a guided pulse's response and the layer's reflection coefficient
  equal the exact solution of the discrete frequency-domain recurrence.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_0809_1547_amd import inputs as I
from test_oracle_yee import cavity_mode, vacuum_oracle


def test_p7_dft_of_a_cavity_mode_is_a_geometric_sum():
    n, m = (12, 10, 8), (1, 2, 1)
    o = vacuum_oracle(n)
    mode = cavity_mode(n, m)
    for c in range(3):
        o.set_field(c, mode[c])
    probe = (1, 5, 4, 3)
    v = mode[1][probe[3], probe[2], probe[1]]
    assert abs(v) > 0.05
    dt = o.coefficients()[O.C_DT]
    S = o.coefficients()[O.C_S]
    theta = 2 * math.asin(S * math.sqrt(sum(math.sin(m[a] * math.pi / (2 * n[a])) ** 2
                                             for a in range(3))))
    om = np.array([0.3, 0.9, 1.0, 1.1, 2.5]) * theta / dt
    o.set_probes(np.array([probe]), om)
    M = 1500
    o.step(M)
    got = o.spectrum()[0]
    # with H^{-1/2} = 0 the amplitude is e_m = cos(m theta + theta/2) / cos(theta/2)
    expect = []
    for w in om:
        tot = 0
        for sgn in (+1, -1):
            r = np.exp(1j * (sgn * theta + w * dt))
            geo = M if abs(1 - r) < 1e-13 else r * (1 - r ** M) / (1 - r)
            tot += np.exp(1j * sgn * theta / 2) * geo
        expect.append(v * tot / (2 * math.cos(theta / 2)))
    expect = np.array(expect)
    assert np.max(np.abs(got - expect)) < 1e-9 * np.max(np.abs(expect))


def test_p7_dft_matches_fft_bins():
    n = (8, 8, 8)
    o = O.Oracle(O.default_params(n, noise=False))
    pk = I.rsa_pack(n, seed=4, count=2, radius=2.0)
    eps, _ = I.voxelize(pk)
    o.set_material(eps, np.zeros_like(eps, dtype=np.uint8))
    o.set_pump(2e24, O.GROUND)
    f = I.random_fields(n, seed=5)
    for c in range(3):
        o.set_field(c, f[c])
    M = 256
    dt = o.coefficients()[O.C_DT]
    ks = np.array([0, 3, 17, 64, 101, 128])
    om = 2 * math.pi * ks / (M * dt)
    probe = (0, 3, 4, 5)
    o.set_probes(np.array([probe]), om)
    series = []
    for _ in range(M):
        o.step(1)
        series.append(o.field(0)[probe[3], probe[2], probe[1]])
    x = np.array(series)
    # sum_{m=1}^{M} x_m e^{2 pi i k m / M} = e^{2 pi i k/M} M ifft(x)[k]
    ref = np.exp(2j * math.pi * ks / M) * M * np.fft.ifft(x)[ks]
    assert np.max(np.abs(o.spectrum()[0] - ref)) < 1e-11 * np.max(np.abs(ref))


def test_p8_source_spectrum_is_the_analytic_transform():
    o = vacuum_oracle((8, 8, 8))
    lam, tau, t0, amp = 532e-9, 1e-15, 8e-15, 0.7
    o.set_source(2, 4, 4, 3, amp=amp, lambda_s=lam, tau_p=tau, t0=t0)
    dt = o.coefficients()[O.C_DT]
    N = int(2 * t0 / dt) + 200
    s = np.array([o.source_value(k) for k in range(N)])
    t = (np.arange(N) + 1) * dt
    ws = 2 * math.pi * 299792458.0 / lam
    for w in np.array([0.2, 0.7, 1.0, 1.3, 2.0]) * ws:
        got = np.sum(s * np.exp(1j * w * t)) * dt
        expect = amp * np.exp(1j * w * t0) * math.sqrt(math.pi) * tau / 2j * (
            math.exp(-tau ** 2 * (w + ws) ** 2 / 4) - math.exp(-tau ** 2 * (w - ws) ** 2 / 4))
        assert abs(got - expect) < 1e-9 * amp * tau


def _mur_reflection(theta, beta, m):
    q = np.exp(-1j * theta)
    p = np.exp(1j * beta)
    return (1 / p + m * q / p - m - q) / (q - p - m * q * p + m)


def test_p8_mur_reflection_of_a_guided_wave():
    nx, ny, nz = 8, 2, 1200
    n = (nx, ny, nz)
    o = O.Oracle(O.default_params(n, noise=False, bc=(O.PEC, O.PEC, O.MUR1)))
    o.set_material(*I.homogeneous(n, 1.0, 0))
    o.set_pump(2e24, O.GROUND)
    kc, sig, beta0, kp = 500, 40.0, 2 * math.pi / 12, 900
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                             indexing="ij")
    ey = np.sin(math.pi * ii / nx) * np.exp(-0.5 * ((kk - kc) / sig) ** 2) * np.cos(beta0 * kk)
    ey[~I.interior_e_mask(n, 1)] = 0.0
    o.set_field(1, ey)
    S = o.coefficients()[O.C_S]
    dt = o.coefficients()[O.C_DT]
    betas = beta0 + np.linspace(-0.04, 0.04, 9)
    thetas = 2 * np.arcsin(S * np.sqrt(np.sin(math.pi / (2 * nx)) ** 2 + np.sin(betas / 2) ** 2))
    o.set_probes(np.array([(1, nx // 2, 0, kp)]), thetas / dt)
    # incident packet passes the probe, then its reflection from the z = nz
    # wall returns before the reflection from the z = 0 wall can arrive
    o.step(1560)
    f_inc = o.spectrum()[0].copy()
    o.step(1106)
    f_ref = o.spectrum()[0] - f_inc
    R_meas = f_ref / f_inc * np.exp(2j * betas * (kp - nz))
    m = (S - 1) / (S + 1)
    R_th = _mur_reflection(thetas, betas, m)
    assert np.all(np.abs(R_th) > 1e-3) and np.all(np.abs(R_th) < 0.2)
    assert np.max(np.abs(R_meas - R_th) / np.abs(R_th)) < 1e-4


def test_loss_box_is_time_sum_of_e_squared():
    n = (8, 8, 8)
    o = O.Oracle(O.default_params(n, noise=False))
    o.set_material(*I.homogeneous(n, 2.0, 0))
    o.set_pump(2e24, O.GROUND)
    f = I.random_fields(n, seed=7)
    for c in range(3):
        o.set_field(c, f[c])
    lo, hi = (2, 3, 1), (6, 7, 5)
    o.set_loss_box(lo, hi)
    tot = 0.0
    for _ in range(30):
        o.step(1)
        for c in range(3):
            e = o.field(c)[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
            msk = I.interior_e_mask(n, c)[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
            tot += float(np.sum(e[msk] ** 2))
    assert o.loss() == pytest.approx(tot, rel=1e-13)


# ----------------------------------------------------- graded lossy layer

def test_lossy_cavity_mode_decays_by_closed_form_factor():
    """Uniform loss a on every E- and H-site (order 0, layer deeper than the
    box gives a = 2 a_max per axis): a cavity mode's amplitude obeys
    z^2 - (2g - d^2 S^2 K^2) z + g^2 = 0 with g = (1-a)/(1+a), d = 1/(1+a), so
    both roots have modulus exactly g and cos(arg z) = (2g - d^2 S^2 K^2)/(2g)."""
    n, m = (12, 10, 8), (1, 2, 1)
    amax = 0.01
    o = O.Oracle(O.default_params(n, noise=False, bc=(O.ABSORB,) * 3, absorb_cells=100,
                                  absorb_order=0, absorb_rate=amax))
    o.set_material(*I.homogeneous(n, 1.0, 0))
    o.set_pump(2e24, O.GROUND)
    mode = cavity_mode(n, m)
    for c in range(3):
        o.set_field(c, mode[c])
    norm2 = sum(float(np.sum(e * e)) for e in mode)
    amps = [1.0]
    for _ in range(400):
        o.step(1)
        amps.append(sum(float(np.sum(o.field(c) * mode[c])) for c in range(3)) / norm2)
    a = np.array(amps)
    y = a[2:]
    X = np.stack([a[1:-1], a[:-2]], axis=1)
    (p, q), *_ = np.linalg.lstsq(X, y, rcond=None)
    aa = 6 * amax
    g, d = (1 - aa) / (1 + aa), 1 / (1 + aa)
    S = o.coefficients()[O.C_S]
    K2 = sum(4 * math.sin(m[k] * math.pi / (2 * n[k])) ** 2 for k in range(3))
    assert abs(-q - g * g) < 1e-12                  # product of the roots
    assert abs(p - (2 * g - d * d * S * S * K2)) < 1e-12   # sum of the roots


def _te10_reflection(bcz, nx=8, beta0=2 * math.pi / 12, **kw):
    ny, nz = 2, 1200
    n = (nx, ny, nz)
    o = O.Oracle(O.default_params(n, noise=False, bc=(O.PEC, O.PEC, bcz), **kw))
    o.set_material(*I.homogeneous(n, 1.0, 0))
    o.set_pump(2e24, O.GROUND)
    kc, sig, kp = 500, 40.0, 900
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                             indexing="ij")
    ey = np.sin(math.pi * ii / nx) * np.exp(-0.5 * ((kk - kc) / sig) ** 2) * np.cos(beta0 * kk)
    ey[~I.interior_e_mask(n, 1)] = 0.0
    o.set_field(1, ey)
    S, dt = o.coefficients()[O.C_S], o.coefficients()[O.C_DT]
    betas = beta0 + np.linspace(-0.04, 0.04, 5)
    th = 2 * np.arcsin(S * np.sqrt(np.sin(math.pi / (2 * nx)) ** 2 + np.sin(betas / 2) ** 2))
    vg = S * S * math.sin(beta0) / math.sin(th[2])
    o.set_probes(np.array([(1, nx // 2, 0, kp)]), th / dt)
    t1 = int((kp - kc + 150) / vg)
    t2 = int((2 * nz - kp - kc + 150) / vg)
    o.step(t1)
    fi = o.spectrum()[0].copy()
    o.step(t2 - t1)
    return np.abs((o.spectrum()[0] - fi) / fi)


def _layer_loss(x, n, L=8, order=2, amax=0.25):
    # the graded profile: a_max ((L - x)/L)^order inside the low layer,
    # a_max ((x - (n - L))/L)^order inside the high one
    v = 0.0
    if x < L:
        v += ((L - x) / L) ** order
    if x > n - L:
        v += ((x - (n - L)) / L) ** order
    return amax * v


def test_lossy_layer_te10_response_is_the_transfer_recurrence_solution():
    """Exact discrete response of the graded layer.  A TE10 pulse (E_y =
    sin(pi i/nx) g(k), uniform in y, H = 0) in a PEC guide whose z ends carry
    the graded lossy layer.  With X^n = X e^{i phi n}, a site of loss a obeys
    (1+a) X' - (1-a) X = increment, i.e. D(a) X = increment with
    D(a) = (1+a) e^{i phi/2} - (1-a) e^{-i phi/2}; eliminating H_x (at z = k+1/2)
    and H_z (at z = k) leaves a three-term recurrence in E_y along z:
      D_k E_k = S^2 [(E_{k+1}-E_k)/D_{k+1/2} - (E_k-E_{k-1})/D_{k-1/2}]
                - mu S^2 E_k/D_k + (1+a_k) e^{i phi/2} g_k,
    mu = 4 sin^2(pi/(2 nx)), E_0 = E_nz = 0 (the conducting wall behind each
    layer).  The oracle's run, transformed over its whole decay, equals the
    solution of that system at every k, inside the layers too; and the
    reflection coefficient of the layer, from the homogeneous recurrence
    started at the wall, equals the ratio of the reflected to the incident
    wave that the oracle's field shows in the source-free part of the guide.
    A profile off by half a cell, a layer missing on one component or a
    different grading moves R by 1e-2; the check holds it to 1e-6."""
    nx, ny, nz = 8, 2, 400
    n = (nx, ny, nz)
    o = O.Oracle(O.default_params(n, noise=False, bc=(O.PEC, O.PEC, O.ABSORB)))
    o.set_material(*I.homogeneous(n, 1.0, 0))
    o.set_pump(2e24, O.GROUND)
    kc, sig, beta0 = 150, 14.0, 2 * math.pi / 12
    k = np.arange(nz + 1)
    g = np.exp(-0.5 * ((k - kc) / sig) ** 2) * np.cos(beta0 * k)
    g[0] = g[nz] = 0.0
    ey = np.broadcast_to(np.sin(math.pi * np.arange(nx + 1) / nx)[None, None, :] * g[:, None, None],
                         (nz + 1, ny + 1, nx + 1)).copy()
    ey[~I.interior_e_mask(n, 1)] = 0.0
    o.set_field(1, ey)
    S = o.coefficients()[O.C_S]
    mu = 4 * math.sin(math.pi / (2 * nx)) ** 2
    betas = beta0 + np.linspace(-0.1, 0.1, 5)
    phis = 2 * np.arcsin(S * np.sqrt(mu / 4 + np.sin(betas / 2) ** 2))   # TE10 dispersion
    F = np.zeros((len(phis), nz + 1), dtype=complex)
    line = g.copy()
    for step in range(8001):
        if step:
            o.step(1)
            line = o.field(1)[:, 0, nx // 2]
        F += line[None, :] * np.exp(-1j * phis * step)[:, None]
    aE = np.array([_layer_loss(q, nz) for q in range(nz + 1)])          # E_y, H_z: integer z
    aH = np.array([_layer_loss(q + 0.5, nz) for q in range(nz)])        # H_x: half z
    for phi, beta, Fo in zip(phis, betas, F):
        zh = np.exp(0.5j * phi)
        DE = (1 + aE) * zh - (1 - aE) / zh
        DH = (1 + aH) * zh - (1 - aH) / zh
        diag = DE[1:nz] + S * S / DH[1:nz] + S * S / DH[:nz - 1] + mu * S * S / DE[1:nz]
        A = np.diag(diag) - np.diag(S * S / DH[1:nz - 1], 1) - np.diag(S * S / DH[1:nz - 1], -1)
        sol = np.zeros(nz + 1, dtype=complex)
        sol[1:nz] = np.linalg.solve(A, (1 + aE[1:nz]) * zh * g[1:nz])
        assert np.max(np.abs(Fo - sol)) < 1e-6 * np.max(np.abs(sol))
        h = np.zeros(nz + 1, dtype=complex)
        h[nz - 1] = 1.0
        for q in range(nz - 1, 0, -1):
            h[q - 1] = ((DE[q] + S * S / DH[q] + S * S / DH[q - 1] + mu * S * S / DE[q]) * h[q]
                        - S * S * h[q + 1] / DH[q]) * DH[q - 1] / (S * S)

        def reflection(v, k1, k2, kref=300):
            # v_k = A e^{-i beta k} (towards +z) + B e^{+i beta k}
            M = np.array([[np.exp(-1j * beta * k1), np.exp(1j * beta * k1)],
                          [np.exp(-1j * beta * k2), np.exp(1j * beta * k2)]])
            a, b = np.linalg.solve(M, [v[k1], v[k2]])
            return b / a * np.exp(2j * beta * kref)
        R = reflection(h, 300, 310)
        assert 0.005 < abs(R) < 0.2
        for k1, k2 in ((290, 297), (320, 333)):          # past 9 sigma from the pulse
            assert abs(reflection(Fo, k1, k2) - R) < 1e-6


def test_lossy_layer_reflection_is_at_most_that_of_mur():
    # a guided wave at ~37 degrees and one near normal incidence
    for nx, beta0 in ((8, 2 * math.pi / 12), (24, 2 * math.pi / 20)):
        r_abs = _te10_reflection(O.ABSORB, nx=nx, beta0=beta0)
        r_mur = _te10_reflection(O.MUR1, nx=nx, beta0=beta0)
        assert np.max(r_abs) < 0.08
        assert np.mean(r_abs) < 1.2 * np.mean(r_mur)


def test_lossy_layer_stable_where_mur_grows():
    """A dielectric sphere tangent to an absorbing wall: first-order Mur turns
    the step into a growing map (the reason the lossy layer exists), the
    graded lossy layer keeps the field bounded."""
    n = (16, 16, 16)
    eps, _ = I.voxelize(I.Packing(n, np.array([[8.0, 8.0, 12.0]]), np.array([4.0])))
    out = {}
    for bc in (O.MUR1, O.ABSORB):
        o = O.Oracle(O.default_params(n, noise=False, bc=(O.PEC, O.PEC, bc)))
        o.set_material(eps, np.zeros_like(eps, dtype=np.uint8))
        o.set_pump(2e24, O.GROUND)
        f = I.random_fields(n, seed=5)
        for c in range(3):
            o.set_field(c, f[c].astype(np.float64))
        o.step(1500)
        out[bc] = math.sqrt(sum(float(np.sum(o.field(c) ** 2)) for c in range(3)))
    start = math.sqrt(sum(float(np.sum(f[c].astype(np.float64) ** 2)) for c in range(3)))
    assert out[O.MUR1] > 1e6 * start
    assert out[O.ABSORB] < start
