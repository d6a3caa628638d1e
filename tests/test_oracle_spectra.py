"""Pins of the oracle's spectral statistics (peak, moments and the Gaussian
fit of the emission spectra, Results section and Figs. 4-5) against closed
forms and hand-worked cases."""
import math

import numpy as np
import pytest

from oracle import spectra as S


def gaussian(omega, A, mu, sigma):
    return A * np.exp(-(omega - mu) ** 2 / (2.0 * sigma ** 2))


def one_probe(Sk):
    """Amplitudes of a single probe whose power spectrum is Sk."""
    return np.sqrt(np.asarray(Sk, dtype=np.float64))[None, :].astype(np.complex128)


@pytest.mark.parametrize("level", [0.05, 0.3, 0.5, 0.9])
def test_exact_gaussian_is_recovered(level):
    # a sampled Gaussian is a parabola in ln S: the fit returns it exactly
    om = np.linspace(3.0e15, 3.4e15, 401)
    A, mu, sig = 7.5, 3.2137e15, 6.0e12
    st = S.spectral_stats(one_probe(gaussian(om, A, mu, sig)), om, level)
    assert st["fit_ok"] == 1
    assert st["fit_center"] == pytest.approx(mu, rel=1e-12)
    assert st["fit_sigma"] == pytest.approx(sig, rel=1e-9)
    assert st["fit_amplitude"] == pytest.approx(A, rel=1e-9)
    # the peak is the sample nearest the centre
    assert st["peak_bin"] == int(np.argmin(np.abs(om - mu)))


def test_exact_gaussian_on_a_nonuniform_grid():
    om = 3.0e15 * np.exp(np.linspace(0.0, 0.12, 300))          # geometric spacing
    A, mu, sig = 2.0, 3.17e15, 1.1e13
    st = S.spectral_stats(one_probe(gaussian(om, A, mu, sig)), om, 0.2)
    assert st["fit_ok"] == 1
    assert st["fit_center"] == pytest.approx(mu, rel=1e-12)
    assert st["fit_sigma"] == pytest.approx(sig, rel=1e-8)
    assert st["fit_amplitude"] == pytest.approx(A, rel=1e-8)


def test_window_cut_by_the_band_edge():
    # centre left of the grid: the run starts at bin 0 and the fit still
    # extrapolates to the true centre
    om = np.linspace(3.0e15, 3.1e15, 200)
    A, mu, sig = 1.0, 2.99e15, 3.0e13
    st = S.spectral_stats(one_probe(gaussian(om, A, mu, sig)), om, 0.5)
    assert st["peak_bin"] == 0 and st["fit_lo"] == 0
    assert st["fit_center"] == pytest.approx(mu, rel=1e-10)
    assert st["fit_sigma"] == pytest.approx(sig, rel=1e-7)


def test_probes_add_their_powers():
    om = np.linspace(1.0, 2.0, 51)
    Sk = gaussian(om, 3.0, 1.43, 0.07)
    F = np.stack([np.sqrt(0.25 * Sk), 1j * np.sqrt(0.75 * Sk)])
    assert np.allclose(S.power_spectrum(F), Sk, rtol=1e-15, atol=0)
    st = S.spectral_stats(F, om, 0.3)
    assert st["fit_sigma"] == pytest.approx(0.07, rel=1e-9)
    assert st["total"] == pytest.approx(np.sum(Sk), rel=1e-14)


def test_moments_of_a_sampled_gaussian():
    # spacing << sigma: the discrete mean and standard deviation equal the
    # continuous ones (the aliasing error is exp(-2 pi^2 sigma^2 / h^2))
    om = np.linspace(2.5e15, 3.9e15, 2001)
    mu, sig = 3.21e15, 8.0e13
    st = S.spectral_stats(one_probe(gaussian(om, 1.0, mu, sig)), om, 0.5)
    assert st["mean_omega"] == pytest.approx(mu, rel=1e-12)
    assert st["std_omega"] == pytest.approx(sig, rel=1e-9)


def test_moments_of_two_lines():
    # two equal spikes at w1, w2: mean (w1+w2)/2, std |w2-w1|/2
    om = np.arange(10, dtype=np.float64)
    Sk = np.zeros(10)
    Sk[2] = Sk[7] = 4.0
    st = S.spectral_stats(one_probe(Sk), om, 0.5)
    assert st["mean_omega"] == 4.5 and st["std_omega"] == 2.5
    assert st["peak_bin"] == 2                      # first of equal maxima
    assert (st["fit_lo"], st["fit_hi"], st["fit_ok"]) == (2, 2, 0)


def test_hand_worked_window():
    Sk = [1.0, 2.0, 5.0, 9.0, 6.0, 1.0]
    om = np.arange(6, dtype=np.float64)
    st = S.spectral_stats(one_probe(Sk), om, 0.5)
    assert (st["peak_bin"], st["fit_lo"], st["fit_hi"]) == (3, 2, 4)
    # three bins: the parabola through ln(5/9), 0, ln(6/9) at x = -1, 0, 1
    y_m, y_p = math.log(5 / 9), math.log(6 / 9)
    c = 0.5 * (y_m + y_p)
    b = 0.5 * (y_p - y_m)
    assert st["fit_center"] == pytest.approx(3.0 - b / (2 * c), rel=1e-13)
    assert st["fit_sigma"] == pytest.approx(math.sqrt(-1.0 / (2 * c)), rel=1e-13)
    assert st["fit_amplitude"] == pytest.approx(9.0 * math.exp(-b * b / (4 * c)), rel=1e-13)
    st = S.spectral_stats(one_probe(Sk), om, 0.1)
    assert (st["fit_lo"], st["fit_hi"]) == (0, 5)
    # a bin exactly at level * S_peak belongs to the run (|F|^2 exact here)
    F = np.array([[1.0, 2.0, 4.0, 2.0, 1.0]], dtype=np.complex128)
    st = S.spectral_stats(F, np.arange(5.0), 0.25)
    assert (st["fit_lo"], st["fit_hi"]) == (1, 3)


def test_degenerate_spectra():
    om = np.linspace(1.0, 2.0, 8)
    st = S.spectral_stats(np.zeros((3, 8), dtype=np.complex128), om, 0.5)
    assert st["peak_bin"] == -1 and st["fit_ok"] == 0 and st["total"] == 0.0
    st = S.spectral_stats(one_probe(np.full(8, 2.0)), om, 0.5)          # flat: no downward parabola
    assert st["peak_bin"] == 0 and (st["fit_lo"], st["fit_hi"]) == (0, 7) and st["fit_ok"] == 0
    st = S.spectral_stats(one_probe([4.0]), np.array([3.0]), 0.5)        # one bin
    assert st["peak_bin"] == 0 and st["mean_omega"] == 3.0 and st["std_omega"] == 0.0
    assert st["fit_ok"] == 0


def test_fit_weights_are_the_squared_spectrum():
    # for data that is not a Gaussian the fit is the weighted least-squares
    # parabola with weights (S/S_peak)^2: its residual is orthogonal to
    # 1, x, x^2 under those weights (and not under S/S_peak)
    om = np.linspace(0.0, 1.0, 101)
    Sk = 1.0 / (1.0 + ((om - 0.52) / 0.05) ** 2)                         # a Lorentzian
    st = S.spectral_stats(one_probe(Sk), om, 0.2)
    lo, hi, kp = st["fit_lo"], st["fit_hi"], st["peak_bin"]
    s = (om[hi] - om[lo]) / (hi - lo)
    x = (om[lo:hi + 1] - om[kp]) / s
    u = Sk[lo:hi + 1] / Sk[kp]
    c = -s * s / (2.0 * st["fit_sigma"] ** 2)
    b = -2.0 * c * (st["fit_center"] - om[kp]) / s
    a = math.log(st["fit_amplitude"] / Sk[kp]) + b * b / (4.0 * c)
    r = np.log(u) - (a + b * x + c * x * x)
    X = np.stack([np.ones_like(x), x, x * x])
    assert np.max(np.abs(X @ (u * u * r))) < 1e-10
    assert np.max(np.abs(X @ (u * r))) > 1e-4


def test_peaks_hand_worked():
    # local maxima 1 (value 5), 4 (9), 7 (plateau 6, 6: first bin), edge 9 (7)
    Sk = [1.0, 5.0, 2.0, 3.0, 9.0, 4.0, 1.0, 6.0, 6.0, 7.0]
    F = one_probe(Sk)
    assert S.spectral_peaks(F, 0.0, 10) == [4, 9, 7, 1]
    assert S.spectral_peaks(F, 0.0, 2) == [4, 9]
    assert S.spectral_peaks(F, 0.6, 10) == [4, 9, 7]          # 5 < 0.6 * 9
    # the rule is local: the first bin of a flat run counts when nothing
    # higher follows right away (the run [3, 3] at the band edge), a falling
    # band edge counts, a flat run after a rise counts at its first bin only
    assert S.spectral_peaks(one_probe([3.0, 3.0, 5.0, 1.0]), 0.0, 5) == [2, 0]
    assert S.spectral_peaks(one_probe([8.0, 3.0, 3.0, 1.0]), 0.0, 5) == [0]
    assert S.spectral_peaks(one_probe([1.0, 4.0, 4.0, 4.0, 2.0]), 0.0, 5) == [1]
    assert S.spectral_peaks(np.zeros((2, 6), dtype=np.complex128), 0.0, 5) == []


def test_peaks_of_separated_lines():
    # three Gaussian lines of distinct heights on a quiet floor: one peak each,
    # in order of height, at the sample nearest each centre
    om = np.linspace(0.0, 1.0, 1001)
    lines = [(0.21, 0.01, 2.0), (0.55, 0.02, 5.0), (0.80, 0.005, 1.0)]
    Sk = sum(gaussian(om, A, mu, sg) for (mu, sg, A) in lines)
    got = S.spectral_peaks(one_probe(Sk), 0.05, 8)
    want = [int(np.argmin(np.abs(om - mu))) for (mu, _, _) in sorted(lines, key=lambda l: -l[2])]
    assert got == want
    # equal heights: lower bin first
    Sk = gaussian(om, 1.0, 0.3, 0.01) + gaussian(om, 1.0, 0.7, 0.01)
    assert S.spectral_peaks(one_probe(Sk), 0.5, 8) == [300, 700]
