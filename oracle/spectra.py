"""Spectral statistics of emission spectra, plain numpy in FP64.

TEST INFRASTRUCTURE ONLY: used by the test-suite to check the library's
spectral-statistics kernel, never by the product library.

The linewidth the Results section compares with theory (Fig. 5b) comes from a
Gaussian fit of the Maxwell-Bloch spectra; the experimental widths (Fig. 4)
are the spectra's standard deviation.  Both are computed here from the
running-DFT amplitudes F[p, k] of the probes (the transform of the
Simulations section):

* S_k = sum_p |F[p, k]|^2, probes added one after another in index order;
* the peak is the first bin holding the largest S_k;
* mean and std are the first moment and the standard deviation of omega
  under the weight S;
* the fit uses the contiguous run of bins around the peak where
  S_k >= level * S_peak: a weighted least-squares parabola
  ln(S_k / S_peak) ~ a + b x + c x^2 with weights (S_k / S_peak)^2 and
  x = (omega_k - omega_peak) / s, s the mean bin spacing in the run; a
  Gaussian A exp(-(omega - mu)^2 / (2 sigma^2)) has c = -1 / (2 (sigma/s)^2),
  mu = omega_peak - s b / (2c), A = S_peak exp(a - b^2 / (4c)).  The fit
  needs three bins and c < 0.
"""
from __future__ import annotations

import numpy as np


def power_spectrum(F: np.ndarray) -> np.ndarray:
    """S_k of complex amplitudes F[p, k], probes added in index order."""
    F = np.asarray(F, dtype=np.complex128)
    S = np.zeros(F.shape[1])
    for p in range(F.shape[0]):
        re, im = F[p].real, F[p].imag
        S = S + (re * re + im * im)
    return S


def spectral_stats(F: np.ndarray, omega: np.ndarray, level: float = 0.5) -> dict:
    omega = np.asarray(omega, dtype=np.float64)
    S = power_spectrum(F)
    K = S.shape[0]
    total = float(np.sum(S))
    out = dict(total=total, peak_bin=-1, peak_omega=0.0, peak_value=0.0, mean_omega=0.0,
               std_omega=0.0, fit_lo=-1, fit_hi=-1, fit_ok=0, fit_center=0.0, fit_sigma=0.0,
               fit_amplitude=0.0)
    if not total > 0.0:
        return out
    kp = int(np.argmax(S))                      # first index of the maximum
    peak = float(S[kp])
    mean = float(np.sum(S * omega) / total)
    var = float(np.sum(S * (omega - mean) ** 2) / total)
    thr = level * peak
    lo = kp
    while lo > 0 and S[lo - 1] >= thr:
        lo -= 1
    hi = kp
    while hi < K - 1 and S[hi + 1] >= thr:
        hi += 1
    out.update(peak_bin=kp, peak_omega=float(omega[kp]), peak_value=peak, mean_omega=mean,
               std_omega=float(np.sqrt(var)), fit_lo=lo, fit_hi=hi)
    if hi - lo < 2 or omega[hi] == omega[lo]:
        return out
    s = (omega[hi] - omega[lo]) / (hi - lo)
    x = (omega[lo:hi + 1] - omega[kp]) / s
    u = S[lo:hi + 1] / peak
    sw = u                                      # sqrt of the weights u^2
    A = np.stack([np.ones_like(x), x, x * x], axis=1) * sw[:, None]
    coef, *_ = np.linalg.lstsq(A, np.log(u) * sw, rcond=None)
    a, b, c = (float(v) for v in coef)
    if c < 0.0:
        out.update(fit_ok=1, fit_center=float(omega[kp] + s * (-b / (2.0 * c))),
                   fit_sigma=float(abs(s) * np.sqrt(-1.0 / (2.0 * c))),
                   fit_amplitude=float(peak * np.exp(a - b * b / (4.0 * c))))
    return out


def spectral_peaks(F: np.ndarray, min_rel: float = 0.1, max_peaks: int = 16) -> list:
    """Bins of the spectral peaks: S_k > 0, S_k >= min_rel * max S and
    S_{k-1} < S_k >= S_{k+1} (a band-edge bin has one neighbour; a flat top
    counts at its first bin), largest first (equal values: lower bin first),
    at most max_peaks (the long-lived modes of a passive spectrum, Fig. 1)."""
    S = power_spectrum(F)
    K = S.shape[0]
    thr = min_rel * float(np.max(S)) if K else 0.0
    peaks = []
    for k in range(K):
        v = S[k]
        left_ok = k == 0 or S[k - 1] < v
        right_ok = k == K - 1 or v >= S[k + 1]
        if v > 0.0 and v >= thr and left_ok and right_ok:
            peaks.append(k)
    peaks.sort(key=lambda k: (-S[k], k))
    return peaks[:max_peaks]
