"""Lasing threshold and ST-law linewidth fit, plain numpy/scipy in FP64.

TEST INFRASTRUCTURE ONLY: used by the test-suite to check the library's
threshold and kappa fits, never by the product library.

Threshold (the E = 1 point of the Gross-Pitaevskii section, found on the
simulations themselves): each run of a pump sweep starts from the pumped
state with a small excitation (a seeded field, or a pulse with no DC
content) and no noise; in the linear regime its
energy follows the least-damped mode, W^n ~ exp(2 gamma n dt), so
    rate(N_a) = least-squares slope of ln W^n over the steps n0 <= n < n1
(per step), and the threshold N_th is the root of the least-squares line
rate = a + b N_a through the sweep (the net gain is linear in the inversion).

Linewidth fit (Gross-Pitaevskii section, Eqs. ee, s1, wth and the waist of
the numerical solution, Fig. 5b): with p = p_th(kappa) N_a / N_th (p_th the
root of E(p) = 1), E(p) = (p - 1) / (kappa sqrt(p)) and the spectral waist
(in frequency omega / 2 pi) W = w_phi(E) sqrt(kappa) / (p^{1/4} t_g), kappa
minimises sum_i (ln W_model(N_a,i) - ln W_i)^2.  w_phi is the waist of the
bound state of Eq. g5 (oracle.gp).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import minimize_scalar

from . import gp as G


def growth_rate(W: np.ndarray, n0: int, n1: int) -> float:
    """Least-squares slope of ln W^n against n over n0 <= n < n1."""
    n = np.arange(n0, n1, dtype=np.float64)
    slope, _ = np.polyfit(n, np.log(np.asarray(W, dtype=np.float64)[n0:n1]), 1)
    return float(slope)


def threshold(Na: np.ndarray, rates: np.ndarray):
    """(a, b, N_th) of the least-squares line rate = a + b N_a and its root."""
    b, a = np.polyfit(np.asarray(Na, dtype=np.float64), np.asarray(rates, dtype=np.float64), 1)
    return float(a), float(b), float(-a / b)


def knee(x, y):
    """Two straight lines joined at a knee (the linewidth-vs-pump collapse of
    Fig. 5b): for every split s, points [0, s) and [s, n) with at least two
    each, the least-squares line of each part and the summed squared
    residuals; the split with the smallest sum (the first on ties) and the
    crossing of its two lines, kept between x[s-1] and x[s] (their midpoint
    when the lines do not cross at a finite point).  Returns (knee, s,
    (aL, bL), (aR, bR), residual sum)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]

    def line(i0, i1):
        b, a = np.polyfit(x[i0:i1], y[i0:i1], 1)
        r = y[i0:i1] - (a + b * x[i0:i1])
        return a, b, float(np.sum(r * r))
    best, best_sse = None, None
    for s in range(2, n - 1):
        sse = line(0, s)[2] + line(s, n)[2]
        if best_sse is None or sse < best_sse:
            best, best_sse = s, sse
    aL, bL, _ = line(0, best)
    aR, bR, _ = line(best, n)
    lo, hi = x[best - 1], x[best]
    with np.errstate(divide="ignore", invalid="ignore"):
        k = (aR - aL) / (bL - bR)
    if not np.isfinite(k):
        k = 0.5 * (lo + hi)
    k = min(max(k, lo), hi)
    return float(k), best, (aL, bL), (aR, bR), best_sse


def model_waist(Na, kappa: float, N_th: float, t_g: float, M: int, L: float, n_nu: int, dnu: float):
    """W_model(N_a) in Hz (frequency omega / 2 pi) for every N_a above
    threshold (E(p) > 1)."""
    pth = G.threshold(kappa)
    out = []
    for na in np.atleast_1d(Na):
        p = pth * float(na) / N_th
        E = G.eigenvalue(p, kappa)
        w = G.gp_solve(E, M, L, n_nu, dnu)["w"]
        out.append(w * math.sqrt(kappa) / (p ** 0.25 * t_g))
    return np.array(out)


def kappa_fit(Na, W, N_th: float, t_g: float, M: int, L: float, n_nu: int, dnu: float,
              lo: float = 1e-3, hi: float = 10.0, xtol: float = 1e-10):
    """kappa minimising the squared log misfit, searched over ln kappa in
    [ln lo, ln hi] (bounded Brent); a kappa for which some pump level's
    eigenvalue would not fit the window (E > (0.7 L)^2, Thomas-Fermi radius
    sqrt(E)) or whose bound state does not converge is rejected.  Returns
    (kappa, W_model at kappa)."""
    Na = np.asarray(Na, dtype=np.float64)
    lw = np.log(np.asarray(W, dtype=np.float64))
    E_cap = (0.7 * L) ** 2

    def f(u):
        k = math.exp(u)
        pth = G.threshold(k)
        if max(G.eigenvalue(pth * na / N_th, k) for na in Na) > E_cap:
            return 1e30
        try:
            return float(np.sum((np.log(model_waist(Na, k, N_th, t_g, M, L, n_nu, dnu)) - lw) ** 2))
        except RuntimeError:
            return 1e30
    r = minimize_scalar(f, bounds=(math.log(lo), math.log(hi)), method="bounded",
                        options={"xatol": xtol, "maxiter": 500})
    k = math.exp(r.x)
    return k, model_waist(Na, k, N_th, t_g, M, L, n_nu, dnu)
