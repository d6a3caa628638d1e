"""Bound states of the dimensionless Gross-Pitaevskii equation of the random
laser, plain numpy/scipy in FP64.

TEST INFRASTRUCTURE ONLY: used by the test-suite to check the library's
Gross-Pitaevskii solver, never by the product library.

The Gross-Pitaevskii section casts the oscillation condition in the form
(Eq. g5)  -phi'' + tau^2 phi + phi^3 = E phi, with E = (p-1)/(kappa sqrt(p))
(Eq. ee); bell-shaped solutions exist for E > 1 (threshold), and near it
phi ~ 2^{1/4} sqrt(E-1) exp(-tau^2/2).

Discretisation (the same discrete problem as the library's): M interior
points tau_i = -L + (i+1) h, h = 2L/(M+1), phi = 0 at +-L, second
differences, F(phi) = A phi + phi^3 - E phi with A = -D2 + diag(tau^2).
Solution path: the discrete linear ground state (lambda0, psi0) of A by a
symmetric eigen-solver; the first-order bifurcating branch
phi = a psi0, a^2 = (E - lambda0) / (h sum psi0^4) (psi0 with h sum psi0^2 = 1)
just above lambda0; then continuation in E up to the target, each stage
solved by Newton's method with a banded solver.  Spectrum:
phit(nu) = (h / 2 pi) sum_i phi_i cos(nu tau_i), S = phit^2 on nu_k = k dnu;
waist w = sigma_nu / (2 pi) with sigma_nu^2 = sum' nu^2 S / sum' S over the
even spectrum (k = 0 once, k >= 1 twice); peak S(0).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import eigh_tridiagonal, solve_banded


def grid(M: int, L: float):
    h = 2.0 * L / (M + 1)
    tau = -L + h * np.arange(1, M + 1)
    return tau, h


def residual(phi, E, tau, h):
    pl = np.concatenate(([0.0], phi[:-1]))
    pr = np.concatenate((phi[1:], [0.0]))
    return (2.0 * phi - pl - pr) / (h * h) + tau * tau * phi + phi ** 3 - E * phi


def linear_ground_state(M: int, L: float):
    """(lambda0, psi0) of A, psi0 > 0 with h sum psi0^2 = 1."""
    tau, h = grid(M, L)
    lam, vec = eigh_tridiagonal(2.0 / (h * h) + tau * tau, np.full(M - 1, -1.0 / (h * h)),
                                select="i", select_range=(0, 0))
    psi = vec[:, 0]
    psi = psi * np.sign(psi[M // 2]) / math.sqrt(h * np.sum(psi * psi))
    return float(lam[0]), psi


def newton(phi, E, tau, h, tol=1e-12, max_iter=100):
    """Newton's method on F(phi) = 0; a step is halved until the residual
    decreases and phi stays positive at the centre (the positive branch).
    Converged when the full update is below tol * max phi, or when the
    residual no longer decreases and is at its rounding level (near the
    bifurcation, where the Jacobian is nearly singular)."""
    M = phi.shape[0]
    scale = lambda q: 4.0 * float(np.max(np.abs(q))) / (h * h) + 1.0
    r0 = float(np.max(np.abs(residual(phi, E, tau, h))))
    for _ in range(max_iter):
        F = residual(phi, E, tau, h)
        ab = np.zeros((3, M))
        ab[0, 1:] = -1.0 / (h * h)
        ab[1, :] = 2.0 / (h * h) + tau * tau + 3.0 * phi * phi - E
        ab[2, :-1] = -1.0 / (h * h)
        delta = solve_banded((1, 1), ab, -F)
        t = 1.0
        while True:
            trial = phi + t * delta
            r1 = float(np.max(np.abs(residual(trial, E, tau, h))))
            if (r1 < r0 and trial[M // 2] > 0.0) or t < 1e-6:
                break
            t *= 0.5
        if not (r1 < r0 and trial[M // 2] > 0.0):
            return phi, r0 <= 1e-12 * scale(phi)
        phi, r0 = trial, r1
        if t == 1.0 and np.max(np.abs(delta)) <= tol * np.max(np.abs(phi)):
            return phi, True
    return phi, False


def gp_solve(E: float, M: int, L: float, n_nu: int, dnu: float) -> dict:
    tau, h = grid(M, L)
    lam0, psi0 = linear_ground_state(M, L)
    if not E > lam0:
        raise ValueError("no bound state below the linear threshold")
    q4 = h * float(np.sum(psi0 ** 4))
    # continuation along the branch from the bifurcation: E - lambda0 grows
    # geometrically (ratio <= 1.25) up to 0.5, then in steps of at most 0.25;
    # each stage starts from the secant through the last two solutions (the
    # first from the first-order law a^2 = (E - lambda0) / (h sum psi0^4))
    d1 = E - lam0
    ds = [min(1e-6, 0.5 * d1)]
    while ds[-1] < min(0.5, d1):
        ds.append(min(ds[-1] * 1.25, min(0.5, d1)))
    while ds[-1] < d1:
        ds.append(min(ds[-1] + 0.25, d1))
    sols = []
    for q, d in enumerate(ds):
        if q == 0:
            guess = math.sqrt(d / q4) * psi0
        elif q == 1:
            guess = sols[-1] * math.sqrt(d / ds[q - 1])
        else:
            guess = sols[-1] + (sols[-1] - sols[-2]) * (d - ds[q - 1]) / (ds[q - 1] - ds[q - 2])
        phi, ok = newton(guess, lam0 + d, tau, h)
        if not ok:
            raise RuntimeError(f"Newton did not converge at E = {lam0 + d}")
        sols = (sols + [phi])[-2:]
    nu = dnu * np.arange(n_nu)
    phit = (h / (2.0 * math.pi)) * (np.cos(np.outer(nu, tau)) @ phi)
    S = phit * phit
    wgt = np.where(np.arange(n_nu) == 0, 1.0, 2.0)
    s0 = float(np.sum(wgt * S))
    w = math.sqrt(float(np.sum(wgt * S * nu * nu)) / s0) / (2.0 * math.pi) if s0 > 0 else 0.0
    return dict(phi=phi, tau=tau, h=h, spec=S, N=h * float(np.sum(phi * phi)), w=w, peak=float(S[0]),
                phi_max=float(np.max(phi)), residual=float(np.max(np.abs(residual(phi, E, tau, h)))),
                converged=ok, lambda0=lam0, psi0=psi0)


def eigenvalue(p: float, kappa: float) -> float:
    """E(p) of Eq. ee."""
    return (p - 1.0) / (kappa * math.sqrt(p))


def threshold(kappa: float) -> float:
    """The pump at which E = 1 (root of E(p) = 1)."""
    return 1.0 + 0.5 * kappa * kappa + 0.5 * kappa * math.sqrt(4.0 + kappa * kappa)
