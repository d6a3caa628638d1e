"""Pins of the oracle's adjoint (rows a9/a10): the tangent-linear step against
central differences of the forward step, the adjoint step against the tangent
step (dot-product identity), and the whole gradient of the loss-box objective
against central differences of the forward run's own loss monitor."""
import numpy as np
import pytest

import oracle as O
from paper_0809_1547_amd import inputs as I

N = (10, 9, 8)
BOX = ((3, 3, 2), (7, 6, 6))


def material(seed=4):
    pk = I.rsa_pack(N, seed=seed, count=2, radius=2.5)
    return I.voxelize(pk)


def make(bc=(O.PEC,) * 3, init=O.PREPUMPED, Na=2e24, eps=None, gain=None, src=True, **kw):
    kw.setdefault("E_sp", 1e-2)
    o = O.Oracle(O.default_params(N, bc=bc, seed=3, realization=1, **kw))
    if eps is None:
        eps, gain = material()
    o.set_material(eps, gain)
    o.set_pump(Na, init)
    if src:
        o.set_source(2, 5, 4, 3, amp=0.3, lambda_s=560e-9, tau_p=0.5e-15, t0=1.5e-15)
    o.set_loss_box(*BOX)
    return o


def state(o):
    return [o.field(f) for f in range(24)]


def scaled_random(X, rng):
    # perturbation with the scale of each field group (E, H, P, P_prev, N1..N3, N0)
    out = []
    for g in range(8):
        scale = max(float(np.max(np.abs(np.concatenate([X[3 * g + c].ravel() for c in range(3)])))), 1e-12)
        out += [scale * rng.standard_normal(X[0].shape) for _ in range(3)]
    return out


def step_from(make_kw, X, nprev):
    o = make(**make_kw)
    o.step(nprev)
    for f in range(24):
        o.set_field(f, X[f])
    o.step(1)
    out = state(o)
    o.close()
    return out


def dot(a, b):
    return sum(float(np.sum(x * y)) for x, y in zip(a, b))


CASES = {
    "pec_gain_noise": dict(),
    "absorbing_layer": dict(bc=(O.ABSORB,) * 3, absorb_cells=3),
    "frozen_populations": dict(frozen_pop=True),
    "ground_start": dict(init=O.GROUND, Na=5e24),
}


@pytest.mark.parametrize("case", list(CASES))
def test_tangent_step_matches_central_differences(case):
    kw = CASES[case]
    o = make(**kw)
    o.step(25)
    X = state(o)
    v = scaled_random(X, np.random.default_rng(1))
    Jv = o.tangent_step(v)
    h = 1e-4
    Fp = step_from(kw, [x + h * d for x, d in zip(X, v)], 25)
    Fm = step_from(kw, [x - h * d for x, d in zip(X, v)], 25)
    fd = [(a - b) / (2 * h) for a, b in zip(Fp, Fm)]
    for g in range(8):
        num = sum(float(np.sum((Jv[3 * g + c] - fd[3 * g + c]) ** 2)) for c in range(3))
        den = sum(float(np.sum(fd[3 * g + c] ** 2)) for c in range(3))
        assert np.sqrt(num) <= 1e-7 * np.sqrt(den) + 1e-300, (case, g)
    o.close()


@pytest.mark.parametrize("case", list(CASES))
def test_adjoint_step_is_the_transpose(case):
    o = make(**CASES[case])
    o.step(25)
    X = state(o)
    rng = np.random.default_rng(2)
    v = scaled_random(X, rng)
    w = scaled_random(X, rng)
    lhs = dot(o.tangent_step(v), w)
    rhs = dot(v, o.adjoint_step(w))
    mag = sum(float(np.sum(np.abs(a * b))) for a, b in zip(o.tangent_step(v), w))
    assert abs(lhs - rhs) <= 1e-13 * mag, (case, lhs, rhs)
    o.close()


def objective(kw, eps, gain, nsteps, Na=None):
    kw = dict(kw)
    if Na is not None:
        kw["Na"] = Na
    o = make(eps=eps, gain=gain, **kw)
    o.step(nsteps)
    L = o.loss()
    o.close()
    return L


@pytest.mark.parametrize("case", ["pec_gain_noise", "absorbing_layer", "ground_start"])
def test_gradient_matches_central_differences(case):
    kw = CASES[case]
    eps, gain = material()
    nsteps = 60
    o = make(eps=eps, gain=gain, **kw)
    L, g_eps, g_na = o.adjoint_run(nsteps)
    o.close()
    assert L == pytest.approx(objective(kw, eps, gain, nsteps), rel=1e-14)
    # eps_r of cells in and around the box, in voids and in spheres
    rng = np.random.default_rng(5)
    cells = [(int(rng.integers(2, 8)), int(rng.integers(2, 7)), int(rng.integers(1, 7))) for _ in range(8)]
    fd, ad = [], []
    for (i, j, k) in cells:
        e0 = float(eps[k, j, i])
        ep, em = eps.copy(), eps.copy()
        ep[k, j, i] = np.float32(e0 * (1 + 1e-5))
        em[k, j, i] = np.float32(e0 * (1 - 1e-5))
        h2 = float(ep[k, j, i]) - float(em[k, j, i])     # the perturbation binary32 can hold
        fd.append((objective(kw, ep, gain, nsteps) - objective(kw, em, gain, nsteps)) / h2)
        ad.append(g_eps[k, j, i])
    fd, ad = np.array(fd), np.array(ad)
    assert np.linalg.norm(ad - fd) <= 1e-6 * np.linalg.norm(fd), (case, ad, fd)
    Na = kw.get("Na", 2e24)
    # L depends weakly on N_a (a relative change of a few 1e-3 per unit
    # relative change): a step of 1e-4 N_a keeps the difference above the
    # rounding of L, and its truncation error (order h^2) is ~1e-8
    hN = 1e-4 * Na
    fdn = (objective(kw, eps, gain, nsteps, Na + hN) - objective(kw, eps, gain, nsteps, Na - hN)) / (2 * hN)
    assert abs(g_na - fdn) <= 1e-6 * abs(fdn), (case, g_na, fdn)
    assert abs(fdn) > 0


def test_adjoint_refuses_mur_walls_and_late_start():
    o = make(bc=(O.MUR1, O.PEC, O.PEC))
    with pytest.raises(ValueError):
        o.adjoint_run(5)
    o.close()
    o = make()
    o.step(1)
    with pytest.raises(ValueError):
        o.adjoint_run(5)
    o.close()
