"""Pins of the oracle's soft-sphere compression packing (the sample's granular
packing of spheres obtained by molecular dynamics, Simulations section; read
as overdamped soft-sphere compression in a closed box).  Each pin is fixed by
mechanics, not by the oracle: the closed-form relaxation of one contact and of
one wall contact, through the whole growth schedule; momentum conservation;
descent of the energy; the force as the gradient of the energy; rest states;
mirror and relabelling symmetry; the end state of a 0.4-fill compression."""
import math

import numpy as np
import pytest

import oracle as O
from paper_0809_1547_amd import inputs as I


def _schedule(s0, stages, iters, final_iters):
    out = []
    for m in range(stages + 1):
        s = s0 + (1.0 - s0) * m / stages if stages > 0 else 1.0
        out += [s] * (iters if m < stages else final_iters)
    return out


@pytest.mark.parametrize("s0,stages,iters,final_iters,eta", [(1.0, 0, 0, 12, 0.15), (0.4, 3, 5, 7, 0.15),
                                                            (0.7, 6, 2, 3, 0.05)])
def test_one_contact_relaxes_in_closed_form(s0, stages, iters, final_iters, eta):
    # two spheres of diameters 6 and 8 (contact distance 7 s) at distance 5 on
    # a generic axis, far from the walls: each moves eta (s sigma - r) apart, so
    # r <- r + 2 eta (s sigma - r) while r < s sigma; the midpoint stays
    box = np.array([60.0, 60.0, 60.0])
    u = np.array([1.0, 2.0, -2.0]) / 3.0
    mid = np.array([30.0, 29.0, 31.0])
    r = 5.0
    x = np.array([mid - 0.5 * r * u, mid + 0.5 * r * u])
    d = np.array([6.0, 8.0])
    got = O.pack_md(box, d, x, s0=s0, stages=stages, iters=iters, final_iters=final_iters, eta=eta)
    for s in _schedule(s0, stages, iters, final_iters):
        if r < 7.0 * s:
            r = r + 2.0 * eta * (7.0 * s - r)
    want = np.array([mid - 0.5 * r * u, mid + 0.5 * r * u])
    assert np.max(np.abs(got - want)) <= 1e-12 * 60.0
    assert np.allclose(got.mean(axis=0), mid, rtol=0, atol=1e-12 * 60.0)


def test_wall_contacts_relax_in_closed_form():
    # one sphere of diameter 10 pressed 3 into the x = 0 wall and 2 into the
    # z = L wall: x_n = 5 - 3 (1-eta)^n, z_n = 55 + 2 (1-eta)^n, y fixed
    box = np.array([60.0, 50.0, 60.0])
    x = np.array([[2.0, 30.0, 57.0]])
    eta, n = 0.15, 9
    got = O.pack_md(box, np.array([10.0]), x, stages=0, final_iters=n, eta=eta)
    want = np.array([[5.0 - 3.0 * (1 - eta) ** n, 30.0, 55.0 + 2.0 * (1 - eta) ** n]])
    assert np.max(np.abs(got - want)) <= 1e-13 * 60.0


def test_pair_forces_conserve_momentum():
    # a cluster of 50 overlapping spheres in the middle of a large box: the pair
    # forces cancel in pairs, so the centroid does not move
    rng = np.random.default_rng(5)
    x = 100.0 + 6.0 * rng.random((50, 3))
    d = 3.0 + rng.random(50)
    box = np.array([200.0, 200.0, 200.0])
    got = O.pack_md(box, d, x, stages=0, final_iters=200, eta=0.1)
    assert np.max(np.abs(got.mean(axis=0) - x.mean(axis=0))) <= 1e-12 * 200.0
    assert O.pack_energy(box, d, got)[0] < 1e-3 * O.pack_energy(box, d, x)[0]


def test_energy_descends_step_by_step():
    box, d, x = I.pack_start((30, 26, 22), seed=2, fill=0.35, mean_d=5.0, sd_d=0.5)
    U = [O.pack_energy(box, d, x)[0]]
    for _ in range(60):
        x = O.pack_md(box, d, x, stages=0, final_iters=1, eta=0.05)
        U.append(O.pack_energy(box, d, x)[0])
    assert U[0] > 1.0 and all(b <= a for a, b in zip(U, U[1:]))
    assert U[-1] < 0.2 * U[0]


@pytest.mark.parametrize("s", [1.0, 0.8])
def test_step_is_the_energy_gradient(s):
    # one step moves x by -eta grad U_s: check every coordinate of a few spheres
    # (pair and wall contacts) against central differences of the energy; s is
    # set through a one-stage schedule of one step
    box, d, x = I.pack_start((24, 20, 18), seed=3, fill=0.3, mean_d=5.0, sd_d=0.5)
    eta = 0.1
    if s == 1.0:
        y = O.pack_md(box, d, x, stages=0, final_iters=1, eta=eta)
    else:
        y = O.pack_md(box, d, x, s0=s, stages=1, iters=1, final_iters=0, eta=eta)
    F = (y - x) / eta
    h = 1e-6
    checked = 0
    for i in range(len(d)):
        if not np.any(F[i]):
            continue
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(O.pack_energy(box, d, xp, s)[0] - O.pack_energy(box, d, xm, s)[0]) / (2 * h)
            assert abs(fd - F[i, a]) <= 1e-6 * max(1.0, abs(F[i, a]))
        checked += 1
        if checked == 12:
            break
    assert checked == 12


def test_separated_spheres_are_at_rest():
    # a simple-cubic arrangement with gaps (and clear of the walls) feels no
    # force: the centres come back bit for bit
    g = np.arange(4) * 7.0 + 4.0
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    d = np.full(x.shape[0], 6.5)
    box = np.array([29.0, 29.0, 29.0])
    got = O.pack_md(box, d, x, s0=0.5, stages=4, iters=3, final_iters=10, eta=0.15)
    assert np.array_equal(got, x)
    assert O.pack_energy(box, d, got) == (0.0, 0.0)


def test_mirror_and_relabelling_symmetry():
    box, d, x = I.pack_start((30, 28, 26), seed=4, fill=0.4, mean_d=5.0, sd_d=0.5)
    kw = dict(s0=0.6, stages=10, iters=10, final_iters=100, eta=0.15)
    ref = O.pack_md(box, d, x, **kw)
    for a in range(3):
        xm = x.copy()
        xm[:, a] = box[a] - xm[:, a]
        got = O.pack_md(box, d, xm, **kw)
        got[:, a] = box[a] - got[:, a]
        assert np.max(np.abs(got - ref)) <= 1e-9 * box[a]
    perm = np.random.default_rng(0).permutation(len(d))
    got = O.pack_md(box, d[perm], x[perm], **kw)
    assert np.max(np.abs(got - ref[perm])) <= 1e-9 * 30.0


def test_compression_reaches_the_target_fill_without_overlap():
    box, d, x = I.pack_start((40, 36, 32), seed=1, fill=0.4, mean_d=6.0, sd_d=0.6)
    assert math.pi / 6 * np.sum(d ** 3) >= 0.4 * np.prod(box)
    assert math.pi / 6 * np.sum(d[:-1] ** 3) < 0.4 * np.prod(box)
    U0, ov0 = O.pack_energy(box, d, x)
    assert ov0 > 3.0
    y = O.pack_md(box, d, x, s0=0.5, stages=100, iters=20, final_iters=1000, eta=0.15)
    U, ov = O.pack_energy(box, d, y)
    assert ov <= 1e-4 * 6.0 and U <= 1e-6 * U0
    r = 0.5 * d[:, None]
    assert np.all(y - r >= -ov) and np.all(y + r <= box + ov)


def test_bad_arguments():
    with pytest.raises(ValueError):
        O.pack_md(np.ones(3), np.ones(2), np.zeros((2, 3)), stages=-1)
    assert O.pack_md(np.ones(3), np.zeros(0), np.zeros((0, 3))).shape == (0, 3)
