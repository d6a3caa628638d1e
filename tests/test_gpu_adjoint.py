"""GPU adjoint of the loss-box objective (checkpoints + reverse sweep) against
the FP64 oracle's adjoint, across checkpoint intervals, and, on the adjoint
workload (96^3 x 1000, K = 50), against central differences of an FP64
forward run."""
import numpy as np
import pytest

import oracle as O
from paper_0809_1547_amd import inputs as I

pytestmark = pytest.mark.gpu

N = (10, 9, 8)
BOX = ((3, 3, 2), (7, 6, 6))
SRC = (2, 5, 4, 3)


def _mbf():
    from paper_0809_1547_amd import mbf
    return mbf


def _material(n=N, seed=4, **kw):
    kw = kw or dict(count=2, radius=2.5)
    return I.voxelize(I.rsa_pack(n, seed=seed, **kw))


def _pair(n, bc, init, Na, precision, eps, gain, box=BOX, src=SRC, **phys):
    mbf = _mbf()
    phys.setdefault("E_sp", 1e-2)
    kinds = {"pec": O.PEC, "absorb": O.ABSORB, "mur": O.MUR1}
    sim = mbf.Sim(n, boundary=bc, precision=precision, seed=3, realization=1, **phys)
    ora = O.Oracle(O.default_params(n, bc=(kinds[bc],) * 3, round_f32=(precision == "fp32"), seed=3,
                                    realization=1, **phys))
    for x in (sim, ora):
        x.set_material(eps, gain)
    sim.set_pump(Na, init)
    ora.set_pump(Na, O.PREPUMPED if init == "prepumped" else O.GROUND)
    if src:
        sim.set_source(*src, amp=0.3, lambda_s=560e-9, tau_p=0.5e-15, t0=1.5e-15)
        ora.set_source(*src, amp=0.3, lambda_s=560e-9, tau_p=0.5e-15, t0=1.5e-15)
    sim.set_loss_box(*box)
    ora.set_loss_box(*box)
    return sim, ora


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.mark.parametrize("bc,init,Na,n,absorb_cells", [
    ("pec", "prepumped", 2e24, N, 8),
    ("absorb", "prepumped", 2e24, N, 3),
    ("pec", "ground", 5e24, N, 8),
    ("absorb", "prepumped", 3e24, (70, 13, 21), 4),
])
def test_fp64_adjoint_matches_oracle(bc, init, Na, n, absorb_cells):
    eps, gain = _material(n, fill=0.35) if n != N else _material()
    src = SRC if n == N else (2, 40, 6, 10)
    box = BOX if n == N else ((30, 4, 6), (50, 10, 15))
    sim, ora = _pair(n, bc, init, Na, "fp64", eps, gain, box=box, src=src, absorb_cells=absorb_cells)
    Lg, gg, ng = sim.adjoint_run(60, K=13)
    Lo, go, no = ora.adjoint_run(60)
    print(bc, init, "L", Lg, Lo, "g_eps rel", _rel(gg, go), "g_Na", ng, no)
    assert Lg == pytest.approx(Lo, rel=1e-12)
    assert _rel(gg, go) <= 1e-10
    assert ng == pytest.approx(no, rel=1e-10)


def test_fp32_adjoint_matches_oracle():
    eps, gain = _material()
    sim, ora = _pair(N, "pec", "prepumped", 2e24, "fp32", eps, gain)
    Lg, gg, ng = sim.adjoint_run(60, K=60)
    Lo, go, no = ora.adjoint_run(60)
    print("fp32: L rel", abs(Lg - Lo) / Lo, "g_eps rel", _rel(gg, go), "g_Na rel", abs(ng - no) / abs(no))
    assert Lg == pytest.approx(Lo, rel=1e-5)
    assert _rel(gg, go) <= 1e-4
    assert ng == pytest.approx(no, rel=1e-4)


def test_checkpoint_interval_does_not_change_the_gradient_and_run_ends_at_nsteps():
    # nor does the schedule of the forward (the split and fused variants
    # recompute the segments and record the trajectory as well)
    mbf = _mbf()
    eps, gain = _material((40, 36, 28), seed=3, fill=0.4)
    out = []
    for K, var in ((90, None), (7, None), (32, None), (32, "two_pass_split"), (7, "fused"), (9, "fused_lds"),
                   (11, "fused_persistent")):
        sim = mbf.Sim((40, 36, 28), boundary="absorb", seed=9, realization=3, E_sp=1e-3)
        if var:
            sim.set_tuning(var, tile_y=4, zseg=2, xcd_remap=2)
        sim.set_material(eps, gain)
        sim.set_pump(2e24)
        sim.set_source(2, 20, 18, 14, amp=0.2)
        sim.set_loss_box((10, 10, 8), (30, 26, 20))
        out.append(sim.adjoint_run(90, K=K) + (sim.step_index, [sim.field(f) for f in range(21)]))
        sim.close()
    ref = mbf.Sim((40, 36, 28), boundary="absorb", seed=9, realization=3, E_sp=1e-3)
    ref.set_material(eps, gain)
    ref.set_pump(2e24)
    ref.set_source(2, 20, 18, 14, amp=0.2)
    ref.set_loss_box((10, 10, 8), (30, 26, 20))
    ref.step(90)
    # the fields, the eps gradient (summed per cell in step order) and the N_a
    # gradient (the reverse steps' own work items) are the same bit for bit;
    # the loss is a sum of per-work-item partials of the forward kernels, so
    # its last bits follow the schedule's partition of the grid
    for L, g, gna, step, fields in out:
        assert L == pytest.approx(out[0][0], rel=1e-14)
        assert gna == out[0][2] and np.array_equal(g, out[0][1])
        assert step == 90
        for a, b in zip(fields, [ref.field(f) for f in range(21)]):
            assert np.array_equal(a, b)
    assert out[0][0] == ref.loss()


def test_adjoint_errors():
    mbf = _mbf()
    eps, gain = _material()
    sim = mbf.Sim(N, boundary="mur")
    sim.set_material(eps, gain)
    sim.set_pump(2e24)
    sim.set_loss_box(*BOX)
    with pytest.raises(mbf.MbfError) as e:
        sim.adjoint_run(5)
    assert e.value.code == mbf.MBF_EINVAL
    sim = mbf.Sim(N)
    sim.set_material(eps, gain)
    sim.set_pump(2e24)
    with pytest.raises(mbf.MbfError) as e:
        sim.adjoint_run(5)                  # no loss box
    assert e.value.code == mbf.MBF_ESTATE
    sim.set_loss_box(*BOX)
    sim.step(1)
    with pytest.raises(mbf.MbfError) as e:
        sim.adjoint_run(5)                  # not at step 0
    assert e.value.code == mbf.MBF_ESTATE


def _c4_sim(precision, eps, gain, Na=2e24):
    mbf = _mbf()
    sim = mbf.Sim(96, boundary="pec", precision=precision, seed=0, realization=0)
    sim.set_material(eps, gain)
    sim.set_pump(Na, "prepumped")
    sim.set_loss_box((40, 40, 40), (56, 56, 56))
    return sim


def test_c4_adjoint_against_fp64_differences():
    # 96^3 x 1000 steps, K = 50, FP32 adjoint; central differences of the FP64
    # forward at 20 cells within 8 cells of the box (h = 1e-4 on eps_r, as
    # binary32 holds it) and at N_a (h = 1e-4 N_a)
    import time
    eps, gain = I.voxelize(I.packing_for("c4", 96, 0))
    nsteps = 1000
    # cost: three pairs of a fresh adjoint run (it must start from the pump)
    # and a fresh forward run of the same steps, after one warm-up pair; the
    # median ratio of reverse sweep to forward must stay within 3
    ratios = []
    for it in range(4):
        sim = _c4_sim("fp32", eps, gain)
        sim.sync()
        t0 = time.perf_counter()
        L, g, gna = sim.adjoint_run(nsteps, K=50)
        t_adj = time.perf_counter() - t0
        sim.close()
        sim = _c4_sim("fp32", eps, gain)
        sim.step(8)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(nsteps)
        sim.sync()
        t_fwd = time.perf_counter() - t0
        sim.close()
        if it:
            ratios.append((t_adj - t_fwd) / t_fwd)
    med = float(np.median(ratios))
    print(f"C4: forward {t_fwd * 1e3:.1f} ms, forward+adjoint {t_adj * 1e3:.1f} ms, "
          f"reverse sweep / forward = {['%.2f' % r for r in ratios]} (median {med:.2f})")
    assert med <= 3.0
    rng = np.random.default_rng(0)
    cells = []
    while len(cells) < 20:
        c = tuple(int(x) for x in rng.integers(32, 64, size=3))
        if c not in cells:
            cells.append(c)

    def L64(e, Na=2e24):
        s = _c4_sim("fp64", e, gain, Na)
        s.step(nsteps)
        v = s.loss()
        s.close()
        return v

    fd, ad = [], []
    for (i, j, k) in cells:
        ep, em = eps.copy(), eps.copy()
        ep[k, j, i] = np.float32(float(eps[k, j, i]) + 1e-4)
        em[k, j, i] = np.float32(float(eps[k, j, i]) - 1e-4)
        h2 = float(ep[k, j, i]) - float(em[k, j, i])
        fd.append((L64(ep) - L64(em)) / h2)
        ad.append(g[k, j, i])
    err = _rel(ad, fd)
    hN = 1e-4 * 2e24
    fdn = (L64(eps, 2e24 + hN) - L64(eps, 2e24 - hN)) / (2 * hN)
    errn = abs(gna - fdn) / abs(fdn)
    print(f"C4: eps gradient error {err:.2e} over 20 cells, N_a gradient error {errn:.2e}")
    assert err <= 1e-3
    assert errn <= 1e-3


def test_torch_autograd_binding():
    import torch
    from paper_0809_1547_amd.autograd import loss_box_objective
    eps, gain = _material()
    e = torch.tensor(eps, requires_grad=True)
    Na = torch.tensor(2e24, dtype=torch.float64, requires_grad=True)
    setup = dict(n=N, gain=gain, box=BOX, nsteps=40, K=9, init="prepumped", source=(*SRC, 0.3),
                 precision="fp64", seed=3, realization=1, E_sp=1e-2)
    L = loss_box_objective(e, Na, setup)
    L.backward()
    mbf = _mbf()
    sim = mbf.Sim(N, precision="fp64", seed=3, realization=1, E_sp=1e-2)
    sim.set_material(eps, gain)
    sim.set_pump(2e24)
    sim.set_source(*SRC, amp=0.3)
    sim.set_loss_box(*BOX)
    L2, g2, gna2 = sim.adjoint_run(40, K=9)
    assert L.item() == L2
    assert np.array_equal(e.grad.numpy(), g2.astype(np.float32))
    assert Na.grad.item() == gna2


def test_torch_autograd_binding_on_device():
    # eps as a device tensor: the library reads it and writes the gradient
    # through device pointers on torch's current stream (a side stream here);
    # the result equals the host path's bit for bit
    import torch
    from paper_0809_1547_amd.autograd import loss_box_objective
    eps, gain = _material()
    setup = dict(n=N, gain=gain, box=BOX, nsteps=40, K=9, init="prepumped", source=(*SRC, 0.3),
                 precision="fp64", seed=3, realization=1, E_sp=1e-2)
    eh = torch.tensor(eps, requires_grad=True)
    Nh = torch.tensor(2e24, dtype=torch.float64, requires_grad=True)
    Lh = loss_box_objective(eh, Nh, setup)
    Lh.backward()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ed = torch.tensor(eps, device="cuda", requires_grad=True)
        Nd = torch.tensor(2e24, dtype=torch.float64, requires_grad=True)
        Ld = loss_box_objective(ed, Nd, setup)
        Ld.backward()
    st.synchronize()
    assert ed.grad.is_cuda and ed.grad.dtype == ed.dtype
    assert Ld.item() == Lh.item() and Nd.grad.item() == Nh.grad.item()
    assert np.array_equal(ed.grad.cpu().numpy(), eh.grad.numpy())
