"""Throughput benchmark of the Maxwell-Bloch FDTD step on one MI355X.

Workload (default, --workload c5): the paper-scale realization -- 320^3 cells
(6.4 um box, 7245 spheres of diameter 300 +- 30 nm, index 2.9, fill 0.4, packed
by the library's soft-sphere compression, gain in the voids), ground-state start, spontaneous-emission noise, 256 probe
sites with running DFT spectra over 450-800 nm at the resolution of the full
3 ps run, graded absorbing walls -- advanced as a batch of 5 pump levels
N_a in {1, 2, 3.5, 5, 7} x 1e24 m^-3, one launch of each step kernel per
time step for all 5.  One bench step = one time step of all 5 realizations
(5 x 320^3 cell-updates).

--workload c3: 64 small realizations of uneven size (N in {48, 64, 80, 96}),
prepumped, stepped as one autotuned batch and then one at a time through the
plain path; both rates are printed.

Prints ONE JSON line: cell-updates/s of the graph-replayed batched steps,
the roofline of the dominant kernel (HBM bound: algorithmic bytes per launch
/ average launch duration, from HIP events around every launch on its stream
in a following pass of up to 64 steps), the FP64 CPU oracle timed on a
bounded sample of the same workload (plus windows of the other workloads),
and three legs: the batch of small realizations against the same members
one at a time and side by side, the adjoint's cost over the forward, and
whole runs of the cache-resident single-grid workloads.

`python bench.py --summarize-profile DIR` prints, as markdown, the kernel
table or the per-dispatch counter means of the rocprofv3 database(s) under
DIR (used to write the summaries kept with the sources).
"""
import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
DENSE_BYTES_PER_CU = 157.0      # 21 FP32 values read, 18 written, material byte
NA_LEVELS = [1e24, 2e24, 3.5e24, 5e24, 7e24]
RUN_STEPS_3PS = 78675          # 3 ps at dt = 3.81315e-17 s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--n", type=int, default=320, help="cells per side")
    ap.add_argument("--batch", type=int, default=5)
    ap.add_argument("--workload", choices=["c5", "c3", "pack", "gp"], default="c5",
                    help="c5: 320^3 batch of pump levels (default); c3: 64 small realizations "
                         "of uneven size, batched against one at a time; pack: the soft-sphere "
                         "compression packing of the 320^3 sample; gp: Gross-Pitaevskii bound "
                         "states of a 256-point pump sweep")
    ap.add_argument("--pack-runs", type=int, default=5, help="timed packings of --workload pack")
    ap.add_argument("--packing", choices=["rsa", "md"], default="md",
                    help="c5 sample: the library's soft-sphere compression packing (default; random "
                         "sequential addition stalls near a nominal fill of 0.36 at 320^3) or RSA at 0.36")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick-cpu", action="store_true", help="time only 2 oracle steps of the c5 realization")
    ap.add_argument("--no-legs", action="store_true",
                    help="c5: skip the batched (c3, reduced), adjoint (c4) and single-grid (c1, c2, c4) legs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain elementwise kernel of known traffic (counter calibration)")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="summarise rocprofv3 results under DIR and exit")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the calibrated HBM traffic summary of --kernel from two rocprofv3 "
                         "--pmc runs (FETCH_SIZE, WRITE_SIZE, each with --calib-copy) and exit")
    ap.add_argument("--kernel", default="k_curl_e_batch")
    ap.add_argument("--tuning", default="two_pass_split/4/2/2",
                    help="variant/tile_y/zseg/xcd_remap the counter runs used")
    return ap.parse_args()


CALIB_BYTES = 1 << 30          # the calibration kernel reads 1 GiB and writes 1 GiB


def pmc_means(d):
    """{(kernel name, counter): mean per dispatch} of the rocprofv3 databases under d."""
    import glob
    import sqlite3
    acc = {}
    for path in sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)):
        db = sqlite3.connect(path)
        for name, _, cn, val in db.execute(
                "select kernel_name, dispatch_id, counter_name, sum(value) from counters_collection "
                "group by dispatch_id, counter_name"):
            acc.setdefault((name, cn), []).append(val)
        db.close()
    return {k: sum(v) / len(v) for k, v in acc.items()}


def write_traffic(fetch_dir, write_dir, kernel, workload, tuning):
    """profiles/<kernel>_<workload>_traffic.md from a FETCH_SIZE and a
    WRITE_SIZE run, each calibrated by the plain add kernel of --calib-copy
    (reads and writes CALIB_BYTES)."""
    f, w = pmc_means(fetch_dir), pmc_means(write_dir)

    def pick(m, counter, pred):
        hits = [(k[0], v) for k, v in m.items() if k[1] == counter and pred(k[0])]
        if len(hits) != 1:
            raise SystemExit(f"expected one kernel for {counter}, found {[h[0] for h in hits]}")
        return hits[0]
    is_k = lambda name: name.startswith(f"void mbf::{kernel}<float")
    is_cal = lambda name: "CUDAFunctorOnSelf_add<float>" in name
    kname, kf = pick(f, "FETCH_SIZE", is_k)
    _, kw = pick(w, "WRITE_SIZE", is_k)
    _, cf = pick(f, "FETCH_SIZE", is_cal)
    _, cw = pick(w, "WRITE_SIZE", is_cal)
    ff = CALIB_BYTES / (cf * 1024.0)
    fw = CALIB_BYTES / (cw * 1024.0)
    rd, wr = kf * 1024.0 * ff, kw * 1024.0 * fw
    cmd = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc {c} -d $OUT/{d} -o run -- "
           "python3 $REPO/bench.py --workload " + workload + " --steps 8 --warmup 4 --no-cpu-baseline --no-legs "
           "--calib-copy")
    out = f"""# HBM traffic of `{kernel}` on the {workload} bench workload

Kernel: `{kname}`

Commands ($REPO the repository, $OUT a scratch directory; the bench's own launch
configuration, 8 timed steps; counters per dispatch):

    {cmd.format(c="FETCH_SIZE", d="fetch")}
    {cmd.format(c="WRITE_SIZE", d="write")}
    python3 bench.py --write-traffic $OUT/fetch $OUT/write --kernel {kernel} --workload {workload} --tuning {tuning}

Calibration: the plain elementwise add of `--calib-copy` reads and writes {CALIB_BYTES} B.
FETCH_SIZE reads {cf:.6g} KiB for it (factor {ff:.4f}: the counter counts a 128-byte request
as 64 bytes); WRITE_SIZE reads {cw:.6g} KiB (factor {fw:.4f}).

| | counter KiB / dispatch | factor | bytes / dispatch |
|---|---:|---:|---:|
| read (FETCH_SIZE) | {kf:.6g} | {ff:.4f} | {rd:.6g} |
| write (WRITE_SIZE) | {kw:.6g} | {fw:.4f} | {wr:.6g} |

traffic_bytes_per_launch: {rd + wr:.6g}
kernel_source_sha256: {kernel_source_sha()}
tuning: {tuning}
"""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    open(path, "w").write(out)
    print(out)


def summarize_profile(d):
    """Markdown digest of rocprofv3 databases (kernel trace or counters)."""
    import glob
    import sqlite3
    dbs = sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True))
    if not dbs:
        print(f"no rocprofv3 database under {d}", file=sys.stderr)
        sys.exit(1)
    for path in dbs:
        db = sqlite3.connect(path)
        print(f"### {os.path.relpath(path, d)}\n")
        n_pmc = db.execute("select count(*) from counters_collection").fetchone()[0]
        if n_pmc == 0:
            rows = db.execute("select name, count(*), sum(duration), avg(duration), "
                              "min(duration), max(duration) from kernels group by name "
                              "order by sum(duration) desc").fetchall()
            total = sum(r[2] for r in rows) or 1
            print("| kernel | calls | total ms | average us | min us | max us | % |")
            print("|---|---:|---:|---:|---:|---:|---:|")
            for name, calls, tot, avg, lo, hi in rows:
                print(f"| `{name}` | {calls} | {tot / 1e6:.3f} | {avg / 1e3:.2f} | {lo / 1e3:.2f} | "
                      f"{hi / 1e3:.2f} | {100.0 * tot / total:.2f} |")
        else:
            rows = db.execute(
                "select kernel_name, dispatch_id, counter_name, sum(value) from counters_collection "
                "group by dispatch_id, counter_name").fetchall()
            acc = {}
            for name, _, cn, val in rows:
                acc.setdefault((name, cn), []).append(val)
            print("| kernel | counter | dispatches | mean per dispatch |")
            print("|---|---|---:|---:|")
            for (name, cn), vals in sorted(acc.items()):
                print(f"| `{name}` | {cn} | {len(vals)} | {sum(vals) / len(vals):.6g} |")
        print()
        db.close()


def traffic_from_profiles(kernel, workload, tuning, kernel_sha):
    """Calibrated HBM bytes per launch of `kernel` from the committed counter
    summary, if it was taken on the current kernel source and schedule."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    s = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", txt)
    t = re.search(r"tuning:\s*(\S+)", txt)
    want = f"{tuning['variant']}/{tuning['tile_y']}/{tuning['zseg']}/{tuning['xcd_remap']}"
    if not m or not s or s.group(1) != kernel_sha or not t or t.group(1) != want:
        return None
    return float(m.group(1))


def kernel_source_sha():
    """Hash of the source that defines the step kernels (their launch shape is
    the tuning, recorded beside it)."""
    import hashlib
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "paper_0809_1547_amd", "csrc", "mbf_kernels.hpp"), "rb").read())
    return h.hexdigest()[:16]


def _omp_threads(k):
    """Set the OpenMP thread count of the calling thread (the oracle's
    parallel regions run on libgomp)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))


def oracle_window(O, n, eps, gain, bc, init, Na, steps, threads):
    """Cell-updates/s of the FP64 oracle, as it stands, over `steps` steps of
    one realization (after one untimed step that pages the arrays in)."""
    _omp_threads(threads)
    p = O.default_params(n, bc=(bc,) * 3, seed=0, realization=0)
    o = O.Oracle(p)
    o.set_material(eps, gain)
    o.set_pump(Na, init)
    o.step(1)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    o.close()
    return n ** 3 * steps / dt, dt


def oracle_adjoint_window(O, I, threads, n=12, steps=1000):
    """The oracle's adjoint (FP64) at n^3: the wall time of its whole
    forward + reverse run over `steps` steps from the pump (PEC, two spheres,
    the soft pulse, loss box [4, 8)^3), beside a plain forward run of the same
    steps; cell-updates/s counts the forward steps."""
    _omp_threads(threads)
    eps, gain = I.voxelize(I.rsa_pack(n, seed=0, count=2, radius=2.5))

    def fresh():
        o = O.Oracle(O.default_params(n, bc=(O.PEC,) * 3, seed=0, realization=0))
        o.set_material(eps, gain)
        o.set_pump(2e24, O.PREPUMPED)
        o.set_source(2, n // 2, n // 2, n // 2, amp=0.3, lambda_s=560e-9, tau_p=0.5e-15, t0=1.5e-15)
        o.set_loss_box((4, 4, 4), (8, 8, 8))
        return o
    o = fresh()
    t0 = time.perf_counter()
    o.adjoint_run(steps)
    t_adj = time.perf_counter() - t0
    o.close()
    o = fresh()
    t0 = time.perf_counter()
    o.step(steps)
    t_fwd = time.perf_counter() - t0
    o.close()
    log(f"oracle adjoint {n}^3 x {steps} steps on {threads} core(s): {t_adj:.2f} s "
        f"(forward alone {t_fwd:.3f} s)")
    return {"workload": "c4-adjoint", "n": n, "steps": steps, "cores": threads,
            "value": n ** 3 * steps / t_adj, "seconds": t_adj, "forward_seconds": t_fwd,
            "reverse_over_forward": (t_adj - t_fwd) / t_fwd}


def cpu_baseline(I, n5, eps5, gain5, quick=False):
    """The FP64 oracle timed on the machine's host cores: the paper-scale
    realization (the metric's workload) on every core of the affinity mask,
    plus windows of the other workloads, on every core and on one core."""
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    mats = {
        "c1": (32, I.voxelize(I.packing_for("c1", 32, 0)), O.PEC, O.PREPUMPED),
        "c2": (128, I.voxelize(I.packing_for("c2", 128, 0)), O.ABSORB, O.PREPUMPED),
        "c4": (96, I.voxelize(I.packing_for("c4", 96, 0)), O.PEC, O.PREPUMPED),
        "c5": (n5, (eps5, gain5), O.ABSORB, O.GROUND),
    }
    # the batched workload's four grid sizes (graded absorbing layer)
    for n3 in (48, 64, 80, 96):
        mats[f"c3/{n3}"] = (n3, I.voxelize(I.packing_for("c3", n3, 0)), O.ABSORB, O.PREPUMPED)
    # (workload, steps on all cores, steps on one core)
    plan = [("c1", 500, 100), ("c2", 200, 10), ("c3/48", 100, 10), ("c3/64", 100, 10), ("c3/80", 100, 10),
            ("c3/96", 100, 10), ("c4", 100, 10), ("c5", 10, 1)]
    if quick:
        plan = [("c5", 2, 0)]
    windows = []
    for name, s_all, s_one in plan:
        n, (eps, gain), bc, init = mats[name]
        for threads, steps in ((cores, s_all), (1, s_one)):
            if steps == 0:
                continue
            v, dt = oracle_window(O, n, eps, gain, bc, init, 2e24, steps, threads)
            windows.append({"workload": name, "n": n, "steps": steps, "cores": threads,
                            "value": v, "seconds": dt})
            log(f"oracle {name} {n}^3 x {steps} steps on {threads} core(s): {v:.3e} cu/s ({dt:.1f} s)")
    if not quick:
        for threads in (cores, 1):
            windows.append(oracle_adjoint_window(O, I, threads))
    _omp_threads(cores)
    main = next(w for w in windows if w["workload"] == "c5" and w["cores"] == cores)
    return {"value": main["value"], "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{main['steps']} steps of one {n5}^3 realization of the paper-scale workload "
                      f"(N_a = 2e24, ground start, absorbing walls, FP64, {cores} OpenMP threads), "
                      "after one untimed step",
            "windows": windows}


def c5_batch(args, I, mbf, stream):
    """The paper-scale workload: a batch of pump levels on one 320^3 packing."""
    n = args.n
    t0 = time.perf_counter()
    if args.packing == "md":
        # the soft-sphere compression packing, computed by the library
        box, d, x = I.pack_start(n, seed=0, fill=0.4)
        x, _, ov = mbf.mbf_pack_md(box, d, x, stream=stream.cuda_stream, **PACK_SCHEDULE)
        pk = I.packing_from_centres(n, d, x)
        log(f"compression packing: largest overlap {ov:.2e} cells")
    else:
        pk = I.rsa_pack(n, seed=0, fill=0.36)
    eps, gain = I.voxelize(pk)
    log(f"packing: {pk.count} spheres, voxel fill {1 - gain.mean():.3f} ({time.perf_counter() - t0:.1f} s)")
    probes = I.select_probes(eps, gain, 256, seed=0)
    cfgs = [mbf.make_config(n, boundary="absorb", seed=0, realization=r) for r in range(args.batch)]
    batch = mbf.Batch(cfgs, stream=stream.cuda_stream)
    om = None
    for r, s in enumerate(batch.members):
        s.set_material(eps, gain)
        s.set_pump(NA_LEVELS[r % len(NA_LEVELS)], "ground")
        dt = s.coefficients()[mbf.MBF_C_DT]
        om = I.dft_omegas(450e-9, 800e-9, RUN_STEPS_3PS, dt)
        s.set_probes(probes, om, decim=32)
    log(f"set-up of {args.batch} x {n}^3 done ({time.perf_counter() - t0:.1f} s), {len(om)} DFT bins")
    config = {
        "workload": f"paper-scale realization {n}^3 x batch of {args.batch} pump levels "
                    f"({'compression-packed' if args.packing == 'md' else 'RSA'} spheres d=300nm n=2.9 "
                    f"fill 0.4, gain in voids, ground start, "
                    f"noise, 256 probes x {len(om)} DFT bins, absorbing walls)",
        "cells_per_realization": n ** 3,
        "batch": args.batch,
        "pump_levels_m3": [NA_LEVELS[r % len(NA_LEVELS)] for r in range(args.batch)],
        # the sample as built: sphere count, achieved diameter mean and sd, voxel fill
        "spheres": pk.count,
        "diameter_nm_mean_sd": [round(float(np.mean(2.0 * pk.radii)) * I.DX * 1e9, 2),
                                round(float(np.std(2.0 * pk.radii)) * I.DX * 1e9, 2)],
        "voxel_fill": round(float(1.0 - gain.mean()), 4),
    }
    return batch, n ** 3 * args.batch, config, (eps, gain)


def c3_batch(args, I, mbf, stream):
    """Many small realizations of uneven size: 64 packings with N drawn from
    {48, 64, 80, 96} behind the graded absorbing layer, prepumped, with
    noise, at eight pump levels relative to each packing's own threshold
    (found first by a pulse-excited pump sweep of every packing)."""
    from paper_0809_1547_amd import sweep
    R = 64
    sizes = I.batch_sizes(R, seed=0)
    mats = [I.voxelize(I.rsa_pack(N, seed=r, fill=0.4)) for r, N in enumerate(sizes)]
    t0 = time.perf_counter()
    n_th, _ = sweep.packing_thresholds(mats, sizes, stream=stream.cuda_stream)
    log(f"c3 thresholds ({time.perf_counter() - t0:.1f} s): " +
        ", ".join(f"{N}^3 {np.mean([t for t, m in zip(n_th, sizes) if m == N]):.3g}" for N in sorted(set(sizes))))
    levels = I.batch_pump_levels(R, n_th)
    cfgs = [mbf.make_config(N, boundary="absorb", seed=0, realization=r) for r, N in enumerate(sizes)]
    batch = mbf.Batch(cfgs, stream=stream.cuda_stream)
    for r in range(R):
        batch[r].set_material(*mats[r])
        batch[r].set_pump(levels[r], "prepumped")
    cells = sum(N ** 3 for N in sizes)
    config = {
        "workload": f"{R} realizations of uneven size (N in {{48,64,80,96}}, {cells} cells in all), "
                    "RSA spheres d=300nm n=2.9 fill 0.4, prepumped, noise, graded absorbing layer, "
                    "8 pump levels 0.5..4 x each packing's threshold from a pump sweep",
        "sizes": sizes,
        "n_th_by_size": {str(N): float(np.mean([t for t, m in zip(n_th, sizes) if m == N]))
                         for N in sorted(set(sizes))},
    }
    return batch, cells, config, (sizes, mats, levels)


def one_at_a_time(mbf, sizes, mats, levels, steps, stream, concurrent=False, reps=1):
    """The same realizations stepped through the plain path, each with its own
    graph and its grid's own default schedule: one after another on the
    batch's stream (concurrent=False, so that one runs at a time), or each on
    a stream of its own, all launched before any is waited for
    (concurrent=True).  Cell-updates/s over the wall time between two
    device-wide synchronisations; the median of `reps` such windows."""
    import torch
    sims, streams = [], []
    for r, N in enumerate(sizes):
        st = torch.cuda.Stream() if concurrent else stream
        streams.append(st)
        s = mbf.Sim(N, boundary="absorb", seed=0, realization=r, stream=st.cuda_stream)
        s.set_material(*mats[r])
        s.set_pump(levels[r], "prepumped")
        s.step(32)
        sims.append(s)
    rates = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in sims:
            s.step(steps)
        torch.cuda.synchronize()
        rates.append(sum(N ** 3 for N in sizes) * steps / (time.perf_counter() - t0))
    for s in sims:
        s.close()
    return float(np.median(rates))


def c3_leg(args, I, mbf, steps=256, budget_ms=3000, reps=5):
    """The batched workload of many small realizations, reduced to `steps`
    steps: the autotuned batch against the same 64 realizations run one at a
    time (serially on one stream) and run side by side (a stream each); each
    rate the median of `reps` windows of `steps` steps."""
    import torch
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    batch, cells, config, (sizes, mats, levels) = c3_batch(args, I, mbf, stream)
    tuning = batch.autotune(budget_ms=budget_ms)
    batch.step(32)
    rates = []
    for _ in range(reps):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        batch.step(steps)
        torch.cuda.synchronize()
        rates.append(cells * steps / (time.perf_counter() - w0))
    batched = float(np.median(rates))
    batch.close()
    serial = one_at_a_time(mbf, sizes, mats, levels, steps, stream, reps=reps)
    conc = one_at_a_time(mbf, sizes, mats, levels, steps, stream, concurrent=True, reps=reps)
    log(f"c3 leg ({steps} steps, {time.perf_counter() - t0:.1f} s): batched {batched:.3e}, one at a time "
        f"{serial:.3e}, side by side {conc:.3e} cu/s; tuning {tuning}")
    return {"workload": config["workload"], "steps": steps, "windows": reps, "tuning": tuning,
            "batched": batched, "one_at_a_time": serial, "side_by_side": conc,
            "batched_over_one_at_a_time": batched / serial, "batched_over_side_by_side": batched / conc}


def configs_leg(I, mbf, runs=10, warm=3):
    """The cache-resident workloads on the GPU: C1 (32^3 x 500, PEC), C2
    (128^3 x 5000, graded absorbing layer) and C4 (96^3 x 1000, PEC), each
    pre-pumped at N_a = 2e24 with noise, FP32, the default schedule for its
    size.  Each config's whole run is timed with events on the handle's
    stream (graph-replayed chunks), `warm` untimed runs first, then the median
    of `runs` (the state carries on from run to run)."""
    import torch
    out = []
    for name, n, steps, bc in (("c1", 32, 500, "pec"), ("c2", 128, 5000, "absorb"), ("c4", 96, 1000, "pec")):
        eps, gain = I.voxelize(I.packing_for(name, n, 0))
        stream = torch.cuda.Stream()
        s = mbf.Sim(n, boundary=bc, precision="fp32", seed=0, realization=0, stream=stream.cuda_stream)
        s.set_material(eps, gain)
        s.set_pump(2e24, "prepumped")
        ms = []
        for q in range(warm + runs):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.step(steps)
            e1.record(stream)
            e1.synchronize()
            if q >= warm:
                ms.append(e0.elapsed_time(e1))
        s.energy()                        # raises on a non-finite energy
        tun = s.tuning()
        s.close()
        med = float(np.median(ms))
        out.append({"workload": name, "n": n, "steps": steps, "boundary": bc,
                    "value": n ** 3 * steps / (med / 1e3), "unit": "cell-updates/s",
                    "ms_median": med, "ms_min": float(min(ms)), "ms_max": float(max(ms)), "runs": runs,
                    "tuning": tun})
        log(f"{name} {n}^3 x {steps}: median {med:.2f} ms ({n ** 3 * steps / (med / 1e3):.3e} cu/s) over "
            f"{runs} runs")
    return out


def adjoint_leg(I, mbf, runs=3):
    """The adjoint workload (96^3, 1000 steps, K = 50, FP32, PEC, loss box
    [40, 56)^3): wall time of the reverse sweep (mbf_adjoint_run minus a
    plain forward run of the same steps) over the plain forward run; the
    median of `runs` ratios, each from a fresh handle (the adjoint run starts
    from the pump)."""
    import torch
    eps, gain = I.voxelize(I.packing_for("c4", 96, 0))

    def fresh():
        s = mbf.Sim(96, boundary="pec", seed=0, realization=0)
        s.set_material(eps, gain)
        s.set_pump(2e24, "prepumped")
        s.set_loss_box((40, 40, 40), (56, 56, 56))
        return s
    ratios, fw, ad = [], [], []
    for _ in range(runs + 1):                    # the first pair warms up
        s = fresh()
        s.sync()
        t0 = time.perf_counter()
        s.adjoint_run(1000, K=50)
        t_adj = time.perf_counter() - t0
        s.close()
        s = fresh()
        s.step(8)
        s.sync()
        t0 = time.perf_counter()
        s.step(1000)
        s.sync()
        t_fwd = time.perf_counter() - t0
        s.close()
        ratios.append((t_adj - t_fwd) / t_fwd)
        fw.append(t_fwd)
        ad.append(t_adj)
    ratios, fw, ad = ratios[1:], fw[1:], ad[1:]
    med = float(np.median(ratios))
    log(f"adjoint leg: reverse sweep / forward = {['%.2f' % r for r in ratios]} (median {med:.2f}); "
        f"forward {np.median(fw) * 1e3:.1f} ms, forward + adjoint {np.median(ad) * 1e3:.1f} ms")
    return {"workload": "96^3 x 1000 steps, K = 50, FP32, PEC, loss box [40,56)^3",
            "reverse_over_forward_median": med, "ratios": ratios, "within_3x": med <= 3.0,
            "forward_ms": float(np.median(fw) * 1e3), "forward_plus_adjoint_ms": float(np.median(ad) * 1e3)}


PACK_SCHEDULE = dict(s0=0.5, stages=100, iters=20, final_iters=1000, eta=0.15)


def pack_bench(args, I, mbf, stream):
    """The 320^3 sample (6.4 um box, 0.4 fill of 300 nm +- 10% spheres)
    packed by soft-sphere compression on the GPU, inputs resident in device
    memory; the oracle (all pairs, FP64) timed on a few steps of the same
    input."""
    import torch
    n = args.n
    box, d, x = I.pack_start(n, seed=11, fill=0.4)
    steps = PACK_SCHEDULE["stages"] * PACK_SCHEDULE["iters"] + PACK_SCHEDULE["final_iters"]
    log(f"packing: {len(d)} spheres in {n}^3, {steps} steps per packing")
    dt = torch.tensor(d, device="cuda")
    x0 = torch.tensor(x, device="cuda")
    xt = x0.clone()
    sid = stream.cuda_stream
    mbf.mbf_pack_md(box, dt, xt, stream=sid, **PACK_SCHEDULE)          # warm-up
    times = []
    for _ in range(args.pack_runs):
        xt.copy_(x0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, U, ov = mbf.mbf_pack_md(box, dt, xt, stream=sid, **PACK_SCHEDULE)
        times.append(time.perf_counter() - t0)
    best = min(times)
    value = len(d) * steps / best
    log(f"packing: best {best * 1e3:.1f} ms of {args.pack_runs} ({np.mean(times) * 1e3:.1f} mean), "
        f"{best / steps * 1e6:.2f} us per step; U = {U:.3e}, largest overlap {ov:.3e}")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        O.pack_md(box, d, x, stages=0, final_iters=1)                # page in
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < min(args.cpu_seconds, 10.0) and k < 200:
            O.pack_md(box, d, x, stages=0, final_iters=1)
            k += 1
        el = time.perf_counter() - t0
        cores = len(os.sched_getaffinity(0))
        cpu = {"value": len(d) * k / el, "unit": "sphere-steps/s", "cores": cores, "kind": "oracle",
               "sample": f"{k} steps of the same {len(d)} spheres (all pairs, FP64, {cores} OpenMP threads)"}
        log(f"cpu baseline: {cpu}")
    out = {"metric": "sphere-steps/s", "value": value, "unit": "sphere-steps/s", "n_gpus": 1,
           "steps": steps, "warmup": 1, "ms_per_step": best / steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"soft-sphere compression packing, {n}^3 box, fill 0.4, 300 nm +- 10% "
                                  f"spheres ({len(d)}), schedule {PACK_SCHEDULE}",
                      "spheres": len(d), "ms_per_packing": best * 1e3, "energy": U, "max_overlap": ov},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


GP_M, GP_L, GP_NU, GP_DNU = 1023, 14.0, 512, 0.02


def gp_bench(args, mbf, stream):
    """Bound states of the Gross-Pitaevskii equation for a pump sweep: 256
    eigenvalues from just above threshold to E = 30 (log-spaced in E - 1),
    1023 points on [-14, 14], 512 spectrum points; the oracle (continuation
    and Newton in FP64 numpy) timed on a sample of the same eigenvalues."""
    E = 1.0 + np.logspace(-3, math.log10(29.0), 256)
    sid = stream.cuda_stream
    mbf.mbf_gp_solve(E, M=GP_M, L=GP_L, n_nu=GP_NU, dnu=GP_DNU, stream=sid)       # warm-up
    times = []
    for _ in range(args.pack_runs):
        t0 = time.perf_counter()
        g = mbf.mbf_gp_solve(E, M=GP_M, L=GP_L, n_nu=GP_NU, dnu=GP_DNU, stream=sid)
        times.append(time.perf_counter() - t0)
    best = min(times)
    ok = int(np.sum(g["converged"]))
    log(f"gp: {len(E)} bound states in {best * 1e3:.2f} ms (best of {args.pack_runs}), {ok} converged, "
        f"Newton steps {int(np.min(g['newton_steps']))}-{int(np.max(g['newton_steps']))}")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import gp as OG
        t0 = time.perf_counter()
        k = 0
        for e in E[::16]:
            OG.gp_solve(float(e), GP_M, GP_L, GP_NU, GP_DNU)
            k += 1
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        cpu = {"value": k / el, "unit": "bound states/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} of the 256 eigenvalues (every 16th), continuation and Newton in FP64 numpy"}
        log(f"cpu baseline: {cpu}")
    out = {"metric": "bound states/s", "value": len(E) / best, "unit": "bound states/s", "n_gpus": 1,
           "steps": len(E), "warmup": 1, "ms_per_step": best / len(E) * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"Gross-Pitaevskii bound states, {len(E)} eigenvalues 1.001-30, "
                                  f"M = {GP_M}, L = {GP_L}, {GP_NU} spectrum points",
                      "ms_per_sweep": best * 1e3, "converged": ok},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile)
        return
    if args.write_traffic:
        t = args.tuning.split("/")
        write_traffic(args.write_traffic[0], args.write_traffic[1], args.kernel, args.workload,
                      "/".join(t[:4]))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is a design note, not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_0809_1547_amd import inputs as I
    from paper_0809_1547_amd import mbf

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if args.workload == "pack":
        pack_bench(args, I, mbf, stream)
        return
    if args.workload == "gp":
        gp_bench(args, mbf, stream)
        return
    if args.workload == "c3":
        batch, cells, config, extra = c3_batch(args, I, mbf, stream)
        tuning = batch.autotune(budget_ms=6000)
        log(f"autotuned: {tuning}")
    else:
        batch, cells, config, extra = c5_batch(args, I, mbf, stream)
        # the schedule a sweep picks at this size: two passes (the E pass
        # prefetching only the dense fields, H written by streaming stores),
        # tiles of 64 x 4 columns over 2-plane segments, layers dealt to the
        # XCDs in turn
        batch.set_tuning("two_pass_split", tile_y=4, zseg=2, xcd_remap=2)
        tuning = batch.tuning()
    config["tuning"] = tuning
    batch.step(args.warmup)
    batch.sync()
    log("warm-up done")

    # throughput: the production path (graph-replayed chunks of batched steps)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    batch.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_ms = ev0.elapsed_time(ev1)
    for s in batch.members:
        s.energy()                        # raises on a non-finite energy
    value = cells * args.steps / (wall_ms / 1e3)
    # kernel roofline: the same kernels launched step by step with HIP events
    # around them on the batch's stream
    kern_ms, launches = batch.step_timed(min(args.steps, 64))
    alg = batch.step_bytes()
    two_pass = tuning["variant"].startswith("two_pass")
    # the dominant kernel: the fused step kernel, or the longer of the two passes
    q = 1 if two_pass and kern_ms[1] >= kern_ms[0] else 0
    kname = ("k_curl_e_batch" if q else "k_curl_h_batch") if two_pass else "k_step_fused_batch"
    kdesc = {"k_curl_e_batch": "k_curl_e_batch (rows a2-a6: Ampere update, Lorentz polarisation, "
                               "rate equations, noise, walls; one launch per step for all realizations)",
             "k_curl_h_batch": "k_curl_h_batch (row a1: Faraday update and the energy partials)",
             "k_step_fused_batch": "k_step_fused_batch (rows a1-a6 in one launch per step for all "
                                   "realizations)"}[kname]
    alg_bytes = alg[1 + q] if two_pass else alg[0]
    avg_kern_s = kern_ms[q] / launches / 1e3
    achieved = alg_bytes / avg_kern_s / 1e9
    sha = kernel_source_sha()
    traffic = traffic_from_profiles(kname, args.workload, tuning, sha)
    log(f"timed {args.steps} batched steps: {wall_ms:.1f} ms; kernel pass per launch "
        f"{kern_ms[0] / launches:.3f} + {kern_ms[1] / launches:.3f} ms; "
        f"{alg[0] / cells:.1f} alg. B/cell per step; kernel source {sha}")

    if args.workload == "c5":
        # the linewidth analysis of the run's spectra (once per run, not per
        # step); with --steps 78675 --warmup 0 this is the whole 3 ps run
        t0 = time.perf_counter()
        stats = batch.spectrum_stats(0.5)
        st_ms = (time.perf_counter() - t0) * 1e3
        log(f"spectral statistics of {len(stats)} members ({batch[0]._np} probes x {batch[0]._nf} bins): "
            f"{st_ms:.2f} ms wall")
        c0 = 299792458.0
        for r, q in enumerate(stats):
            if q["peak_bin"] < 0:
                continue
            lam = 2.0 * math.pi * c0 / q["peak_omega"]
            to_nm = lam * lam / (2.0 * math.pi * c0) * 1e9      # d(lambda)/d(omega) at the peak
            log(f"  N_a = {NA_LEVELS[r % len(NA_LEVELS)]:.2e}: W = {batch[r].energy()[0]:.3e}, peak "
                f"{lam * 1e9:.1f} nm, std {q['std_omega'] * to_nm:.1f} nm, Gaussian-fit sigma "
                f"{q['fit_sigma'] * to_nm:.2f} nm")

    if args.calib_copy:
        a = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.add(a, 1.0, out=b)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b

    # what a plain streaming copy reaches on this device (reads 1 GiB, writes
    # 1 GiB; best of 10, events on torch's stream where the add runs)
    a = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.add(a, 1.0, out=b)
    best_copy = float("inf")
    for _ in range(10):
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        torch.add(a, 1.0, out=b)
        c1.record()
        c1.synchronize()
        best_copy = min(best_copy, c0.elapsed_time(c1) / 1e3)
    copy_gbs = 2.0 * CALIB_BYTES / best_copy / 1e9
    del a, b
    log(f"plain copy: {copy_gbs:.0f} GB/s (the dominant kernel reaches {achieved / copy_gbs:.1%} of it)")

    cpu = None
    extra_out = {}
    if args.workload == "c3":
        batch.close()
        sizes, mats, levels = extra
        solo = one_at_a_time(mbf, sizes, mats, levels, args.steps, stream)
        conc = one_at_a_time(mbf, sizes, mats, levels, args.steps, stream, concurrent=True)
        extra_out["one_at_a_time"] = {"value": solo, "unit": "cell-updates/s",
                                      "ratio_batched_over_solo": value / solo}
        extra_out["side_by_side"] = {"value": conc, "unit": "cell-updates/s",
                                     "ratio_batched_over_side_by_side": value / conc}
        log(f"one at a time: {solo:.3e} cu/s, side by side {conc:.3e} cu/s; batched / one at a time = "
            f"{value / solo:.2f}, batched / side by side = {value / conc:.2f}")
    else:
        batch.close()
        eps, gain = extra
        if not args.no_legs:
            extra_out["batched_leg"] = c3_leg(args, I, mbf)
            extra_out["adjoint_leg"] = adjoint_leg(I, mbf)
            extra_out["configs_leg"] = configs_leg(I, mbf)
        if not args.no_cpu_baseline:
            cpu = cpu_baseline(I, args.n, eps, gain, quick=args.quick_cpu)
            log(f"cpu baseline: {cpu['value']:.3e} cu/s on {cpu['cores']} cores")
            # each config's GPU rate over the oracle's on every core
            for c in extra_out.get("configs_leg", []):
                w = [x for x in cpu["windows"] if x["workload"] == c["workload"] and x["cores"] == cpu["cores"]]
                if w:
                    c["oracle_all_cores"] = w[0]["value"]
                    c["gpu_over_oracle"] = c["value"] / w[0]["value"]

    out = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": kdesc,
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_ms": avg_kern_s * 1e3,
            "step_alg_bytes": alg[0],
            "step_kernels_ms": [kern_ms[0] / launches, kern_ms[1] / launches],
            # the whole step (every kernel of a time step, graph-replayed):
            # its algorithmic bytes over the timed milliseconds per step
            "step_achieved": alg[0] / (wall_ms / args.steps / 1e3) / 1e9,
            "step_frac": alg[0] / (wall_ms / args.steps / 1e3) / 1e9 / HBM_PEAK_GBS,
            # cell-updates/s priced at the dense 157 B per cell-update (every
            # cell with three gain sites), over the same peak
            "effective_frac_157B": value * DENSE_BYTES_PER_CU / (HBM_PEAK_GBS * 1e9),
            "measured_copy_GBs": copy_gbs,
        },
        "cpu_baseline": cpu,
    }
    out.update(extra_out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
