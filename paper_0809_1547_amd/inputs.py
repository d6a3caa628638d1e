"""Seeded synthetic inputs shared by the GPU library's tests and the CPU oracle.

This module holds no Maxwell-Bloch arithmetic.  It only produces the data the
simulations start from:

* sphere packings standing in for the paper's granular sample of TiO2 spheres
  (Simulations section: mean diameter 300 nm, refractive index 2.9, gain only in
  the voids between spheres);
* the per-cell permittivity map and gain mask obtained by voxelising a packing;
* probe sites for the spectral monitor, random initial fields, and the named
  workload presets (grid, step count, pump density).

The paper obtains its packing by molecular dynamics; random sequential addition
(RSA) with Gaussian diameters stands in for it by default, and ``pack_start``
gives the seeded start (diameters and random centres) of the soft-sphere
compression packing that the library computes.  Every generator is keyed
by an explicit integer seed (numpy PCG64), so a given call returns the same
arrays on every machine.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Physical constants of the workloads (SI), as printed in the Simulations section.
DX = 20e-9                 # Yee cell size [m]
COURANT = 0.99             # dt = COURANT * dx / (c * sqrt(3))
N_SPHERE = 2.9             # refractive index of the spheres
EPS_SPHERE = N_SPHERE ** 2 # 8.41
EPS_BACKGROUND = 1.0       # background (the paper does not state it; vacuum here)
MEAN_DIAMETER = 300e-9
SD_DIAMETER = 30e-9
LAMBDA0 = 590e-9           # gain centre wavelength
DLAMBDA = 230e-9           # gain bandwidth
NA_LOW, NA_HIGH = 2e24, 5e24   # pump densities shown for the lasing spectra [m^-3]


def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed) & 0xFFFFFFFF, int(seed) >> 32, int(stream)]))


@dataclasses.dataclass
class Packing:
    """Spheres in cell units: centres (K,3) as (x, y, z), radii (K,)."""
    n: Tuple[int, int, int]
    centres: np.ndarray
    radii: np.ndarray

    @property
    def count(self) -> int:
        return int(self.radii.shape[0])

    def nominal_fill(self) -> float:
        vol = float(np.prod(self.n))
        return float(np.sum(4.0 / 3.0 * math.pi * self.radii ** 3)) / vol


def rsa_pack(n: Tuple[int, int, int] | int, *, seed: int,
             fill: Optional[float] = None, count: Optional[int] = None,
             radius: Optional[float] = None,
             mean_d: float = 300.0 / 20.0, sd_d: float = 30.0 / 20.0,
             max_attempts: int = 5_000_000) -> Packing:
    """Random sequential addition of non-overlapping spheres (cell units).

    Centres are uniform over the whole box and spheres may be cut by the walls.
    Diameters are Gaussian (mean_d, sd_d) truncated to +-3 sd by redrawing, or
    all equal to 2*radius when ``radius`` is given.  Each sphere's diameter is
    drawn once, before its first placement attempt, and kept until a centre
    for it is found: redrawing the diameter on every rejected attempt would
    favour small spheres (large ones are rejected more often) and bias the
    accepted diameters low.  Insertion stops once ``count`` spheres are
    placed, or once the summed full-sphere volume reaches ``fill`` times the
    box volume.

    Candidate centres are drawn uniformly from the unit voxels not yet known to
    be fully excluded for the sphere being placed, then tested exactly; the
    accepted spheres therefore follow the same distribution as plain RSA
    (uniform centre over the box, rejection on overlap), only with far fewer
    wasted draws near jamming.  Exclusion is tracked for a few radius classes
    (class radii from the smallest possible radius upwards); a sphere draws
    from the map of the largest class radius not above its own, which never
    excludes a position the sphere could take.
    """
    if isinstance(n, int):
        n = (n, n, n)
    n = tuple(int(v) for v in n)
    if (fill is None) == (count is None):
        raise ValueError("give exactly one of fill= or count=")
    rng = _rng(seed, 1)
    nx, ny, nz = n
    box = np.array(n, dtype=np.float64)
    target_vol = None if fill is None else fill * float(np.prod(box))
    if radius is not None:
        rmin = rmax = float(radius)
    else:
        rmin, rmax = 0.5 * (mean_d - 3 * sd_d), 0.5 * (mean_d + 3 * sd_d)
    n_cls = 1 if rmax == rmin else 8
    cls_r = [rmin + (rmax - rmin) * q / n_cls for q in range(n_cls)]
    cell = 2.0 * rmax
    grid_shape = tuple(max(1, int(math.ceil(b / cell))) for b in n)
    buckets: Dict[Tuple[int, int, int], List[int]] = {}
    centres: List[np.ndarray] = []
    radii: List[float] = []
    excluded = np.zeros((n_cls, nz, ny, nx), dtype=bool)
    half_diag = 0.5 * math.sqrt(3.0)
    vol = 0.0
    attempts = 0
    r = None                                   # radius of the sphere being placed
    q = 0                                      # its radius class
    free = [None] * n_cls
    cursor = [0] * n_cls
    batch = 4096

    def draw_radius() -> float:
        if radius is not None:
            return float(radius)
        while True:
            d = rng.normal(mean_d, sd_d)
            if abs(d - mean_d) <= 3 * sd_d:
                return 0.5 * d

    while True:
        if count is not None and len(radii) >= count:
            break
        if target_vol is not None and vol >= target_vol:
            break
        if attempts >= max_attempts:
            raise RuntimeError(f"RSA jammed after {attempts} attempts with {len(radii)} spheres")
        if r is None:
            r = draw_radius()
            q = 0 if n_cls == 1 else min(n_cls - 1, int((r - rmin) / (rmax - rmin) * n_cls))
        exq = excluded[q]
        if free[q] is None or cursor[q] >= len(free[q]):
            idx = np.flatnonzero(~exq.ravel())
            if idx.size == 0:
                raise RuntimeError(f"RSA jammed: no free voxel left with {len(radii)} spheres")
            free[q] = idx[rng.integers(0, idx.size, size=batch)]
            cursor[q] = 0
        v = int(free[q][cursor[q]])
        cursor[q] += 1
        attempts += 1
        if exq.flat[v]:
            continue
        vk, rem = divmod(v, nx * ny)
        vj, vi = divmod(rem, nx)
        c = np.array([vi, vj, vk], dtype=np.float64) + rng.random(3)
        g = tuple(min(int(c[a] // cell), grid_shape[a] - 1) for a in range(3))
        ok = True
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    for idx_s in buckets.get((g[0] + dx, g[1] + dy, g[2] + dz), ()):
                        if np.sum((centres[idx_s] - c) ** 2) < (radii[idx_s] + r) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        buckets.setdefault(g, []).append(len(radii))
        centres.append(c)
        radii.append(r)
        vol += 4.0 / 3.0 * math.pi * r ** 3
        # voxels whose every point lies closer than r + (class radius) to this
        # centre can never hold the centre of a sphere of that class
        for qq in range(n_cls):
            reach = r + cls_r[qq] - half_diag
            if reach <= 0:
                continue
            lo = [max(0, int(math.floor(c[a] - reach - 1))) for a in range(3)]
            hi = [min(n[a], int(math.ceil(c[a] + reach + 1))) for a in range(3)]
            xs = np.arange(lo[0], hi[0]) + 0.5 - c[0]
            ys = np.arange(lo[1], hi[1]) + 0.5 - c[1]
            zs = np.arange(lo[2], hi[2]) + 0.5 - c[2]
            d2 = zs[:, None, None] ** 2 + ys[None, :, None] ** 2 + xs[None, None, :] ** 2
            excluded[qq, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] |= d2 < reach * reach
        r = None
    return Packing(n, np.array(centres, dtype=np.float64).reshape(-1, 3),
                   np.array(radii, dtype=np.float64))


def pack_start(n: Tuple[int, int, int] | int, *, seed: int, fill: float,
               mean_d: float = 300.0 / 20.0, sd_d: float = 30.0 / 20.0):
    """Seeded start of a compression packing (cell units).

    Diameters are drawn as in ``rsa_pack`` (Gaussian, truncated to +-3 sd by
    redrawing) until their summed full-sphere volume reaches ``fill`` times the
    box volume; centres are uniform over the box and may overlap.  Returns
    (box (3,), diameters (K,), centres (K, 3) as (x, y, z)).
    """
    if isinstance(n, int):
        n = (n, n, n)
    box = np.array([float(v) for v in n])
    rng = _rng(seed, 2)
    target = fill * float(np.prod(box))
    diam: List[float] = []
    vol = 0.0
    while vol < target:
        d = rng.normal(mean_d, sd_d)
        if abs(d - mean_d) <= 3 * sd_d:
            diam.append(float(d))
            vol += math.pi / 6.0 * d ** 3
    d = np.array(diam, dtype=np.float64)
    centres = rng.random((d.shape[0], 3)) * box
    return box, d, centres


def packing_from_centres(n: Tuple[int, int, int] | int, diam: np.ndarray, centres: np.ndarray) -> Packing:
    """A Packing (for ``voxelize``) from diameters and centres."""
    if isinstance(n, int):
        n = (n, n, n)
    return Packing(tuple(int(v) for v in n), np.asarray(centres, dtype=np.float64).reshape(-1, 3),
                   0.5 * np.asarray(diam, dtype=np.float64).reshape(-1))


def voxelize(p: Packing, eps_sphere: float = EPS_SPHERE,
             eps_background: float = EPS_BACKGROUND) -> Tuple[np.ndarray, np.ndarray]:
    """Per-cell relative permittivity (float32) and gain mask (uint8).

    Arrays have shape (nz, ny, nx) with x fastest.  A cell belongs to a sphere
    when its centre lies inside it; sphere cells carry eps_sphere and no gain,
    all other cells carry eps_background and gain (the voids are infiltrated
    with the active medium).
    """
    nx, ny, nz = p.n
    inside = np.zeros((nz, ny, nx), dtype=bool)
    for c, r in zip(p.centres, p.radii):
        lo = [max(0, int(math.floor(c[a] - r - 0.5))) for a in range(3)]
        hi = [min(p.n[a], int(math.ceil(c[a] + r + 0.5)) + 1) for a in range(3)]
        if any(hi[a] <= lo[a] for a in range(3)):
            continue
        xs = np.arange(lo[0], hi[0]) + 0.5 - c[0]
        ys = np.arange(lo[1], hi[1]) + 0.5 - c[1]
        zs = np.arange(lo[2], hi[2]) + 0.5 - c[2]
        d2 = zs[:, None, None] ** 2 + ys[None, :, None] ** 2 + xs[None, None, :] ** 2
        inside[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] |= d2 < r * r
    eps = np.where(inside, np.float32(eps_sphere), np.float32(eps_background)).astype(np.float32)
    gain = (~inside).astype(np.uint8)
    return eps, gain


def homogeneous(n: Tuple[int, int, int] | int, eps: float = 1.0, gain: int = 1):
    if isinstance(n, int):
        n = (n, n, n)
    nx, ny, nz = n
    return (np.full((nz, ny, nx), eps, dtype=np.float32),
            np.full((nz, ny, nx), gain, dtype=np.uint8))


# Yee-site bookkeeping shared by tests: E-site (c, i, j, k) of component c lives
# on the edge of cell (i, j, k); interior sites are those not on a wall.
def interior_e_mask(n: Tuple[int, int, int], comp: int) -> np.ndarray:
    """Boolean (nz+1, ny+1, nx+1) mask of E-sites of component ``comp`` that are
    updated by the curl equation (not on a wall, inside the stored range)."""
    nx, ny, nz = n
    m = np.zeros((nz + 1, ny + 1, nx + 1), dtype=bool)
    lo = [1, 1, 1]
    lo[comp] = 0
    m[lo[2]:nz, lo[1]:ny, lo[0]:nx] = True
    return m


def select_probes(eps: np.ndarray, gain: np.ndarray, n_probes: int, *, seed: int,
                  comp: int = 2) -> np.ndarray:
    """Pick ``n_probes`` distinct interior E-sites of component ``comp`` lying in
    void (gain) cells.  Returns int32 rows (comp, i, j, k)."""
    nz, ny, nx = gain.shape
    mask = interior_e_mask((nx, ny, nz), comp)[:nz, :ny, :nx] & (gain > 0)
    ks, js, is_ = np.nonzero(mask)
    if len(ks) < n_probes:
        raise ValueError("not enough void sites for the requested probes")
    rng = _rng(seed, 2)
    pick = rng.choice(len(ks), size=n_probes, replace=False)
    pick.sort()
    out = np.empty((n_probes, 4), dtype=np.int32)
    out[:, 0] = comp
    out[:, 1] = is_[pick]
    out[:, 2] = js[pick]
    out[:, 3] = ks[pick]
    return out


def nearest_void_site(gain: np.ndarray, comp: int = 2) -> Tuple[int, int, int, int]:
    """Interior E-site of component ``comp`` in a void cell closest to the box centre."""
    nz, ny, nx = gain.shape
    mask = interior_e_mask((nx, ny, nz), comp)[:nz, :ny, :nx] & (gain > 0)
    ks, js, is_ = np.nonzero(mask)
    c = np.array([nx / 2.0, ny / 2.0, nz / 2.0])
    d2 = (is_ + 0.5 - c[0]) ** 2 + (js + 0.5 - c[1]) ** 2 + (ks + 0.5 - c[2]) ** 2
    t = int(np.argmin(d2))
    return comp, int(is_[t]), int(js[t]), int(ks[t])


def random_fields(n: Tuple[int, int, int], *, seed: int, amplitude: float = 1.0,
                  comps=(0, 1, 2)) -> Dict[int, np.ndarray]:
    """Random E-field components on interior sites, zero elsewhere.  Values are
    float32 (exactly representable in both precisions)."""
    rng = _rng(seed, 3)
    out = {}
    for c in comps:
        a = rng.standard_normal((n[2] + 1, n[1] + 1, n[0] + 1)).astype(np.float32)
        a *= np.float32(amplitude)
        a[~interior_e_mask(n, c)] = 0.0
        out[c] = a
    return out


def dft_omegas(lam_min: float, lam_max: float, n_steps: int, dt: float) -> np.ndarray:
    """Angular frequencies uniform in frequency between two wavelengths at the
    run's natural resolution 1/(n_steps*dt)."""
    c = 299792458.0
    f_lo, f_hi = c / lam_max, c / lam_min
    df = 1.0 / (n_steps * dt)
    k0 = int(math.ceil(f_lo / df))
    k1 = int(math.floor(f_hi / df))
    return 2.0 * math.pi * df * np.arange(k0, k1 + 1, dtype=np.float64)


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    steps: int
    boundary: str          # "pec" or "mur"
    init: str              # "prepumped" or "ground"
    Na: float
    seed: int = 0
    realization: int = 0

    def cells(self) -> int:
        return self.n ** 3


def packing_for(name: str, n: int, seed: int) -> Packing:
    """The synthetic packing of a named workload (see the workload table)."""
    if name == "c1":
        return rsa_pack(n, seed=seed, count=8, radius=150.0 / 20.0)
    return rsa_pack(n, seed=seed, fill=0.4)


WORKLOADS = {
    # 32^3 x 500, 8 spheres r = 150 nm, PEC, pre-pumped, N_a = 2e24
    "c1": Workload("c1", 32, 500, "pec", "prepumped", NA_LOW),
    # 128^3 x 5000, fill 0.4, Mur, pre-pumped lasing run
    "c2": Workload("c2", 128, 5000, "mur", "prepumped", NA_LOW),
    # 96^3 x 1000 adjoint workload, PEC
    "c4": Workload("c4", 96, 1000, "pec", "prepumped", NA_LOW),
    # 320^3 paper-scale realization, Mur, ground start, 3 ps
    "c5": Workload("c5", 320, 78675, "mur", "ground", NA_LOW),
}


def batch_sizes(count: int = 64, seed: int = 0) -> List[int]:
    """Grid sizes of the batched workload: uniform over {48, 64, 80, 96}, one
    host draw per realization keyed by (seed, r)."""
    out = []
    for r in range(count):
        g = np.random.Generator(np.random.PCG64([seed, r, 4]))
        out.append(int(g.choice([48, 64, 80, 96])))
    return out


def batch_pump_levels(count: int, n_th) -> List[float]:
    """Pump densities of the batched workload: level p = r mod 8 at
    0.5 * 8**(p/7) times threshold (8 log-spaced levels, 0.5x to 4x).
    n_th is one threshold for every realization or one per realization."""
    th = np.broadcast_to(np.asarray(n_th, dtype=np.float64), (count,))
    return [0.5 * 8.0 ** ((r % 8) / 7.0) * float(th[r]) for r in range(count)]


def synthetic_spectra(n_probes: int, n_freq: int, *, seed: int,
                      lines: Sequence[Tuple[float, float, float]] = ((0.45, 0.03, 1.0),),
                      noise: float = 0.02, lam_min: float = 450e-9,
                      lam_max: float = 800e-9) -> Tuple[np.ndarray, np.ndarray]:
    """Complex probe amplitudes F (n_probes, n_freq) on a uniform omega grid
    between two wavelengths, shaped like running-DFT emission spectra: every
    probe is a sum of lines (centre and width as fractions of the band,
    amplitude) with Gaussian |F| profiles at random phases, plus complex
    Gaussian noise of the given amplitude.  Returns (F, omega)."""
    c = 299792458.0
    w_lo, w_hi = 2.0 * math.pi * c / lam_max, 2.0 * math.pi * c / lam_min
    omega = np.linspace(w_lo, w_hi, n_freq) if n_freq > 1 else np.array([0.5 * (w_lo + w_hi)])
    g = _rng(seed, 7)
    x = (omega - w_lo) / (w_hi - w_lo)
    F = np.zeros((n_probes, n_freq), dtype=np.complex128)
    for p in range(n_probes):
        for (x0, wid, amp) in lines:
            phase = g.uniform(0.0, 2.0 * math.pi)
            scale = g.uniform(0.5, 1.5)
            F[p] += amp * scale * np.exp(-0.5 * ((x - x0) / wid) ** 2) * np.exp(1j * phase)
        F[p] += noise * (g.standard_normal(n_freq) + 1j * g.standard_normal(n_freq))
    return F, omega
