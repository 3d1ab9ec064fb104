"""Seeded synthetic inputs shaped like the paper's MD scenarios.

This module only builds particle positions, velocities and box sizes.  It holds
none of the force or integration arithmetic, so both the GPU path and the FP64
CPU oracle can take their inputs from it without sharing any of the method.

Every system is a cubic or orthorhombic periodic box in reduced Lennard-Jones
units (epsilon = sigma = m = 1), as the paper uses for its scenarios (Sec. 4.2
and the appendix table of aluminium parameters).  Generators:

* ``fcc``      -- face-centred-cubic lattice of n^3 unit cells (4 sites each) at a
                  given number density, with i.i.d. uniform jitter per component;
* ``fcc_subset`` -- the smallest FCC lattice with at least N sites, scaled to a
                  box of volume N/rho, keeping a seeded subset of N sites;
* ``slab``     -- a liquid slab (one third of the box along z) plus vapour, in a
                  1:1:3 box;
* ``replicas`` -- many independent FCC-jittered systems of uneven size;
* ``maxwell_boltzmann`` -- Gaussian velocities, zero net momentum, rescaled to
                  an exact kinetic temperature with 3N-3 degrees of freedom.

Seeds follow one rule: workload number w draws from PCG64(1000 + w); replica r
of the batched workload draws its own lattice and velocities from PCG64(5000 + r).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

FCC_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]], dtype=np.float64
)

# Interaction parameters shared by every workload (reduced units).
EPSILON = 1.0
SIGMA = 1.0
MASS = 1.0
RC_PAIR = 2.5
RC_TRIPLET = 2.5
NU = 0.073
DT = 0.001


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _wrap_into_box(x: np.ndarray, box: np.ndarray) -> np.ndarray:
    # Input preparation only: bring jittered sites back into [0, L).
    return np.mod(x, box[None, :])


def fcc_sites(n: tuple, spacing: np.ndarray) -> np.ndarray:
    """All 4*nx*ny*nz FCC sites, cell-major order (z slowest, then y, x), basis fastest."""
    nx, ny, nz = n
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    sites = (cells[:, None, :] + FCC_BASIS[None, :, :]).reshape(-1, 3)
    return sites * spacing[None, :]


def fcc(n_cells: int, density: float, jitter: float, rng: Optional[np.random.Generator]):
    """Cubic FCC crystal of n_cells^3 unit cells; returns (x [N,3], box [3])."""
    a = (4.0 / density) ** (1.0 / 3.0)
    box = np.full(3, n_cells * a)
    x = fcc_sites((n_cells, n_cells, n_cells), np.full(3, a))
    if jitter > 0.0:
        x = x + rng.uniform(-jitter, jitter, size=x.shape)
    return _wrap_into_box(x, box), box


def fcc_subset(n_particles: int, density: float, jitter: float, rng: np.random.Generator):
    """N sites drawn without replacement from the smallest FCC lattice holding N."""
    n = int(math.ceil((n_particles / 4.0) ** (1.0 / 3.0) - 1e-12))
    while 4 * n ** 3 < n_particles:
        n += 1
    length = (n_particles / density) ** (1.0 / 3.0)
    box = np.full(3, length)
    sites = fcc_sites((n, n, n), np.full(3, length / n))
    keep = np.sort(rng.choice(sites.shape[0], size=n_particles, replace=False))
    x = sites[keep]
    if jitter > 0.0:
        x = x + rng.uniform(-jitter, jitter, size=x.shape)
    return _wrap_into_box(x, box), box


def maxwell_boltzmann(n_particles: int, temperature: float, rng: np.random.Generator,
                      mass: float = MASS) -> np.ndarray:
    v = rng.normal(0.0, math.sqrt(temperature / mass), size=(n_particles, 3))
    v -= v.mean(axis=0, keepdims=True)
    dof = 3 * n_particles - 3
    if dof > 0:
        t_now = mass * float(np.sum(v * v)) / dof
        if t_now > 0.0:
            v *= math.sqrt(temperature / t_now)
    return v


def slab(n_particles: int, rho_liquid: float, rho_vapour: float, rng: np.random.Generator,
         jitter: float = 0.05, min_sep: float = 1.0):
    """Liquid slab filling z in [Lz/3, 2Lz/3) of an Lx:Lx:3Lx box, vapour elsewhere.

    Lx solves N = Lx^3 * (rho_liquid + 2 * rho_vapour).  The liquid is a seeded subset
    of a jittered FCC lattice stretched over the slab; vapour particles are uniform
    in the rest of the box, rejected when closer than ``min_sep`` to any particle.
    """
    from scipy.spatial import cKDTree

    lx = (n_particles / (rho_liquid + 2.0 * rho_vapour)) ** (1.0 / 3.0)
    box = np.array([lx, lx, 3.0 * lx])
    n_liq = int(round(rho_liquid * lx ** 3))
    n_liq = min(n_liq, n_particles)
    n = int(math.ceil((n_liq / 4.0) ** (1.0 / 3.0) - 1e-12))
    while 4 * n ** 3 < n_liq:
        n += 1
    sites = fcc_sites((n, n, n), np.full(3, lx / n))
    keep = np.sort(rng.choice(sites.shape[0], size=n_liq, replace=False))
    liq = sites[keep] + rng.uniform(-jitter, jitter, size=(n_liq, 3))
    liq[:, 2] += lx + 0.25 * lx / n  # slab occupies [Lz/3, 2Lz/3); no site on its faces
    liq = _wrap_into_box(liq, box)

    n_vap = n_particles - n_liq
    placed = [liq]
    tree = cKDTree(liq, boxsize=box)
    vap: List[np.ndarray] = []
    got = 0
    while got < n_vap:
        m = max(1024, 2 * (n_vap - got))
        cand = rng.uniform(0.0, 1.0, size=(m, 3)) * np.array([lx, lx, 2.0 * lx])
        cand[:, 2] = np.where(cand[:, 2] < lx, cand[:, 2], cand[:, 2] + lx)  # skip the slab
        dist, _ = tree.query(cand, k=1)
        cand = cand[dist >= min_sep]
        accepted = []
        for p in cand:
            if got + len(accepted) >= n_vap:
                break
            if accepted:
                d = np.abs(np.asarray(accepted) - p)
                d = np.minimum(d, box - d)
                if np.min(np.sum(d * d, axis=1)) < min_sep * min_sep:
                    continue
            accepted.append(p)
        if accepted:
            acc = np.asarray(accepted)
            vap.append(acc)
            got += acc.shape[0]
            placed.append(acc)
            tree = cKDTree(np.concatenate(placed), boxsize=box)
    x = np.concatenate([liq] + vap) if vap else liq
    return x, box


@dataclasses.dataclass
class Workload:
    """One seeded input: concatenated systems, per-system boxes and sizes."""

    name: str
    x: np.ndarray            # [N_total, 3] float64, systems concatenated
    v: np.ndarray            # [N_total, 3] float64
    box: np.ndarray          # [n_systems, 3] float64
    n_particles: np.ndarray  # [n_systems] int64
    temperature: np.ndarray  # [n_systems]
    epsilon: float = EPSILON
    sigma: float = SIGMA
    mass: float = MASS
    rc_pair: float = RC_PAIR
    rc_triplet: float = RC_TRIPLET
    nu: float = NU
    dt: float = DT
    k: int = 1
    n_iter: int = 100
    precision: str = "fp64"
    method: str = "cutoff"   # "direct": DirectSum, no cutoff, open boundaries
    k_outer: int = 1         # > 1: nested r-RESPA over two triplet distance classes
    rc_triplet_inner: float = 0.0

    @property
    def n_systems(self) -> int:
        return int(self.n_particles.shape[0])

    @property
    def n_total(self) -> int:
        return int(self.x.shape[0])


def _single(name, x, box, temperature, rng, **kw) -> Workload:
    v = maxwell_boltzmann(x.shape[0], temperature, rng)
    return Workload(name=name, x=np.ascontiguousarray(x), v=np.ascontiguousarray(v),
                    box=box[None, :].copy(), n_particles=np.array([x.shape[0]], dtype=np.int64),
                    temperature=np.array([temperature]), **kw)


def fcc_workload(name: str, n_cells: int, seed: int, density: float = 0.8,
                 temperature: float = 0.7, jitter: float = 0.05, **kw) -> Workload:
    rng = rng_for(seed)
    x, box = fcc(n_cells, density, jitter, rng)
    return _single(name, x, box, temperature, rng, **kw)


def plain_fp64() -> Workload:
    """500 particles (5^3 FCC cells) at rho 0.8, jitter 0.05, T 0.7; VV as r-RESPA k=1, 100 steps."""
    return fcc_workload("fcc500_fp64_k1", 5, 1001, k=1, n_iter=100)


def fp64_at_scale() -> Workload:
    """32,000 particles (20^3 FCC cells), T 0.7, r-RESPA k=10, 1,000 inner steps."""
    return fcc_workload("fcc32k_fp64_k10", 20, 1002, k=10, n_iter=1000)


def nested_at_scale() -> Workload:
    """The 32,000-particle system under nested r-RESPA: triplets with all edges <= 2.0
    every 2 steps, the rest of the 2.5 cutoff set every 10 (the same full step as k=10)."""
    w = fcc_workload("fcc32k_nested_k2x5", 20, 1002, k=2, n_iter=1000)
    w.k_outer = 5
    w.rc_triplet_inner = 2.0
    return w


def precision_form(k: int = 10, precision: str = "fp64") -> Workload:
    """1,048,576 particles (64^3 FCC cells), r-RESPA k in {1,5,10,20}: the FP64 path and
    the FP32 form compared on it."""
    return fcc_workload("fcc1m_k%d" % k, 64, 1003, k=k, n_iter=1000, precision=precision)


def fcc4000(seed: int = 1003) -> Workload:
    """Standalone 4,000-particle system (10^3 FCC cells) used for full-oracle energy checks."""
    return fcc_workload("fcc4000", 10, seed)


def inhomogeneous(rc_triplet: float = 2.5, n_particles: int = 500_000) -> Workload:
    """Liquid slab (rho 0.75) plus vapour (rho 0.02) in a 1:1:3 box, T 0.85, FP32, k=10."""
    rng = rng_for(1004)
    x, box = slab(n_particles, 0.75, 0.02, rng)
    return _single("slab%dk_rc3_%.1f" % (n_particles // 1000, rc_triplet), x, box, 0.85, rng,
                   rc_triplet=rc_triplet, k=10, n_iter=1000, precision="fp32")


def batched(n_replicas: int = 256, n_min: int = 200, n_max: int = 20_000) -> Workload:
    """Replicas with N log-uniform in [n_min, n_max], rho U[0.6,0.9], T U[0.6,1.2]."""
    rng = rng_for(1005)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_replicas)))
    sizes = sizes.astype(np.int64)
    dens = rng.uniform(0.6, 0.9, size=n_replicas)
    temps = rng.uniform(0.6, 1.2, size=n_replicas)
    xs, vs, boxes = [], [], []
    for r in range(n_replicas):
        rr = rng_for(5000 + r)
        x, box = fcc_subset(int(sizes[r]), float(dens[r]), 0.05, rr)
        xs.append(x)
        vs.append(maxwell_boltzmann(x.shape[0], float(temps[r]), rr))
        boxes.append(box)
    return Workload(name="replicas%d" % n_replicas, x=np.concatenate(xs), v=np.concatenate(vs),
                    box=np.stack(boxes), n_particles=sizes, temperature=temps, k=10,
                    n_iter=1000, precision="fp32")


def open_cluster(n_particles: int, length: float, jitter: float, rng: np.random.Generator):
    """N sites drawn without replacement from the smallest FCC lattice holding N that fills
    a cube of edge `length`, jittered and not wrapped (open boundaries); returns (x, box)."""
    n = int(math.ceil((n_particles / 4.0) ** (1.0 / 3.0) - 1e-12))
    while 4 * n ** 3 < n_particles:
        n += 1
    sites = fcc_sites((n, n, n), np.full(3, length / n))
    keep = np.sort(rng.choice(sites.shape[0], size=n_particles, replace=False))
    x = sites[keep] + rng.uniform(-jitter, jitter, size=(n_particles, 3))
    return x, np.full(3, length)


def toy(nu: float = 0.073, n_particles: int = 675, length: float = 10.0, temperature: float = 0.7,
        seed: int = 1006) -> Workload:
    """Toy scenario of the RVITE study (Sec. 4.2.1): 675 particles in a 10^3 domain,
    eps = sigma = 1, dt = 0.001, nu varied; DirectSum (open boundaries).  Initial state
    (the paper gives none): a jittered FCC subset filling the domain, T 0.7."""
    rng = rng_for(seed)
    x, box = open_cluster(n_particles, length, 0.05, rng)
    return _single("toy%d_nu%.3g" % (n_particles, nu), x, box, temperature, rng, nu=nu, k=1,
                   n_iter=1200, method="direct")


def aluminium(seed: int = 1007) -> Workload:
    """Aluminium scenario (appendix table): 4,995 particles in a 20^3 domain, nu 0.3095,
    dt 0.00304, T 1.1 (reduced units); DirectSum (open boundaries).  Initial state: a
    jittered FCC subset filling the domain."""
    rng = rng_for(seed)
    n, length = 4995, 20.0
    x, box = open_cluster(n, length, 0.05, rng)
    return _single("al4995", x, box, 1.1, rng, nu=0.3095, dt=0.00304, k=12, n_iter=24000,
                   method="direct")


def aluminium_periodic(seed: int = 1008) -> Workload:
    """The aluminium parameters (appendix table) on the cutoff path: 4,995 particles in a
    periodic 20^3 box, cutoffs 2.5 sigma for pairs and triplets.  Initial state: a jittered
    FCC subset of the box."""
    rng = rng_for(seed)
    n, length = 4995, 20.0
    x, box = fcc_subset(n, n / length ** 3, 0.05, rng)
    return _single("al4995_pbc", x, box, 1.1, rng, nu=0.3095, dt=0.00304, k=1, n_iter=24000)


def perfect_fcc(n_cells: int, density: float = 0.8):
    """Unjittered lattice (x, box): every force vanishes by inversion symmetry."""
    return fcc(n_cells, density, 0.0, None)
