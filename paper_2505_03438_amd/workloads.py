"""Seeded synthetic inputs for the Lennard-Jones workloads.

This module only places particles and draws velocities.  It holds none of the
method's arithmetic (no pair potential, no forces, no cells) and imports
nothing else from this package, so that the FP64 oracle and the HIP path are
fed the very same arrays without sharing any code.

Positions are SoA ``[3, n]`` float64 in ``[0, L)``; velocities ``[3, n]``
float64; types int32.

Initial placement.  Uniformly random positions at liquid density overlap (a
third of the particles have a neighbour closer than 0.5 sigma), which a
force-based relaxation would have to undo; relaxing with any force code
would put method arithmetic into the inputs.  Instead every homogeneous
workload starts from an FCC lattice at the target density with each site
displaced uniformly within +-jitter per axis, in a random particle order
(ids carry no spatial information).  The minimum pair distance is then
bounded below by construction; at T >= 0.7 the lattice melts within the
first few hundred steps.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 2505034380


def seed_for(config_index: int) -> int:
    return BASE_SEED + config_index


def _wrap(x: np.ndarray, L: float) -> np.ndarray:
    x = np.mod(x, L)
    return np.where(x >= L, 0.0, x)


def fcc_sites(ncx: int, ncy: int, ncz: int, a: float) -> np.ndarray:
    """All sites of an FCC lattice of ncx*ncy*ncz cubic unit cells, [3, 4 n]."""
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    ix, iy, iz = np.meshgrid(np.arange(ncx), np.arange(ncy), np.arange(ncz), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    return np.ascontiguousarray(sites.T)


def fcc_lattice(ncell: int, density: float):
    """Perfect FCC lattice, ncell^3 unit cells at the given number density.
    Returns (pos [3, 4 ncell^3], box [3])."""
    a = (4.0 / density) ** (1.0 / 3.0)
    L = ncell * a
    pos = fcc_sites(ncell, ncell, ncell, a)
    box = np.array([L, L, L])
    return np.ascontiguousarray(_wrap(pos, L)), box


def maxwell_boltzmann(n: int, T: float, rng: np.random.Generator, mass=None) -> np.ndarray:
    """Velocities drawn per component from N(0, sqrt(T/m)), net momentum
    removed, then rescaled so that 2K/(3n-3) equals T exactly (k_B = 1)."""
    m = np.ones(n) if mass is None else np.asarray(mass, dtype=np.float64)
    v = rng.standard_normal((3, n)) * np.sqrt(T / m)[None, :]
    p = (v * m[None, :]).sum(axis=1) / m.sum()
    v -= p[:, None]
    K = 0.5 * float((m[None, :] * v * v).sum())
    dof = 3 * n - 3
    if K > 0.0 and dof > 0:
        v *= math.sqrt(T * dof / (2.0 * K))
    return np.ascontiguousarray(v)


def jittered_fcc(ncell, density: float, jitter: float, rng: np.random.Generator,
                 shuffle: bool = True):
    """FCC lattice (ncell or (nx, ny, nz) unit cells) at `density`, each site
    displaced uniformly in [-jitter, jitter] per axis (jitter in units of the
    lattice constant), particle order randomly permuted."""
    if np.isscalar(ncell):
        ncell = (int(ncell),) * 3
    a = (4.0 / density) ** (1.0 / 3.0)
    box = np.array([ncell[0] * a, ncell[1] * a, ncell[2] * a])
    pos = fcc_sites(ncell[0], ncell[1], ncell[2], a)
    pos = pos + rng.uniform(-jitter * a, jitter * a, size=pos.shape)
    if shuffle:
        pos = pos[:, rng.permutation(pos.shape[1])]
    for d in range(3):
        pos[d] = _wrap(pos[d], box[d])
    return np.ascontiguousarray(pos), box


# --------------------------------------------------------------------------
# The named workloads.


def plain_fcc_864(seed: int | None = None):
    """864 particles on a 6x6x6 FCC lattice at density 0.8442, velocities
    Maxwell-Boltzmann at T = 0.722 with zero net momentum."""
    rng = np.random.default_rng(seed_for(0) if seed is None else seed)
    pos, box = fcc_lattice(6, 0.8442)
    vel = maxwell_boltzmann(pos.shape[1], 0.722, rng)
    return dict(pos=pos, vel=vel, box=box, types=np.zeros(pos.shape[1], np.int32),
                eps=[1.0], sig=[1.0], rc=2.5, dt=0.005, steps=100, T=0.722)


def homogeneous_fluid(ncell: int = 64, density: float = 0.8, T: float = 1.0,
                      seed: int | None = None, jitter: float = 0.06):
    """LJ fluid stand-in: jittered FCC with 4 ncell^3 particles (ncell = 64
    gives 1,048,576 particles, L = 109.438 at density 0.8)."""
    rng = np.random.default_rng(seed_for(1) if seed is None else seed)
    pos, box = jittered_fcc(ncell, density, jitter, rng)
    vel = maxwell_boltzmann(pos.shape[1], T, rng)
    return dict(pos=pos, vel=vel, box=box, types=np.zeros(pos.shape[1], np.int32),
                eps=[1.0], sig=[1.0], rc=2.5, skin=0.3, dt=0.005, T=T)


def droplet(n: int = 2_000_000, density: float = 0.8, T: float = 0.7, fill: float = 0.05,
            seed: int | None = None, jitter: float = 0.06):
    """Spherical liquid droplet of n particles at `density`, centred in a
    periodic cubic box of which it fills the fraction `fill` by volume."""
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    a = (4.0 / density) ** (1.0 / 3.0)
    L = (n / density / fill) ** (1.0 / 3.0)
    R = (3.0 * n / (4.0 * math.pi * density)) ** (1.0 / 3.0)
    nc = int(math.ceil(2.0 * R / a)) + 2
    sites = fcc_sites(nc, nc, nc, a)
    sites -= (nc * a / 2.0)
    r2 = (sites * sites).sum(axis=0)
    keep = np.argsort(r2, kind="stable")[:n]
    pos = sites[:, keep] + L / 2.0
    pos = pos + rng.uniform(-jitter * a, jitter * a, size=pos.shape)
    pos = pos[:, rng.permutation(n)]
    box = np.array([L, L, L])
    for d in range(3):
        pos[d] = _wrap(pos[d], L)
    vel = maxwell_boltzmann(n, T, rng)
    return dict(pos=np.ascontiguousarray(pos), vel=vel, box=box, types=np.zeros(n, np.int32),
                eps=[1.0], sig=[1.0], rc=2.5, skin=0.3, dt=0.005, T=T)


def exploding_liquid(n: int = 1_048_576, density: float = 0.8, T: float = 2.0, fill: float = 1.0 / 27.0,
                     seed: int | None = None):
    """A hot liquid sphere (T well above the critical temperature) in a box
    of 27 times its volume: it expands into the vacuum, so the spread of the
    particles over the cells falls as the run goes (the exploding liquid of
    Sec. 6.2, at GPU size)."""
    d = droplet(n=n, density=density, T=T, fill=fill, seed=seed_for(2) + 1 if seed is None else seed)
    return d


def slab(n: int = 2_000_000, rho_l: float = 0.75, rho_v: float = 0.02, T: float = 0.7,
         seed: int | None = None, jitter: float = 0.06):
    """Two-phase slab: liquid (rho_l) of thickness Lz/3 centred along z in a
    box Lx = Ly, Lz = 3 Lx; vapour (rho_v) elsewhere; n particles in total."""
    rng = np.random.default_rng(seed_for(2) + 1000 if seed is None else seed)
    # n = rho_l Lx^3 + rho_v 2 Lx^3
    Lx = (n / (rho_l + 2.0 * rho_v)) ** (1.0 / 3.0)
    Lz = 3.0 * Lx
    a = (4.0 / rho_l) ** (1.0 / 3.0)
    ncx = int(math.floor(Lx / a))
    ax = Lx / ncx
    ncz = int(round(Lx / ax))
    liq = fcc_sites(ncx, ncx, ncz, ax)
    liq[2] += Lx
    n_liq = liq.shape[1]
    n_vap = n - n_liq
    # vapour: a random subset of a grid about twice as fine as the mean
    # spacing, filling the space between the slab's faces (the liquid
    # lattice, fitted to whole cells, may hold slightly fewer particles than
    # rho_l Lx^3, and the vapour takes the rest).  Its layers keep `gap` plus
    # half a layer step from the outermost liquid layers (z = Lx and z = top),
    # so that no vapour particle starts inside the repulsive core of a liquid
    # one.
    top = Lx + (ncz - 0.5) * ax
    gap = 1.0
    hv = Lz - (top - Lx) - 2.0 * gap
    av = 0.5 * (1.0 / rho_v) ** (1.0 / 3.0)
    nvx = int(math.floor(Lx / av))
    avx = Lx / nvx
    nvz = int(math.floor(hv / av))
    avz = hv / nvz
    gx, gy, gz = np.meshgrid(np.arange(nvx), np.arange(nvx), np.arange(nvz), indexing="ij")
    vap = np.stack([(gx.ravel() + 0.5) * avx, (gy.ravel() + 0.5) * avx,
                    top + gap + (gz.ravel() + 0.5) * avz]).astype(np.float64)
    if vap.shape[1] < n_vap:
        raise ValueError("vapour lattice too small")
    vap = vap[:, rng.choice(vap.shape[1], n_vap, replace=False)]
    vap = vap + rng.uniform(-0.2, 0.2, size=vap.shape) * np.array([[avx], [avx], [avz]])
    liq = liq + rng.uniform(-jitter * ax, jitter * ax, size=liq.shape)
    pos = np.concatenate([liq, vap], axis=1)
    pos = pos[:, rng.permutation(n)]
    box = np.array([Lx, Lx, Lz])
    for d in range(3):
        pos[d] = _wrap(pos[d], box[d])
    vel = maxwell_boltzmann(n, T, rng)
    return dict(pos=np.ascontiguousarray(pos), vel=vel, box=box, types=np.zeros(n, np.int32),
                eps=[1.0], sig=[1.0], rc=2.5, skin=0.3, dt=0.005, T=T)


def splitmix64(x: int) -> int:
    """One output of the SplitMix64 generator (Steele, Lea, Flood 2014)."""
    M = (1 << 64) - 1
    x = (x + 0x9E3779B97F4A7C15) & M
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def batched_systems(n_sys: int = 4096, n_min: int = 256, n_max: int = 8192,
                    rho_range=(0.3, 0.9), T_range=(0.7, 1.5), seed: int | None = None,
                    jitter: float = 0.03):
    """Independent periodic LJ systems: counts log-uniform in [n_min, n_max],
    density and temperature uniform in the given ranges.  Each system s is
    generated from its own seed splitmix64(base ^ s).  Returns a list of dicts."""
    base = seed_for(3) if seed is None else seed
    rng = np.random.default_rng(base)
    ns = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_sys))).astype(np.int64)
    rhos = rng.uniform(rho_range[0], rho_range[1], n_sys)
    Ts = rng.uniform(T_range[0], T_range[1], n_sys)
    out = []
    for s in range(n_sys):
        r = np.random.default_rng(splitmix64(base ^ s))
        n = int(ns[s])
        L = (n / rhos[s]) ** (1.0 / 3.0)
        nc = int(math.ceil((n / 4.0) ** (1.0 / 3.0) - 1e-12))
        a = L / nc
        sites = fcc_sites(nc, nc, nc, a)
        sel = r.choice(sites.shape[1], n, replace=False)
        pos = sites[:, sel] + r.uniform(-jitter * a, jitter * a, size=(3, n))
        pos = pos[:, r.permutation(n)]
        for d in range(3):
            pos[d] = _wrap(pos[d], L)
        vel = maxwell_boltzmann(n, float(Ts[s]), r)
        out.append(dict(pos=np.ascontiguousarray(pos), vel=vel, box=np.array([L, L, L]),
                        types=np.zeros(n, np.int32), rho=float(rhos[s]), T=float(Ts[s])))
    return out


def binary_mixture(ncell: int = 32, density: float = 1.2, T: float = 1.0, frac_a: float = 0.8,
                   seed: int | None = None, jitter: float = 0.04):
    """80/20 A/B mixture on a jittered FCC lattice (ncell = 32 gives 131,072
    particles at density 1.2, L = 47.80).  Per-type parameters
    eps = (1.0, 0.5), sig = (1.0, 0.88); the cutoff is 2.5 sig_ab."""
    rng = np.random.default_rng(seed_for(4) if seed is None else seed)
    pos, box = jittered_fcc(ncell, density, jitter, rng)
    n = pos.shape[1]
    n_a = int(round(frac_a * n))
    types = np.ones(n, np.int32)
    types[rng.permutation(n)[:n_a]] = 0
    vel = maxwell_boltzmann(n, T, rng)
    return dict(pos=pos, vel=vel, box=box, types=types, eps=[1.0, 0.5], sig=[1.0, 0.88],
                rc_factor=2.5, T=T)


def perturb_params(theta, rel: float = 0.05, seed: int | None = None):
    """theta * (1 + rel * xi), xi ~ N(0, 1), seeded."""
    rng = np.random.default_rng(seed_for(4) + 7 if seed is None else seed)
    theta = np.asarray(theta, dtype=np.float64)
    return theta * (1.0 + rel * rng.standard_normal(theta.shape))


def random_gas(n: int, L: float, rng: np.random.Generator):
    """n uniformly random positions in a cubic box (small tests only)."""
    pos = rng.uniform(0.0, L, size=(3, n))
    return np.ascontiguousarray(_wrap(pos, L)), np.array([L, L, L])


def thinned_fcc(ncell: int, rho_max: float, field, rng: np.random.Generator, jitter: float = 0.06):
    """Particles following a density field rho(x) <= rho_max without
    overlaps: an FCC lattice at rho_max fills the cubic box (ncell unit cells
    per side), each site is kept with probability rho(site) / rho_max, then
    displaced within +-jitter lattice constants per axis; random order.
    field(sites [3, m], L) -> densities [m]."""
    a = (4.0 / rho_max) ** (1.0 / 3.0)
    L = ncell * a
    sites = fcc_sites(ncell, ncell, ncell, a)
    keep = rng.random(sites.shape[1]) < np.clip(field(sites, L) / rho_max, 0.0, 1.0)
    pos = sites[:, keep]
    pos = pos + rng.uniform(-jitter * a, jitter * a, size=pos.shape)
    pos = pos[:, rng.permutation(pos.shape[1])]
    box = np.array([L, L, L])
    return np.ascontiguousarray(_wrap(pos, L)), box


def _periodic_d2(sites, c, L):
    d = sites - np.asarray(c, dtype=np.float64)[:, None]
    d -= L * np.rint(d / L)
    return (d * d).sum(axis=0)


def selection_scenarios(seed: int | None = None):
    """Generative scenarios for training a configuration-selection model,
    after the families of the paper's Random Forest dataset (uniform
    distributions over a range of particle counts, clusters of Gaussian
    blobs, a dense cuboid in a dilute gas, a sphere in an empty box), made
    overlap-free by thinning a lattice, in boxes large enough to load the
    GPU.  Yields (name, dict(pos, vel, box, skin))."""
    rng = np.random.default_rng(seed_for(5) if seed is None else seed)
    rho_max = 1.0

    def emit(name, pos, box, skin=0.3):
        vel = maxwell_boltzmann(pos.shape[1], 1.0, rng)
        return name, dict(pos=pos, vel=vel, box=box, skin=skin)

    # uniform: densities 0.02 .. 1.0 at three box sizes (and three skins at the middle size)
    for ncell in (16, 32, 56):
        for rho in (0.02, 0.05, 0.1, 0.2, 0.4, 0.6, 0.8, 1.0):
            skins = (0.2, 0.3, 0.4) if ncell == 32 else (0.3,)
            for skin in skins:
                pos, box = thinned_fcc(ncell, rho_max, lambda s, L, r=rho: np.full(s.shape[1], r), rng)
                yield emit("uniform-n%d-rho%.2f-skin%.1f" % (pos.shape[1], rho, skin), pos, box, skin)
    # Gaussian blobs: k blobs of standard deviation L/12 at random centres
    for ncell in (32, 56):
        for k in (10, 40, 160):
            def blobs(s, L, k=k):
                cs = rng.uniform(0.0, L, size=(k, 3))
                w = 2.0 * (L / 12.0) ** 2
                acc = np.zeros(s.shape[1])
                for c in cs:
                    acc += np.exp(-_periodic_d2(s, c, L) / w)
                return np.minimum(rho_max, 0.9 * acc)
            pos, box = thinned_fcc(ncell, rho_max, blobs, rng)
            yield emit("blobs-%d-n%d" % (k, pos.shape[1]), pos, box)
    # dense cuboid (density 0.9) of thickness f L across the box, in a gas at 0.02
    for ncell in (32, 56):
        for f in (0.125, 0.25, 0.5):
            def cuboid(s, L, f=f):
                inside = np.abs(s[0] - 0.5 * L) < 0.5 * f * L
                return np.where(inside, 0.9, 0.02)
            pos, box = thinned_fcc(ncell, rho_max, cuboid, rng)
            yield emit("cuboid-%.3f-n%d" % (f, pos.shape[1]), pos, box)
    # sphere (density 0.85) of radius f L in an empty box
    for ncell in (32, 56):
        for f in (0.15, 0.25, 0.35):
            def sphere(s, L, f=f):
                return np.where(_periodic_d2(s, (0.5 * L,) * 3, L) < (f * L) ** 2, 0.85, 0.0)
            pos, box = thinned_fcc(ncell, rho_max, sphere, rng)
            yield emit("sphere-%.2f-n%d" % (f, pos.shape[1]), pos, box)
