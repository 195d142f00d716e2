"""Seeded synthetic workloads: BCC lattices, vacancies, displacements, velocities.

Units: Angstrom, fs, eV, amu.  The recipes follow the stated benchmark
configurations (BCC a = 3.304 A, mass 180.95 amu, dt = 1 fs, skin 0.3 A).
The paper's own benchmark slabs (801,792 Cu/W/Ta atoms equilibrated with real
EAM potentials, Sec. IV-B and Table "realistic") are not available; these
synthetic boxes stand in for them.

Random draw order for every box: vacancies -> displacements -> velocities,
all from one numpy Generator.  No EAM arithmetic lives here.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

# Shared physical constants, passed as data to both the oracle and the library.
FTM2V = 1.602176634e-19 / 1e-10 / 1.66053906660e-27 * 1e-20  # (eV/A)/amu -> A/fs^2
KBOLTZ = 8.617333262e-5  # eV/K
MASS = 180.95
A_LAT = 3.304
DT = 1.0
SKIN = 0.3


@dataclasses.dataclass
class Box:
    """One periodic cubic system."""

    x: np.ndarray  # (N, 3) float64, wrapped into [0, L)
    v: np.ndarray  # (N, 3) float64, A/fs
    box: np.ndarray  # (3,) float64
    n_cells: int  # lattice cells per edge
    temperature: float
    site_ids: np.ndarray  # (N,) int64 lattice site id of each atom
    types: np.ndarray = None  # (N,) int32 atom types of a multi-species box, else None

    @property
    def n(self) -> int:
        return self.x.shape[0]


def bcc_sites(n: int, a: float = A_LAT) -> np.ndarray:
    """Sites of an n x n x n BCC crystal; site id = ((ix*n + iy)*n + iz)*2 + b."""
    i = np.arange(n, dtype=np.float64)
    ix, iy, iz = np.meshgrid(i, i, i, indexing="ij")
    base = np.stack([ix, iy, iz], axis=-1).reshape(-1, 1, 3)
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    return ((base + basis[None]) * a).reshape(-1, 3)


def wrap_into_box(x: np.ndarray, box: np.ndarray) -> np.ndarray:
    x = np.mod(x, box)
    return np.where(x >= box, 0.0, x)


def maxwell_boltzmann(rng: np.random.Generator, n: int, temperature: float,
                      mass: float = MASS) -> np.ndarray:
    """Velocities at `temperature` with zero net momentum and KE = (3N-3)/2 kB T exactly."""
    sigma = np.sqrt(KBOLTZ * temperature * FTM2V / mass)
    v = sigma * rng.standard_normal((n, 3))
    v -= v.mean(axis=0)
    if temperature <= 0.0 or n < 2:
        return np.zeros_like(v)
    ke = 0.5 * mass * np.sum(v * v) / FTM2V
    target = 0.5 * (3 * n - 3) * KBOLTZ * temperature
    return v * np.sqrt(target / ke)


def make_box(n_cells: int, rng: np.random.Generator, *, vacancy_fraction: float = 0.0,
             sigma_x: float = 0.01, temperature: float = 300.0, a: float = A_LAT) -> Box:
    sites = bcc_sites(n_cells, a)
    n_sites = sites.shape[0]
    n_vac = int(np.floor(vacancy_fraction * n_sites))
    keep = np.ones(n_sites, dtype=bool)
    if n_vac:
        keep[rng.choice(n_sites, n_vac, replace=False)] = False
    ids = np.nonzero(keep)[0]
    x = sites[ids]
    x = x + sigma_x * rng.standard_normal(x.shape)
    box = np.full(3, n_cells * a)
    x = wrap_into_box(x, box)
    v = maxwell_boltzmann(rng, x.shape[0], temperature)
    return Box(x=x, v=v, box=box, n_cells=n_cells, temperature=temperature, site_ids=ids)


# --- the five stated workloads ------------------------------------------------

def config_small() -> Box:
    """2,000 atoms (10^3 BCC cells), 300 K, seed 1."""
    return make_box(10, np.random.default_rng(1))


def config_128k() -> Box:
    """128,000 atoms (40^3 BCC cells), 300 K, seed 2."""
    return make_box(40, np.random.default_rng(2))


def config_810k() -> Box:
    """810,448 sites (74^3 BCC cells) minus 1 % vacancies = 802,344 atoms, 2,500 K, seed 3."""
    return make_box(74, np.random.default_rng(3), vacancy_fraction=0.01, temperature=2500.0)


def config_batch(n_rep: int = 256) -> List[Box]:
    """Independent replicas: edge n ~ U{5..20} cells, vacancies ~ U[0, 2 %], T ~ U[300, 2000] K."""
    out = []
    for r in range(n_rep):
        rng = np.random.default_rng([4, r])
        n = int(rng.integers(5, 21))
        frac = float(rng.uniform(0.0, 0.02))
        temp = float(rng.uniform(300.0, 2000.0))
        out.append(make_box(n, rng, vacancy_fraction=frac, temperature=temp))
    return out


def fm_sigma(temperature: float) -> float:
    """Static thermal displacement width used for force-matching snapshots (Debye-type estimate)."""
    return 0.065 * np.sqrt(temperature / 300.0)


def config_fm(n_cfg: int = 64, n_cells: int = 10) -> List[Box]:
    """Force-matching snapshots: BCC at a = 3.304, T_c ~ U(500, 3000) K, static displacements."""
    out = []
    for c in range(n_cfg):
        rng = np.random.default_rng([5, c])
        temp = float(rng.uniform(500.0, 3000.0))
        out.append(make_box(n_cells, rng, sigma_x=fm_sigma(temp), temperature=0.0))
        out[-1].temperature = temp
    return out


def small_box(n_cells: int, seed: int, *, sigma_x: float = 0.01, temperature: float = 300.0,
              vacancy_fraction: float = 0.0, a: float = A_LAT) -> Box:
    """Tiny test boxes with the same recipe."""
    return make_box(n_cells, np.random.default_rng(seed), vacancy_fraction=vacancy_fraction,
                    sigma_x=sigma_x, temperature=temperature, a=a)


# --- slab with open lateral boundaries --------------------------------------

def bcc_block(nx: int, ny: int, nz: int, a: float = A_LAT) -> np.ndarray:
    """Sites of an nx x ny x nz BCC block, site id = ((ix*ny + iy)*nz + iz)*2 + b."""
    ix, iy, iz = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nz, dtype=np.float64), indexing="ij")
    base = np.stack([ix, iy, iz], axis=-1).reshape(-1, 1, 3)
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    return ((base + basis[None]) * a).reshape(-1, 3)


def ortho_box(nx: int, ny: int, nz: int, seed: int, *, sigma_x: float = 0.05,
              temperature: float = 300.0, a: float = A_LAT) -> Box:
    """A periodic BCC box of nx x ny x nz cells with three different edge
    lengths (a cube cannot tell the x, y and z image lengths apart)."""
    rng = np.random.default_rng(seed)
    x = bcc_block(nx, ny, nz, a)
    x = x + sigma_x * rng.standard_normal(x.shape)
    box = np.array([nx * a, ny * a, nz * a])
    x = np.mod(x, box)
    v = maxwell_boltzmann(rng, x.shape[0], temperature)
    return Box(x=x, v=v, box=box, n_cells=nx, temperature=temperature,
               site_ids=np.arange(x.shape[0], dtype=np.int64))


def slab(nx: int, ny: int, nz: int, seed: int, *, vacuum: float = 12.0,
         temperature: float = 300.0, sigma_x: float = 0.01, a: float = A_LAT) -> Box:
    """A thin BCC slab, open in x and y, periodic in z (the paper's geometry:
    thin slabs with open lateral boundaries, Sec. IV-B).  The block sits
    `vacuum` A inside the lower x and y cell-grid edges; the box lengths of
    the open dimensions are negative (the convention of both the oracle and
    the library: a negative length marks an open dimension and gives the
    extent of its cell grid)."""
    rng = np.random.default_rng(seed)
    x = bcc_block(nx, ny, nz, a)
    x = x + sigma_x * rng.standard_normal(x.shape)
    x[:, 0] += vacuum
    x[:, 1] += vacuum
    lz = nz * a
    x[:, 2] = np.mod(x[:, 2], lz)
    x[:, 2] = np.where(x[:, 2] >= lz, 0.0, x[:, 2])
    box = np.array([-(nx * a + 2.0 * vacuum), -(ny * a + 2.0 * vacuum), lz])
    v = maxwell_boltzmann(rng, x.shape[0], temperature)
    return Box(x=x, v=v, box=box, n_cells=nx, temperature=temperature,
               site_ids=np.arange(x.shape[0], dtype=np.int64))


def config_slab_801792() -> Box:
    """The paper's benchmark slab shape: 256 x 261 x 6 BCC cells = 801,792 atoms,
    open in x and y, 300 K, seed 6."""
    return slab(256, 261, 6, 6)


# --- random substitutional binary alloy ---------------------------------------

def maxwell_boltzmann_masses(rng: np.random.Generator, mass: np.ndarray,
                             temperature: float) -> np.ndarray:
    """Velocities for per-atom masses: zero net momentum, KE = (3N-3)/2 kB T exactly."""
    mass = np.asarray(mass, dtype=np.float64)
    n = mass.shape[0]
    v = np.sqrt(KBOLTZ * temperature * FTM2V / mass)[:, None] * rng.standard_normal((n, 3))
    if temperature <= 0.0 or n < 2:
        return np.zeros_like(v)
    v -= (mass[:, None] * v).sum(axis=0) / mass.sum()
    ke = 0.5 * np.sum(mass[:, None] * v * v) / FTM2V
    return v * np.sqrt(0.5 * (3 * n - 3) * KBOLTZ * temperature / ke)


def alloy_box(n_cells: int, seed: int, *, frac_1: float = 0.5, masses=(180.95, 95.95),
              sigma_x: float = 0.01, temperature: float = 300.0, a: float = A_LAT) -> Box:
    """BCC box whose sites hold type 1 with probability frac_1, else type 0.
    Draw order: displacements, types, velocities."""
    rng = np.random.default_rng(seed)
    sites = bcc_sites(n_cells, a)
    x = sites + sigma_x * rng.standard_normal(sites.shape)
    box = np.full(3, n_cells * a)
    x = wrap_into_box(x, box)
    types = (rng.random(x.shape[0]) < frac_1).astype(np.int32)
    v = maxwell_boltzmann_masses(rng, np.asarray(masses)[types], temperature)
    return Box(x=x, v=v, box=box, n_cells=n_cells, temperature=temperature,
               site_ids=np.arange(x.shape[0], dtype=np.int64), types=types)


def multi_box(n_cells: int, seed: int, masses, *, sigma_x: float = 0.05,
              temperature: float = 300.0, a: float = A_LAT) -> Box:
    """BCC box whose sites hold types drawn uniformly from range(len(masses)).
    Draw order: displacements, types, velocities."""
    rng = np.random.default_rng(seed)
    sites = bcc_sites(n_cells, a)
    x = sites + sigma_x * rng.standard_normal(sites.shape)
    box = np.full(3, n_cells * a)
    x = wrap_into_box(x, box)
    types = rng.integers(0, len(masses), x.shape[0]).astype(np.int32)
    v = maxwell_boltzmann_masses(rng, np.asarray(masses)[types], temperature)
    return Box(x=x, v=v, box=box, n_cells=n_cells, temperature=temperature,
               site_ids=np.arange(x.shape[0], dtype=np.int64), types=types)


def config_alloy_128k() -> Box:
    """128,000-atom random equiatomic binary BCC alloy (40^3 cells), 300 K, seed 7."""
    return alloy_box(40, 7)
