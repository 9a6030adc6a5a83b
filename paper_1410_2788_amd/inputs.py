"""Seeded synthetic workloads for the NPB solver (inputs only).

This module draws molecules (atom positions, partial charges, radii) and
picks grids and run parameters.  It holds none of the solver's arithmetic:
no dielectric map, no charge spreading, no boundary potential, no time step.
Both the CPU oracle (through the tests and the benchmark) and the HIP
library consume what it returns, so it is the only code the two sides share.

Physical quantities are given as the paper states them (Sec. 2.1 and
Sec. 5.1): ionic strength in mol/L and temperature in K, not the derived
modified Debye-Hueckel parameter, which each side computes for itself.

Recipe (stand-ins for the paper's PDB proteins, which are not available):
  * positions: uniform in a ball (or an axis-scaled ball = ellipsoid):
    radius R * U**(1/3) times a normalised Gaussian direction;
  * radii: U[1.2, 2.0] Angstrom;
  * charges: N(0, 0.35) e, then shifted by one constant so that the sum
    equals the requested net charge.
All draws use numpy.random.default_rng (PCG64) with the stated seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


@dataclass
class Molecule:
    xyz: np.ndarray      # (N, 3) float64, Angstrom
    q: np.ndarray        # (N,) float64, units of e
    radius: np.ndarray   # (N,) float64, Angstrom

    @property
    def n_atoms(self) -> int:
        return int(self.q.shape[0])


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    h: float
    origin: Sequence[float]  # coordinates of node (0, 0, 0)

    @property
    def shape_zyx(self):
        return (self.nz, self.ny, self.nx)

    @property
    def interior_points(self) -> int:
        return (self.nx - 2) * (self.ny - 2) * (self.nz - 2)


@dataclass
class RunParams:
    eps_in: float
    eps_out: float
    ionic_molar: float
    temperature_K: float
    alpha: float
    dt: float
    n_steps: int
    scheme: str = "LODIE2"      # LODIE2 | LODIE1 | AOSIE2 | AOSIE1 | LODCN1 | LODCN2 |
                                # AOSCN1 | AOSCN2 | MAOSIE | MAOSCN
    richardson: bool = False
    vacuum: bool = True
    precision: str = "f64"      # f64 | f32 (GPU sweeps; the oracle is FP64)
    face_rule: str = "harmonic"  # harmonic (mean of the nodal eps) | location (eps at the half point)


@dataclass
class Workload:
    name: str
    molecule: Molecule
    grid: Grid
    params: RunParams
    extra: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# molecules

def random_cluster(seed, n_atoms: int, semi_axes, net_charge: float,
                   q_sigma: float = 0.35, r_lo: float = 1.2, r_hi: float = 2.0,
                   center=(0.0, 0.0, 0.0)) -> Molecule:
    """Atoms uniform in an ellipsoid with the given semi-axes (a ball when
    all three are equal), radii U[r_lo, r_hi], charges N(0, q_sigma)
    shifted to the requested net charge."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n_atoms, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = rng.random(n_atoms) ** (1.0 / 3.0)
    xyz = d * rad[:, None] * np.asarray(semi_axes, dtype=np.float64)[None, :]
    xyz += np.asarray(center, dtype=np.float64)[None, :]
    radius = rng.uniform(r_lo, r_hi, n_atoms)
    q = rng.normal(0.0, q_sigma, n_atoms)
    q += (net_charge - q.sum()) / n_atoms
    return Molecule(xyz=np.ascontiguousarray(xyz), q=q, radius=radius)


def single_ion(q: float = 1.0, radius: float = 2.0, pos=(0.0, 0.0, 0.0)) -> Molecule:
    return Molecule(xyz=np.array([pos], dtype=np.float64),
                    q=np.array([q], dtype=np.float64),
                    radius=np.array([radius], dtype=np.float64))


def cubic_grid(n: int, h: float, center=(0.0, 0.0, 0.0), ny=None, nz=None) -> Grid:
    """Grid of n (x) by ny by nz nodes with spacing h, centred on `center`."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    o = [center[0] - 0.5 * h * (n - 1), center[1] - 0.5 * h * (ny - 1),
         center[2] - 0.5 * h * (nz - 1)]
    return Grid(nx=n, ny=ny, nz=nz, h=h, origin=o)


def cluster_radius(n_atoms: int) -> float:
    """Ball radius that keeps the atom density of 2000 atoms in 20 Angstrom."""
    return 20.0 * (n_atoms / 2000.0) ** (1.0 / 3.0)


def grid_size_for(n_atoms: int, h: float, n_min: int, n_max: int) -> int:
    """Odd node count whose box half-width is twice the cluster radius."""
    R = cluster_radius(n_atoms)
    n = 2 * int(math.ceil(2.0 * R / h)) + 1
    return int(min(max(n, n_min), n_max))


# --------------------------------------------------------------------------
# named workloads

def born_sphere() -> Workload:
    """One +1 e ion of radius 2 at the origin (a grid node); eps 1/80;
    0.1 M salt at 300 K; box [-8, 8]^3, 65^3 nodes (h = 0.25); alpha 1,
    dt 0.1, 100 steps, plus the uniform-eps vacuum solve; FP64."""
    return Workload(
        name="born_sphere_65",
        molecule=single_ion(1.0, 2.0),
        grid=cubic_grid(65, 0.25),
        params=RunParams(eps_in=1.0, eps_out=80.0, ionic_molar=0.1,
                         temperature_K=300.0, alpha=1.0, dt=0.1, n_steps=100,
                         scheme="LODIE2", richardson=False, vacuum=True,
                         precision="f64"))


def globular_2000(precision: str = "f32", scheme: str = "LODIE2") -> Workload:
    """2000 atoms in a 20 A ball (seed 2), net -3 e; eps 2/80; 0.15 M at
    298 K; 161^3 nodes at h = 0.5; alpha 1/25; dt 0.2 / 0.1 with Richardson,
    20 / 40 steps, solvated and vacuum loops."""
    mol = random_cluster(2, 2000, (20.0, 20.0, 20.0), -3.0)
    return Workload(
        name="globular_2000_161",
        molecule=mol,
        grid=cubic_grid(161, 0.5),
        params=RunParams(eps_in=2.0, eps_out=80.0, ionic_molar=0.15,
                         temperature_K=298.0, alpha=1.0 / 25.0, dt=0.2,
                         n_steps=20, scheme=scheme, richardson=True,
                         vacuum=True, precision=precision))


def globular_2000_euler(n_steps: int = 1_000_000, dt: float = 1e-5) -> Workload:
    """The 2000-atom workload for the explicit Euler reference solver: FP64,
    dt = 1e-5 with alpha = 1/25 (T = n_steps dt; the paper's reference uses
    T = 10), no Richardson; the vacuum potential comes from the direct
    Poisson solve (vacuum_direct), as in Eq. (deltaG2)."""
    w = globular_2000(precision="f64", scheme="EULER")
    w.name = "globular_2000_161_euler"
    w.params = RunParams(eps_in=2.0, eps_out=80.0, ionic_molar=0.15, temperature_K=298.0,
                         alpha=1.0 / 25.0, dt=dt, n_steps=n_steps, scheme="EULER",
                         richardson=False, vacuum=False, precision="f64")
    return w


def large_complex(precision: str = "f32", scheme: str = "LODIE2", dt: float = 0.4,
                  n_steps: int = 20) -> Workload:
    """30000 atoms in a 45:36:27 A ellipsoid (seed 5), net -12 e; eps 4/80;
    0.5 M at 298 K; 321^3 nodes at h = 0.35; alpha 1/25."""
    mol = random_cluster(5, 30000, (45.0, 36.0, 27.0), -12.0)
    return Workload(
        name="large_complex_321",
        molecule=mol,
        grid=cubic_grid(321, 0.35),
        params=RunParams(eps_in=4.0, eps_out=80.0, ionic_molar=0.5,
                         temperature_K=298.0, alpha=1.0 / 25.0, dt=dt,
                         n_steps=n_steps, scheme=scheme, richardson=True,
                         vacuum=True, precision=precision))


def small_globular(seed=7, n_atoms=120, n=41, h=0.5, precision="f64",
                   scheme="LODIE2", richardson=True, ny=None, nz=None,
                   n_steps=6, dt=0.2, alpha=1.0 / 25.0, ionic_molar=0.15,
                   eps_in=2.0, eps_out=80.0, net=-1.0) -> Workload:
    """A reduced globular molecule the oracle solves in about a second;
    same distributions as the 2000-atom case, cluster radius scaled to the
    atom count.  Optional ny/nz give non-cubic (ragged) grids."""
    R = cluster_radius(n_atoms)
    mol = random_cluster(seed, n_atoms, (R, R, R), net)
    return Workload(
        name=f"globular_{n_atoms}_{n}",
        molecule=mol,
        grid=cubic_grid(n, h, ny=ny, nz=nz),
        params=RunParams(eps_in=eps_in, eps_out=eps_out, ionic_molar=ionic_molar,
                         temperature_K=298.0, alpha=alpha, dt=dt, n_steps=n_steps,
                         scheme=scheme, richardson=richardson, vacuum=True,
                         precision=precision))


def batch_mix(n_mol: int = 64, seed: int = 3, precision: str = "f32",
              scheme: str = "LODIE2", n_min: int = 65, n_max: int = 193,
              a_lo: float = 200.0, a_hi: float = 5000.0, n_steps: int = 20) -> List[Workload]:
    """Uneven batch: atom counts log-uniform in [a_lo, a_hi] (seeds (seed, i)),
    same distributions as above, h = 0.5, grid from the cluster size."""
    out = []
    for i in range(n_mol):
        rng = np.random.default_rng((seed, i))
        n_atoms = int(round(math.exp(rng.uniform(math.log(a_lo), math.log(a_hi)))))
        R = cluster_radius(n_atoms)
        mol = random_cluster((seed, i, 1), n_atoms, (R, R, R), float(round(rng.normal(0, 3))))
        n = grid_size_for(n_atoms, 0.5, n_min, n_max)
        out.append(Workload(
            name=f"batch_{seed}_{i}",
            molecule=mol,
            grid=cubic_grid(n, 0.5),
            params=RunParams(eps_in=2.0, eps_out=80.0, ionic_molar=0.15,
                             temperature_K=298.0, alpha=1.0 / 25.0, dt=0.2,
                             n_steps=n_steps, scheme=scheme, richardson=True,
                             vacuum=True, precision=precision)))
    return out


def serve_requests(n_req: int, seed: int = 4, precision: str = "f32") -> List[Workload]:
    """Serving requests: atom counts log-uniform in [500, 20000] (seeds
    (seed, i)), grids 103..257 nodes at h = 0.5 from the cluster size,
    LODIE2 RE+V with 20 / 40 steps."""
    return batch_mix(n_mol=n_req, seed=seed, precision=precision, n_min=103, n_max=257,
                     a_lo=500.0, a_hi=20000.0, n_steps=20)


def poisson_arrivals(rate_per_s: float, n_req: int, seed: int = 4) -> np.ndarray:
    """Arrival times (s) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n_req))


# --------------------------------------------------------------------------
# the analytic benchmark: a charged spherical cavity (Sec. 4.1)

@dataclass
class SphereBenchmark:
    """Fields of the charged-cavity benchmark on [-L, L]^3 (dimensionless).

    exact  : Eq. (NPB_analytical_1), 1/(eps R) - 1/R + 1/r inside the ball
             of radius R, 1/(eps r) outside, eps = eps_out / eps_in
    rho    : Eq. (NPB_analytical_2): kbar^2 sinh(1/(eps r)) outside the ball,
             and the centred charge 4 pi eps_in delta as 4 pi eps_in / h^3 on
             the centre node (a node-centred trilinear spread); zero on the
             ball's surface nodes (they count as solute, where kbar = 0) and
             on the outer shell
    u0     : Eq. (InitSolutions), H cos(pi x/6) cos(pi y/6) cos(pi z/6) +
             1/(eps r); the singular term is dropped at the centre node.  Its
             outer shell equals the exact solution (the Dirichlet data).
    valid  : nodes entering the error norms: all but the singular centre"""
    grid: Grid
    solute: Molecule
    u0: np.ndarray
    rho: np.ndarray
    exact: np.ndarray
    valid: np.ndarray
    eps_in: float
    eps_out: float
    kbar_sq: float
    radius: float
    H: float


def sphere_benchmark(h: float, H: float = 1.0, radius: float = 1.0, eps_in: float = 1.0,
                     eps_out: float = 80.0, kbar_sq: float = 1.0, half_width: float = 3.0
                     ) -> SphereBenchmark:
    """Sec. 4.1: R = 1 Angstrom, eps_in = 1, eps_out = 80, kbar = 1 on the
    cube [-3, 3]^3 with spacing h (h must divide 3)."""
    n = int(round(2.0 * half_width / h)) + 1
    if abs((n - 1) * h - 2.0 * half_width) > 1e-12:
        raise ValueError("h must divide the box width")
    grid = cubic_grid(n, h)
    ax = grid.origin[0] + np.arange(n) * h
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    c = n // 2
    eps = eps_out / eps_in
    rs = r.copy()
    rs[c, c, c] = 1.0  # placeholder at the singular node
    exact = np.where(r < radius, 1.0 / (eps * radius) - 1.0 / radius + 1.0 / rs, 1.0 / (eps * rs))
    exact[c, c, c] = 0.0
    valid = np.ones(r.shape, dtype=bool)
    valid[c, c, c] = False
    # solute: nodes with r^2 <= R^2 (on the surface included)
    solvent = (X * X + Y * Y) + Z * Z > radius * radius
    rho = np.where(solvent, kbar_sq * np.sinh(1.0 / (eps * rs)), 0.0)
    rho[c, c, c] = 4.0 * math.pi * eps_in / h ** 3
    shell = np.zeros(r.shape, dtype=bool)
    shell[0, :, :] = shell[-1, :, :] = shell[:, 0, :] = shell[:, -1, :] = True
    shell[:, :, 0] = shell[:, :, -1] = True
    rho[shell] = 0.0
    u0 = H * np.cos(math.pi * X / 6.0) * np.cos(math.pi * Y / 6.0) * np.cos(math.pi * Z / 6.0) \
        + 1.0 / (eps * rs)
    u0[c, c, c] = H
    u0[shell] = exact[shell]
    solute = Molecule(xyz=np.zeros((1, 3)), q=np.zeros(1), radius=np.array([radius]))
    return SphereBenchmark(grid, solute, u0, rho, exact, valid, eps_in, eps_out, kbar_sq, radius,
                           H)
