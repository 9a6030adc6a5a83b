"""FP64 CPU oracle: pseudo-transient NPB solver with LOD / AOS time splitting.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import or run this module.
It shares no code with the HIP library and never imports it.

Plain NumPy, float64, no fast-math, written to be checked against the paper
by eye (Wilson & Zhao, "Unconditionally stable time splitting methods for
the electrostatic analysis of solvated biomolecules"):

  * model and units ............ Sec. 2.1, Eqs. (NPB), (RhoEq), (DebyeHuckel),
                                 (BoundaryCond)
  * pseudo-time equation ....... Sec. 2.2, Eq. (TimeDepNPB)
  * analytic sinh sub-step ..... Sec. 3.1, Eqs. (ana1)-(ana3)
  * LODIE1 / LODIE2 ............ Sec. 3.1, Eqs. (LODIE1_1)-(LODIE1_5),
                                 (SpatialOperators); LODIE2 = same five
                                 equations with the source first and the
                                 nonlinear sub-step last
  * LODCN1 / LODCN2 ............ Sec. 3.1, Eqs. (LODCN1_2)-(LODCN1_4) in
                                 place of the three implicit sweeps
  * AOSIE1 / AOSIE2 ............ Sec. 3.2, Eqs. (AOSIE1_1)-(AOSIE1_5),
                                 (AOSIE2_2)-(AOSIE2_4)
  * AOSCN1 / AOSCN2 ............ Sec. 3.2, Eqs. (AOSCN1_2)-(AOSCN1_4),
                                 (AOSCN2_2)-(AOSCN2_4)
  * MAOSIE / MAOSCN ............ Sec. 3.3, Eqs. (MAOS1_1)-(MAOS1_5), implicit
                                 Euler or Crank-Nicolson in the three
                                 directional sub-systems
  * explicit Euler ............. Sec. 2.3 (the scheme the splittings
                                 replace) and Sec. 5.2 / 5.4 (the reference
                                 energies): Eq. (TimeDepNPB) stepped
                                 explicitly with Eq. (SpatialOperators)
  * solvation energy ........... Sec. 5.1, Eq. (deltaG); vacuum by the same
                                 scheme, Sec. 5.3, Eq. (deltaG3)
  * Richardson extrapolation ... Sec. 5.3, Eq. (rich)
  * vacuum potential by a fast   Sec. 5.1 (text after Eq. (deltaG)),
    Poisson solver, energy and   Sec. 5.3, Eq. (deltaG2); recovered
    recovered potential ........ potential, Sec. 5.4 (surface potential
                                 paragraph)

Readings of points the paper leaves open (each listed in the design notes):
  * kT(T) = 0.592183 * T / 298 kcal/mol; Bjerrum length l_B = 332.06371 / kT
    Angstrom, so rho = 4 pi l_B sum q delta and the boundary prefactor
    e^2/(k_B T) = l_B;
  * the modified Debye-Hueckel parameter at temperature T is
    8.486902807 * (298 / T) * I (Angstrom^-2, I in mol/L);
  * solute region = union of atomic balls, a node on a sphere counts as
    solute; face dielectric = harmonic mean of the two nodal values, or,
    with face_rule "location", eps_in or eps_out by whether the half point
    itself lies in the solute (the paper's own rule, applied to the same
    union of balls);
  * the AOS nonlinear sub-step is the exact flow of alpha w_t = -4 kbar^2
    sinh(w) over dt, i.e. Eq. (ana3) with theta replaced by 4 theta (the
    printed leading factor 4 would map u to 4u when kbar = 0);
  * the vacuum problem uses eps_in everywhere, kbar = 0 and Coulomb
    boundary data in eps_in;
  * a charge stencil (8 trilinear nodes) must lie in the interior;
  * explicit Euler evaluates kbar^2 sinh(u) at the old step, and the term
    is absent (not 0 * sinh) where kbar = 0;
  * the recovered potential is phi_m - phi_0^LOD + phi_0^FFT (the printed
    "+ phi_0^LOD - phi_0^FFT" is the only other sign pattern; with it
    (1/2) sum Q (phi_rec - phi_0^FFT) would not equal the RE+V energy).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.fft import dstn, idstn

# ---------------------------------------------------------------------------
# constants (Sec. 2.1)

KT_298_KCAL = 0.592183          # kcal/mol per unit dimensionless potential at 298 K
KBAR2_PER_MOLAR_298 = 8.486902807  # Angstrom^-2 per mol/L at 298 K
COULOMB_KCAL_A = 332.06371      # e^2/(4 pi eps0) in kcal Angstrom / mol (CODATA)

SCHEMES = ("LODIE2", "LODIE1", "AOSIE2", "AOSIE1", "LODCN1", "LODCN2", "AOSCN1", "AOSCN2",
           "MAOSIE", "MAOSCN", "EULER")


def thermal_energy(T: float) -> float:
    """k_B T in kcal/mol: the paper's 0.592183 at 298 K, scaled to T."""
    return KT_298_KCAL * T / 298.0


def bjerrum_length(T: float) -> float:
    """e^2/(k_B T) in Angstrom (vacuum), the prefactor of Eqs. (RhoEq) and
    (BoundaryCond) in the dimensionless form."""
    return COULOMB_KCAL_A / thermal_energy(T)


def kappa_bar_sq(ionic_molar: float, T: float) -> float:
    """Eq. (DebyeHuckel): kbar^2 = 8.486902807 I Angstrom^-2 at 298 K; the
    1/T dependence of the prefactor gives the value at T."""
    return KBAR2_PER_MOLAR_298 * (298.0 / T) * ionic_molar


class ChargeStencilError(ValueError):
    """An atom's trilinear stencil touches the Dirichlet boundary shell."""


# ---------------------------------------------------------------------------
# grid helpers; arrays are indexed [k, j, i] = [z, y, x]

def axis_coords(grid, axis_xyz: int) -> np.ndarray:
    """x_i = origin + i h along x (0), y (1) or z (2)."""
    n = (grid.nx, grid.ny, grid.nz)[axis_xyz]
    return grid.origin[axis_xyz] + np.arange(n, dtype=np.float64) * grid.h


def shape_zyx(grid):
    return (grid.nz, grid.ny, grid.nx)


def boundary_shell(grid) -> np.ndarray:
    """True on the outer layer of nodes (the Dirichlet set)."""
    B = np.zeros(shape_zyx(grid), dtype=bool)
    B[0, :, :] = B[-1, :, :] = True
    B[:, 0, :] = B[:, -1, :] = True
    B[:, :, 0] = B[:, :, -1] = True
    return B


# ---------------------------------------------------------------------------
# setup: dielectric map, charges, boundary data

def solute_mask(grid, xyz, radius) -> np.ndarray:
    """Nodes inside or on any atomic sphere: |x - r_a|^2 <= R_a^2, evaluated
    as ((dx^2 + dy^2) + dz^2) in float64.  Per-atom bounding box."""
    X, Y, Z = (axis_coords(grid, d) for d in range(3))
    M = np.zeros(shape_zyx(grid), dtype=bool)
    h = grid.h
    for a in range(xyz.shape[0]):
        xa, ya, za = xyz[a]
        R = radius[a]
        lo, hi = [], []
        for d, c in enumerate((xa, ya, za)):
            n = (grid.nx, grid.ny, grid.nz)[d]
            lo.append(max(int(math.floor((c - R - grid.origin[d]) / h)) - 1, 0))
            hi.append(min(int(math.ceil((c + R - grid.origin[d]) / h)) + 1, n - 1))
        if any(l > u for l, u in zip(lo, hi)):
            continue
        dx = X[lo[0]:hi[0] + 1] - xa
        dy = Y[lo[1]:hi[1] + 1] - ya
        dz = Z[lo[2]:hi[2] + 1] - za
        d2 = (dx * dx)[None, None, :] + (dy * dy)[None, :, None]
        d2 = d2 + (dz * dz)[:, None, None]
        M[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] |= d2 <= R * R
    return M


def face_solute(grid, xyz, radius, axis_xyz: int) -> np.ndarray:
    """Half points between consecutive nodes along x (0), y (1) or z (2)
    that lie inside or on an atomic sphere; the half point of nodes i and
    i + 1 has coordinate origin + (i + 1/2) h, and |x - r_a|^2 is evaluated
    as in solute_mask.  Shape: the node array with one fewer entry along
    that axis."""
    h = grid.h
    n = (grid.nx, grid.ny, grid.nz)
    C = []
    for d in range(3):
        if d == axis_xyz:
            C.append(grid.origin[d] + (np.arange(n[d] - 1, dtype=np.float64) + 0.5) * h)
        else:
            C.append(axis_coords(grid, d))
    shape = [len(C[2]), len(C[1]), len(C[0])]
    F = np.zeros(shape, dtype=bool)
    for a in range(xyz.shape[0]):
        xa, ya, za = xyz[a]
        R = radius[a]
        sl = []
        for d, c in enumerate((xa, ya, za)):
            m = len(C[d])
            lo = max(int(math.floor((c - R - grid.origin[d]) / h)) - 1, 0)
            hi = min(int(math.ceil((c + R - grid.origin[d]) / h)) + 1, m - 1)
            sl.append((lo, hi))
        if any(l > u for l, u in sl):
            continue
        dx = C[0][sl[0][0]:sl[0][1] + 1] - xa
        dy = C[1][sl[1][0]:sl[1][1] + 1] - ya
        dz = C[2][sl[2][0]:sl[2][1] + 1] - za
        d2 = (dx * dx)[None, None, :] + (dy * dy)[None, :, None]
        d2 = d2 + (dz * dz)[:, None, None]
        F[sl[2][0]:sl[2][1] + 1, sl[1][0]:sl[1][1] + 1, sl[0][0]:sl[0][1] + 1] |= d2 <= R * R
    return F


def spread_charges(grid, xyz, q) -> np.ndarray:
    """Trilinear distribution Q(x_i, y_j, z_k) of the point charges (Sec. 3.1,
    text after Eq. (SpatialOperators)): with g = (r_a - origin)/h, i0 =
    floor(g), f = g - i0, corner (dx, dy, dz) gets q_a * wx * wy * wz where
    w = f for the upper corner and 1 - f for the lower one.  Accumulated atom
    by atom, in atom order.  Units: e."""
    Q = np.zeros(shape_zyx(grid), dtype=np.float64)
    n = (grid.nx, grid.ny, grid.nz)
    for a in range(xyz.shape[0]):
        i0, f = [], []
        for d in range(3):
            g = (xyz[a, d] - grid.origin[d]) / grid.h
            fl = math.floor(g)
            i0.append(int(fl))
            f.append(g - fl)
            if i0[d] < 1 or i0[d] + 1 > n[d] - 2:
                raise ChargeStencilError(f"atom {a}: stencil touches the boundary")
        for cz in (0, 1):
            wz = f[2] if cz else 1.0 - f[2]
            for cy in (0, 1):
                wy = f[1] if cy else 1.0 - f[1]
                for cx in (0, 1):
                    wx = f[0] if cx else 1.0 - f[0]
                    w = wx * wy * wz
                    Q[i0[2] + cz, i0[1] + cy, i0[0] + cx] += q[a] * w
    return Q


def source_density(Q: np.ndarray, h: float, T: float) -> np.ndarray:
    """Eq. (RhoEq) on the grid: rho = 4 pi l_B Q / h^3 (a unit charge spread
    over one cell volume)."""
    return (4.0 * math.pi * bjerrum_length(T) / (h * h * h)) * Q


def boundary_potential(grid, xyz, q, eps: float, kbar2: float, T: float,
                       chunk: int = 4096) -> np.ndarray:
    """Eq. (BoundaryCond) on the boundary shell, zero inside:
    u = l_B sum_i q_i exp(-kbar d / sqrt(eps)) / (eps d), d = |r - r_i|."""
    u = np.zeros(shape_zyx(grid), dtype=np.float64)
    B = boundary_shell(grid)
    kk, jj, ii = np.nonzero(B)
    P = np.stack([axis_coords(grid, 0)[ii], axis_coords(grid, 1)[jj],
                  axis_coords(grid, 2)[kk]], axis=1)
    kappa = math.sqrt(kbar2 / eps)
    lB = bjerrum_length(T)
    vals = np.empty(P.shape[0])
    for s in range(0, P.shape[0], chunk):
        p = P[s:s + chunk]
        d = np.sqrt(((p[:, None, :] - xyz[None, :, :]) ** 2).sum(axis=2))
        vals[s:s + chunk] = lB * (q[None, :] * np.exp(-kappa * d) / (eps * d)).sum(axis=1)
    u[kk, jj, ii] = vals
    return u


# ---------------------------------------------------------------------------
# the split operators

def face_eps(eps_node: np.ndarray, axis: int) -> np.ndarray:
    """eps at the half points between consecutive nodes along `axis` (array
    axis), harmonic mean of the two nodal values (the default face rule)."""
    n = eps_node.shape[axis]
    e0 = np.take(eps_node, np.arange(0, n - 1), axis=axis)
    e1 = np.take(eps_node, np.arange(1, n), axis=axis)
    return 2.0 * e0 * e1 / (e0 + e1)


def thomas(a, b, c, d):
    """Thomas algorithm, no pivoting, for independent systems stored along
    axis 0: a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i], i = 0..m-1
    (a[0] and c[m-1] are ignored)."""
    m = d.shape[0]
    cp = np.empty_like(d)
    dp = np.empty_like(d)
    cp[0] = c[0] / b[0]
    dp[0] = d[0] / b[0]
    for i in range(1, m):
        den = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / den
        dp[i] = (d[i] - a[i] * dp[i - 1]) / den
    x = np.empty_like(d)
    x[m - 1] = dp[m - 1]
    for i in range(m - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def implicit_sweep(s: np.ndarray, eps_node: np.ndarray, tau: float, h: float,
                   axis: int, faces=None) -> np.ndarray:
    """One implicit-Euler 1-D sub-step (Eqs. (LODIE1_2)-(LODIE1_4)):
    solve (1 - tau delta^2) v = s on every interior grid line along array
    axis `axis` (0 = z, 1 = y, 2 = x), with delta^2 the central difference of
    Eq. (SpatialOperators) and Dirichlet values taken from s at both ends.
    Nodes not on an interior line are returned unchanged.  `faces` (eps at
    the half points along `axis`) replaces the harmonic means when given."""
    S = np.moveaxis(s, axis, 0)                 # (n, A, B) view
    E = np.moveaxis(face_eps(eps_node, axis) if faces is None else faces, axis, 0)
    n = S.shape[0]
    Si = S[:, 1:-1, 1:-1]
    Ei = E[:, 1:-1, 1:-1]
    r = tau / (h * h)
    eL = Ei[0:n - 2]          # eps at i - 1/2 for i = 1..n-2
    eR = Ei[1:n - 1]          # eps at i + 1/2
    a = -r * eL
    c = -r * eR
    b = 1.0 + r * (eL + eR)
    d = Si[1:n - 1].copy()
    d[0] -= a[0] * Si[0]
    d[-1] -= c[-1] * Si[n - 1]
    L = d.shape[1] * d.shape[2]
    x = thomas(a.reshape(n - 2, L), b.reshape(n - 2, L), c.reshape(n - 2, L),
               d.reshape(n - 2, L)).reshape(d.shape)
    out = s.copy()
    O = np.moveaxis(out, axis, 0)
    O[1:n - 1, 1:-1, 1:-1] = x
    return out


def explicit_half(s: np.ndarray, eps_node: np.ndarray, c: float, h: float,
                  axis: int, faces=None) -> np.ndarray:
    """(1 + c delta^2) s along array axis `axis` on the interior nodes (the
    central difference of Eq. (SpatialOperators), neighbours on the shell
    included); other nodes are returned unchanged."""
    S = np.moveaxis(s, axis, 0)
    E = np.moveaxis(face_eps(eps_node, axis) if faces is None else faces, axis, 0)
    out = s.copy()
    O = np.moveaxis(out, axis, 0)
    mid = S[1:-1, 1:-1, 1:-1]
    up = S[2:, 1:-1, 1:-1]
    dn = S[:-2, 1:-1, 1:-1]
    e_up = E[1:, 1:-1, 1:-1]     # eps at i + 1/2, i = 1..n-2
    e_dn = E[:-1, 1:-1, 1:-1]    # eps at i - 1/2
    O[1:-1, 1:-1, 1:-1] = mid + (c / (h * h)) * (e_up * (up - mid) + e_dn * (dn - mid))
    return out


def cn_sweep(s: np.ndarray, eps_node: np.ndarray, tau: float, h: float, axis: int,
             faces=None) -> np.ndarray:
    """One Crank-Nicolson 1-D sub-step (Eqs. (LODCN1_2)-(LODCN1_4)):
    (1 - tau/2 delta^2) v = (1 + tau/2 delta^2) s on every interior line,
    Dirichlet values at both ends."""
    return implicit_sweep(explicit_half(s, eps_node, 0.5 * tau, h, axis, faces), eps_node,
                          0.5 * tau, h, axis, faces)


def nonlinear_substep(u: np.ndarray, theta: np.ndarray, interior: np.ndarray) -> np.ndarray:
    """Exact flow of alpha w_t = -kbar^2 sinh(w) over one step (Eq. (ana3)):
    w = ln[(cosh t + e^{-u} sinh t) / (e^{-u} cosh t + sinh t)], t = theta
    per node.  Where theta = 0 (solute, kbar = 0) the flow is the identity.
    Applied on interior nodes only; the Dirichlet shell is never changed."""
    w = u.copy()
    sel = interior & (theta != 0.0)
    t = theta[sel]
    us = u[sel]
    # Same ratio; for u < 0 numerator and denominator are multiplied by e^{u}
    # so that e^{-u} never overflows double (|u| > 709 occurs in AOS runs).
    pos = us >= 0.0
    e = np.exp(-np.abs(us))           # e^{-u} for u >= 0, e^{u} for u < 0
    ch, sh = np.cosh(t), np.sinh(t)
    num = np.where(pos, ch + e * sh, e * ch + sh)
    den = np.where(pos, e * ch + sh, ch + e * sh)
    w[sel] = np.log(num / den)
    return w


# ---------------------------------------------------------------------------
# one problem (solvated or vacuum) and its time loop

@dataclass
class Problem:
    grid: object
    eps_node: np.ndarray     # nodal dielectric
    kbar2_node: np.ndarray   # kbar^2 per node (0 in the solute)
    Q: np.ndarray            # trilinear charges (e)
    rho: np.ndarray          # source density
    u0: np.ndarray           # initial field: boundary data on the shell, 0 inside
    interior: np.ndarray
    T: float
    # eps at the half points per array axis (z, y, x); None: harmonic means
    # of eps_node (the default face rule)
    faces: object = None

    def face(self, axis: int):
        return None if self.faces is None else self.faces[axis]


def location_faces(grid, xyz, radius, eps_in: float, eps_out: float):
    """eps at every half point by its own location (Sec. 3.1, text after
    Eq. (SpatialOperators)): eps_in where the half point lies in the solute
    (on or inside a sphere), eps_out elsewhere; per array axis (z, y, x)."""
    return [np.where(face_solute(grid, xyz, radius, ax), float(eps_in), float(eps_out))
            for ax in (2, 1, 0)]


def make_problem(mol, grid, params, medium: str = "solvated") -> Problem:
    """Time-independent data of Sec. 3.1 (text after Eq. (SpatialOperators)):
    Q and eps computed once; Dirichlet data from Eq. (BoundaryCond).  The
    face rule (params.face_rule): "harmonic" (harmonic mean of the nodal
    values) or "location" (by the half point's own location); the vacuum
    problem is uniform, so both rules agree there."""
    T = params.temperature_K
    Q = spread_charges(grid, mol.xyz, mol.q)
    rho = source_density(Q, grid.h, T)
    interior = ~boundary_shell(grid)
    if medium == "solvated":
        kb2 = kappa_bar_sq(params.ionic_molar, T)
        M = solute_mask(grid, mol.xyz, mol.radius)
        eps_node = np.where(M, params.eps_in, params.eps_out)
        kbar2_node = np.where(M, 0.0, kb2)
        u0 = boundary_potential(grid, mol.xyz, mol.q, params.eps_out, kb2, T)
        if getattr(params, "face_rule", "harmonic") == "location":
            return Problem(grid, eps_node, kbar2_node, Q, rho, u0, interior, T,
                           location_faces(grid, mol.xyz, mol.radius, params.eps_in,
                                          params.eps_out))
    elif medium == "vacuum":
        eps_node = np.full(shape_zyx(grid), float(params.eps_in))
        kbar2_node = np.zeros(shape_zyx(grid))
        u0 = boundary_potential(grid, mol.xyz, mol.q, params.eps_in, 0.0, T)
    else:
        raise ValueError(medium)
    return Problem(grid, eps_node, kbar2_node, Q, rho, u0, interior, T)


def problem_from_fields(grid, solute, eps_in: float, eps_out: float, kbar2: float,
                        rho: np.ndarray, u0: np.ndarray, T: float = 298.0,
                        face_rule: str = "harmonic") -> Problem:
    """A problem posed by fields (the analytic benchmark of Sec. 4.1): the
    solute balls set eps and kbar^2 as in make_problem, rho is the given
    dense source and u0 the given initial field, whose shell is the
    Dirichlet data.  Q is zero (no energies)."""
    M = solute_mask(grid, solute.xyz, solute.radius)
    interior = ~boundary_shell(grid)
    faces = (location_faces(grid, solute.xyz, solute.radius, eps_in, eps_out)
             if face_rule == "location" else None)
    return Problem(grid, np.where(M, eps_in, eps_out), np.where(M, 0.0, kbar2),
                   np.zeros(shape_zyx(grid)), np.where(interior, rho, 0.0), u0.copy(), interior,
                   T, faces)


def lod_step(u, pb: Problem, dt: float, alpha: float, order: str = "LODIE2"):
    """One LOD step.  LODIE1: N, X, Y, Z, S (Eqs. (LODIE1_1)-(LODIE1_5));
    LODIE2: S, X, Y, Z, N (Sec. 3.1, last paragraph); LODCN1 / LODCN2: the
    same orders with the Crank-Nicolson sweeps of Eqs. (LODCN1_2)-(LODCN1_4)."""
    tau = dt / alpha
    theta = pb.kbar2_node * dt / (2.0 * alpha)
    h = pb.grid.h
    if order == "LODIE2":
        s = u + tau * pb.rho
        v = implicit_sweep(s, pb.eps_node, tau, h, axis=2, faces=pb.face(2))
        p = implicit_sweep(v, pb.eps_node, tau, h, axis=1, faces=pb.face(1))
        qq = implicit_sweep(p, pb.eps_node, tau, h, axis=0, faces=pb.face(0))
        return nonlinear_substep(qq, theta, pb.interior)
    if order == "LODIE1":
        w = nonlinear_substep(u, theta, pb.interior)
        v = implicit_sweep(w, pb.eps_node, tau, h, axis=2, faces=pb.face(2))
        p = implicit_sweep(v, pb.eps_node, tau, h, axis=1, faces=pb.face(1))
        qq = implicit_sweep(p, pb.eps_node, tau, h, axis=0, faces=pb.face(0))
        return qq + tau * pb.rho
    if order == "LODCN2":
        s = u + tau * pb.rho
        v = cn_sweep(s, pb.eps_node, tau, h, axis=2, faces=pb.face(2))
        p = cn_sweep(v, pb.eps_node, tau, h, axis=1, faces=pb.face(1))
        qq = cn_sweep(p, pb.eps_node, tau, h, axis=0, faces=pb.face(0))
        return nonlinear_substep(qq, theta, pb.interior)
    if order == "LODCN1":
        w = nonlinear_substep(u, theta, pb.interior)
        v = cn_sweep(w, pb.eps_node, tau, h, axis=2, faces=pb.face(2))
        p = cn_sweep(v, pb.eps_node, tau, h, axis=1, faces=pb.face(1))
        qq = cn_sweep(p, pb.eps_node, tau, h, axis=0, faces=pb.face(0))
        return qq + tau * pb.rho
    raise ValueError(order)


def aos_step(u, pb: Problem, dt: float, alpha: float, variant: str = "AOSIE2"):
    """One AOS step (Eqs. (AOSIE1_1)-(AOSIE1_5); AOSIE2 replaces the three
    sweeps by Eqs. (AOSIE2_2)-(AOSIE2_4); AOSCN1 / AOSCN2 by Eqs.
    (AOSCN1_2)-(AOSCN1_4) / (AOSCN2_2)-(AOSCN2_4)).  Four independent
    sub-solves from u^n, then their arithmetic mean.  In the Crank-Nicolson
    forms the source stays outside the explicit half."""
    tau = dt / alpha
    h = pb.grid.h
    theta4 = 4.0 * pb.kbar2_node * dt / (2.0 * alpha)
    if variant in ("AOSIE1", "AOSCN1"):
        cx, cy, cz = 4.0, 0.0, 0.0
    elif variant in ("AOSIE2", "AOSCN2"):
        cx = cy = cz = 4.0 / 3.0
    else:
        raise ValueError(variant)
    w = nonlinear_substep(u, theta4, pb.interior)
    if variant.startswith("AOSIE"):
        v = implicit_sweep(u + cx * tau * pb.rho, pb.eps_node, 4.0 * tau, h, 2, pb.face(2))
        p = implicit_sweep(u + cy * tau * pb.rho, pb.eps_node, 4.0 * tau, h, 1, pb.face(1))
        qq = implicit_sweep(u + cz * tau * pb.rho, pb.eps_node, 4.0 * tau, h, 0, pb.face(0))
    else:
        def cn(axis, c):
            rhs = explicit_half(u, pb.eps_node, 2.0 * tau, h, axis, pb.face(axis))
            rhs = rhs + c * tau * pb.rho
            return implicit_sweep(rhs, pb.eps_node, 2.0 * tau, h, axis, pb.face(axis))
        v, p, qq = cn(2, cx), cn(1, cy), cn(0, cz)
    out = u.copy()
    I = pb.interior
    out[I] = 0.25 * (w[I] + v[I] + p[I] + qq[I])
    return out


def maos_step(u, pb: Problem, dt: float, alpha: float, variant: str = "MAOSIE"):
    """One MAOS step (Sec. 3.3, Eqs. (MAOS1_1)-(MAOS1_5)): the exact flow of
    the sinh term first (Eq. (ana3), theta = kbar^2 dt / (2 alpha)), then
    three independent directional sub-solves of alpha v_t = 3 d/dx(eps dv/dx)
    + rho from it -- implicit Euler, (1 - 3 tau delta^2) v = w + tau rho, or
    Crank-Nicolson, (1 - 3 tau/2 delta^2) v = (1 + 3 tau/2 delta^2) w + tau rho
    -- and their arithmetic mean."""
    tau = dt / alpha
    h = pb.grid.h
    theta = pb.kbar2_node * dt / (2.0 * alpha)
    w = nonlinear_substep(u, theta, pb.interior)
    subs = []
    for axis in (2, 1, 0):
        if variant == "MAOSIE":
            subs.append(implicit_sweep(w + tau * pb.rho, pb.eps_node, 3.0 * tau, h, axis,
                                       pb.face(axis)))
        elif variant == "MAOSCN":
            rhs = explicit_half(w, pb.eps_node, 1.5 * tau, h, axis, pb.face(axis)) + tau * pb.rho
            subs.append(implicit_sweep(rhs, pb.eps_node, 1.5 * tau, h, axis, pb.face(axis)))
        else:
            raise ValueError(variant)
    out = u.copy()
    I = pb.interior
    out[I] = (subs[0][I] + subs[1][I] + subs[2][I]) / 3.0
    return out


def euler_step(u, pb: Problem, dt: float, alpha: float):
    """One explicit Euler step of Eq. (TimeDepNPB) with the spatial operator
    of Eq. (SpatialOperators) (the paper's reference solver, Sec. 5.2 and
    Sec. 5.4): u + tau (sum over x, y, z of delta(eps delta u) - kbar^2
    sinh u + rho), tau = dt / alpha, on the interior nodes; the Dirichlet
    shell is unchanged."""
    tau = dt / alpha
    h = pb.grid.h
    div = np.zeros_like(u)
    for axis in (2, 1, 0):
        div += explicit_half(u, pb.eps_node, 1.0, h, axis, pb.face(axis)) - u
    # the sinh term exists only where kbar != 0 (solvent): elsewhere it is
    # absent, not 0 * sinh(u) (which would overflow for |u| > 710)
    nl = np.zeros_like(u)
    sel = pb.interior & (pb.kbar2_node != 0.0)
    nl[sel] = pb.kbar2_node[sel] * np.sinh(u[sel])
    out = u.copy()
    I = pb.interior
    out[I] = u[I] + tau * (div[I] - nl[I] + pb.rho[I])
    return out


def run(pb: Problem, dt: float, alpha: float, n_steps: int, scheme: str = "LODIE2",
        u_init=None) -> np.ndarray:
    """Fixed number of pseudo-time steps from u^0 (zero inside)."""
    u = pb.u0.copy() if u_init is None else u_init.copy()
    for _ in range(n_steps):
        if scheme in ("LODIE2", "LODIE1", "LODCN1", "LODCN2"):
            u = lod_step(u, pb, dt, alpha, scheme)
        elif scheme.startswith("MAOS"):
            u = maos_step(u, pb, dt, alpha, scheme)
        elif scheme == "EULER":
            u = euler_step(u, pb, dt, alpha)
        else:
            u = aos_step(u, pb, dt, alpha, scheme)
    return u


def energy(pb: Problem, u: np.ndarray) -> float:
    """(1/2) sum Q phi with phi = kT u (Eq. (deltaG), one medium), kcal/mol."""
    return 0.5 * float(np.sum(pb.Q * (thermal_energy(pb.T) * u)))


def richardson(u_dt: np.ndarray, u_half: np.ndarray) -> np.ndarray:
    """Eq. (rich): 2 phi^{dt/2} - phi^{dt}, pointwise."""
    return 2.0 * u_half - u_dt


# ---------------------------------------------------------------------------
# the vacuum potential without pseudo-time (Sec. 5.1, text after Eq. (deltaG))

def poisson_direct(pb: Problem) -> np.ndarray:
    """phi_0 from the Poisson equation with a constant dielectric, solved
    directly: -eps delta^2 u = rho on the interior nodes (the operator of
    Eq. (SpatialOperators) summed over x, y, z, eps constant), u = u0 (the
    Dirichlet data) on the shell.  The Dirichlet couplings move to the
    right-hand side; the type-I discrete sine transform along each axis
    diagonalises what remains (eigenvalue of mode m on an axis with N
    interior nodes: (eps/h^2) 4 sin^2(pi m / (2 (N + 1)))), which is the
    fast-transform Poisson solver the paper uses for phi_0."""
    e = float(pb.eps_node.flat[0])
    if not np.all(pb.eps_node == e):
        raise ValueError("the direct Poisson solve needs a uniform dielectric")
    h = pb.grid.h
    g = pb.u0
    c = e / (h * h)
    f = pb.rho[1:-1, 1:-1, 1:-1].copy()
    f[0, :, :] += c * g[0, 1:-1, 1:-1]
    f[-1, :, :] += c * g[-1, 1:-1, 1:-1]
    f[:, 0, :] += c * g[1:-1, 0, 1:-1]
    f[:, -1, :] += c * g[1:-1, -1, 1:-1]
    f[:, :, 0] += c * g[1:-1, 1:-1, 0]
    f[:, :, -1] += c * g[1:-1, 1:-1, -1]

    def eig(N):
        return 4.0 * np.sin(np.pi * np.arange(1, N + 1) / (2.0 * (N + 1))) ** 2

    Nz, Ny, Nx = f.shape
    lam = c * (eig(Nz)[:, None, None] + eig(Ny)[None, :, None] + eig(Nx)[None, None, :])
    u = g.copy()
    u[1:-1, 1:-1, 1:-1] = idstn(dstn(f, type=1) / lam, type=1)
    return u


def solve(mol, grid, params, want_fields: bool = False, vacuum_direct: bool = False) -> dict:
    """Full solve as the C library defines it: solvated loop(s) and, if
    requested, the vacuum loop(s) by the same scheme (Eq. (deltaG3)), with
    Richardson extrapolation on each medium when requested (Eq. (rich)).
    Returns energies in kcal/mol:
      G_m[0], G_0[0]  : (1/2) sum Q phi at dt (n steps)
      G_m[1], G_0[1]  : the same at dt/2 (2n steps), only with Richardson
      dG_plain        : (1/2) sum Q (phi_m - phi_0) at dt
      dG              : the same from the Richardson-combined potentials
                        (equal to dG_plain without Richardson).
    With vacuum_direct also (params.vacuum may be off: the direct solve is
    then the only vacuum problem):
      dG_direct       : (1/2) sum Q (phi_m - phi_0^FFT), Eq. (deltaG2), with
                        phi_m Richardson-combined when Richardson is on and
                        phi_0^FFT from poisson_direct
      (fields) phi_0_direct = kT u_0^FFT, phi_rec = phi_m - phi_0 + phi_0^FFT"""
    T = params.temperature_K
    kT = thermal_energy(T)
    out = {"G_m": [0.0, 0.0], "G_0": [0.0, 0.0]}
    levels = [(params.dt, params.n_steps)]
    if params.richardson:
        levels.append((params.dt / 2.0, 2 * params.n_steps))
    media = ["solvated"] + (["vacuum"] if params.vacuum else [])
    fields = {}
    for medium in media:
        pb = make_problem(mol, grid, params, medium)
        us = []
        for li, (dt, ns) in enumerate(levels):
            u = run(pb, dt, params.alpha, ns, params.scheme)
            us.append(u)
            key = "G_m" if medium == "solvated" else "G_0"
            out[key][li] = energy(pb, u)
        u_fin = richardson(us[0], us[1]) if params.richardson else us[0]
        fields[medium] = (us, u_fin)
        Qc = pb.Q
    if params.vacuum:
        um0 = fields["solvated"][0][0]
        uv0 = fields["vacuum"][0][0]
        out["dG_plain"] = 0.5 * float(np.sum(Qc * (kT * um0 - kT * uv0)))
        umf = fields["solvated"][1]
        uvf = fields["vacuum"][1]
        out["dG"] = 0.5 * float(np.sum(Qc * (kT * umf - kT * uvf)))
    else:
        out["dG_plain"] = float("nan")
        out["dG"] = float("nan")
    if vacuum_direct:
        u_dir = poisson_direct(make_problem(mol, grid, params, "vacuum"))
        umf = fields["solvated"][1]
        out["dG_direct"] = 0.5 * float(np.sum(Qc * (kT * umf - kT * u_dir)))
        if want_fields:
            out["phi_0_direct"] = kT * u_dir
            if params.vacuum:
                out["phi_rec"] = kT * umf - kT * fields["vacuum"][1] + kT * u_dir
    if want_fields:
        out["phi_m"] = kT * fields["solvated"][1]
        out["u_m_levels"] = fields["solvated"][0]
        if params.vacuum:
            out["phi_0"] = kT * fields["vacuum"][1]
            out["u_0_levels"] = fields["vacuum"][0]
        out["Q"] = Qc
    return out
