"""Pins of the FP64 oracle against the paper and the mathematics (CPU only).

Each test checks the oracle against something other than itself: values
the paper prints (tests/golden), closed forms, brute-force dense solves on
tiny grids, library routines, invariants and convergence orders.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_1410_2788_amd import inputs
from tests import _dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
N_AVOGADRO = 6.02214076e23


def _params(**kw):
    base = dict(eps_in=2.0, eps_out=80.0, ionic_molar=0.0, temperature_K=298.0,
                alpha=1.0, dt=0.05, n_steps=10, scheme="LODIE2", richardson=False,
                vacuum=True, precision="f64")
    base.update(kw)
    return inputs.RunParams(**base)


def _tiny(n=9, h=0.5, ny=None, nz=None):
    return inputs.cubic_grid(n, h, ny=ny, nz=nz)


def _two_atoms():
    return inputs.Molecule(xyz=np.array([[0.13, -0.21, 0.07], [-0.4, 0.35, 0.3]]),
                           q=np.array([1.0, -0.6]), radius=np.array([1.1, 0.8]))


# --------------------------------------------------------------------------
# constants (Sec. 2.1)

def test_constants_match_paper():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert oracle.thermal_energy(298.0) == pytest.approx(g["kT_298_kcal_per_mol"], rel=1e-15)
    # Gaussian-unit identity kbar^2 = 8 pi l_B N_A I / (1000 cm^3 -> A^3):
    lB = oracle.bjerrum_length(298.0)
    kb2_from_lB = 8.0 * math.pi * lB * N_AVOGADRO * 1e-27
    assert kb2_from_lB == pytest.approx(g["kbar2_per_molar_298_inv_A2"], rel=2e-5)
    assert oracle.kappa_bar_sq(1.0, 298.0) == pytest.approx(g["kbar2_per_molar_298_inv_A2"], rel=1e-15)
    # the protein runs: 300 K constant times 9.48955 M is 80 A^-2
    assert oracle.kappa_bar_sq(g["ionic_strength_proteins_molar"], 300.0) == pytest.approx(80.0, rel=1e-4)


# --------------------------------------------------------------------------
# solute mask

def test_mask_matches_brute_force_including_on_sphere_nodes():
    grid = inputs.cubic_grid(17, 0.25)
    rng = np.random.default_rng(11)
    xyz = rng.uniform(-1.2, 1.2, (6, 3))
    xyz[0] = [0.0, 0.0, 0.0]            # a node: nodes at distance exactly R
    xyz[1] = [0.25, -0.5, 0.75]
    rad = rng.uniform(0.3, 0.9, 6)
    rad[0] = 0.5
    rad[1] = 0.75
    M = oracle.solute_mask(grid, xyz, rad)
    X, Y, Z = (oracle.axis_coords(grid, d) for d in range(3))
    B = np.zeros_like(M)
    for k in range(grid.nz):
        for j in range(grid.ny):
            for i in range(grid.nx):
                for a in range(xyz.shape[0]):
                    dx = X[i] - xyz[a, 0]
                    dy = Y[j] - xyz[a, 1]
                    dz = Z[k] - xyz[a, 2]
                    if dx * dx + dy * dy + dz * dz <= rad[a] * rad[a]:
                        B[k, j, i] = True
                        break
    assert np.array_equal(M, B)
    # the node at distance exactly 0.5 from atom 0 is solute ("on" counts)
    assert M[8, 8, 10] and M[8, 10, 8] and M[10, 8, 8]


def test_mask_volume_of_a_large_sphere():
    grid = inputs.cubic_grid(41, 0.25)
    M = oracle.solute_mask(grid, np.array([[0.01, 0.02, 0.03]]), np.array([4.0]))
    vol = M.sum() * 0.25 ** 3
    assert vol == pytest.approx(4.0 / 3.0 * math.pi * 4.0 ** 3, rel=0.02)


# --------------------------------------------------------------------------
# trilinear charges

def test_charge_spreading_preserves_charge_and_dipole():
    grid = inputs.cubic_grid(21, 0.5)
    rng = np.random.default_rng(5)
    xyz = rng.uniform(-3.0, 3.0, (40, 3))
    q = rng.normal(0, 0.5, 40)
    Q = oracle.spread_charges(grid, xyz, q)
    assert Q.sum() == pytest.approx(q.sum(), abs=1e-12)
    X, Y, Z = (oracle.axis_coords(grid, d) for d in range(3))
    dip = np.array([(Q * X[None, None, :]).sum(), (Q * Y[None, :, None]).sum(),
                    (Q * Z[:, None, None]).sum()])
    assert np.allclose(dip, (q[:, None] * xyz).sum(axis=0), atol=1e-11)
    assert np.count_nonzero(Q) <= 8 * 40


def test_node_centred_charge_lands_on_one_node():
    grid = inputs.cubic_grid(9, 0.5)
    Q = oracle.spread_charges(grid, np.array([[0.5, -1.0, 0.0]]), np.array([2.5]))
    assert np.count_nonzero(Q) == 1
    assert Q[4, 2, 5] == 2.5


def test_charge_stencil_touching_boundary_is_an_error():
    grid = inputs.cubic_grid(9, 0.5)
    with pytest.raises(oracle.ChargeStencilError):
        oracle.spread_charges(grid, np.array([[1.7, 0.0, 0.0]]), np.array([1.0]))


# --------------------------------------------------------------------------
# boundary data (Eq. (BoundaryCond))

def _point_potential(P, xyz, q, eps, kb2, T=298.0):
    """Evaluate the boundary formula at an arbitrary point through a 1x1x1
    grid (its only node lies on the shell)."""
    g = inputs.Grid(nx=1, ny=1, nz=1, h=1.0, origin=list(P))
    return oracle.boundary_potential(g, xyz, q, eps, kb2, T)[0, 0, 0]


@pytest.mark.parametrize("kb2", [0.0, 1.27, 4.24])
def test_boundary_potential_solves_linearised_pb_away_from_charges(kb2):
    # eps_s Laplace(u) - kbar^2 u = 0 away from the charges (Debye-Hueckel).
    xyz = np.array([[0.3, -0.2, 0.1], [-0.5, 0.4, 0.2]])
    q = np.array([1.0, -0.4])
    eps = 80.0
    P = np.array([2.0, 1.5, -1.0])
    d = 1e-2
    u0 = _point_potential(P, xyz, q, eps, kb2)
    lap = 0.0
    for ax in range(3):
        for s in (-1, 1):
            Pn = P.copy()
            Pn[ax] += s * d
            lap += _point_potential(Pn, xyz, q, eps, kb2)
    lap = (lap - 6 * u0) / d ** 2
    resid = eps * lap - kb2 * u0
    scale = eps * abs(u0) + kb2 * abs(u0) + 1e-30
    assert abs(resid) < 1e-3 * scale + 1e-9


def test_boundary_potential_coulomb_limit_and_superposition():
    lB = oracle.bjerrum_length(298.0)
    x1 = np.array([[0.0, 0.0, 0.0]])
    P = np.array([3.0, 4.0, 0.0])      # d = 5
    assert _point_potential(P, x1, np.array([1.0]), 2.0, 0.0) == pytest.approx(lB / (2.0 * 5.0), rel=1e-14)
    xyz = _two_atoms().xyz
    q = _two_atoms().q
    both = _point_potential(P, xyz, q, 80.0, 1.3)
    one = _point_potential(P, xyz[:1], q[:1], 80.0, 1.3) + _point_potential(P, xyz[1:], q[1:], 80.0, 1.3)
    assert both == pytest.approx(one, rel=1e-14)
    # screening lowers the magnitude
    assert abs(_point_potential(P, x1, np.array([1.0]), 80.0, 1.3)) < abs(_point_potential(P, x1, np.array([1.0]), 80.0, 0.0))


# --------------------------------------------------------------------------
# one implicit sweep

def _random_eps(shape, seed):
    rng = np.random.default_rng(seed)
    return np.where(rng.random(shape) < 0.4, 2.0, 80.0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sweep_matches_dense_solve(axis):
    grid = inputs.cubic_grid(7, 0.5, ny=8, nz=9)
    shape = oracle.shape_zyx(grid)
    eps = _random_eps(shape, 3 + axis)
    rng = np.random.default_rng(axis)
    s = rng.normal(0, 10, shape)
    tau = 0.37
    v = oracle.implicit_sweep(s, eps, tau, grid.h, axis)
    D = _dense.dense_second_difference(eps, grid.h, axis)
    A = np.eye(s.size) - tau * D
    vd = np.linalg.solve(A, s.ravel()).reshape(shape)
    assert np.max(np.abs(v - vd)) <= 1e-12 * np.max(np.abs(vd))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sweep_keeps_constant_flux_profiles(axis):
    # e_{i+1/2} (v_{i+1} - v_i) = F on every line => delta^2 v = 0.
    n = 12
    grid = inputs.cubic_grid(n, 0.5)
    shape = oracle.shape_zyx(grid)
    # eps depends on the sweep coordinate only, so every line is alike
    e1 = np.where(np.arange(n) % 3 == 0, 2.0, 80.0)
    ebc = [1] * 3
    ebc[axis] = n
    eps = np.broadcast_to(e1.reshape(ebc), shape).copy()
    ef = 2 * e1[:-1] * e1[1:] / (e1[:-1] + e1[1:])
    prof = np.concatenate([[1.0], 1.0 + np.cumsum(3.0 / ef)])
    s = np.broadcast_to(prof.reshape(ebc), shape).copy()
    v = oracle.implicit_sweep(s, eps, 5.0, grid.h, axis)
    assert np.max(np.abs(v - s)) < 1e-11 * np.max(np.abs(s))


def test_sweep_constant_fixed_point_and_maximum_principle():
    grid = inputs.cubic_grid(10, 0.5)
    shape = oracle.shape_zyx(grid)
    eps = _random_eps(shape, 1)
    c = np.full(shape, 3.25)
    for ax in range(3):
        assert np.max(np.abs(oracle.implicit_sweep(c, eps, 2.0, grid.h, ax) - 3.25)) < 1e-13
    rng = np.random.default_rng(2)
    s = rng.normal(0, 1, shape)
    v = oracle.implicit_sweep(s, eps, 2.0, grid.h, 2)
    lo = s.min(axis=2, keepdims=True)
    hi = s.max(axis=2, keepdims=True)
    assert np.all(v >= lo - 1e-12) and np.all(v <= hi + 1e-12)


def test_sweep_single_line_matches_banded_library_solver():
    n = 30
    grid = inputs.Grid(nx=n, ny=3, nz=3, h=0.4, origin=[0, 0, 0])
    shape = oracle.shape_zyx(grid)
    rng = np.random.default_rng(8)
    eps = np.where(rng.random(shape) < 0.5, 4.0, 80.0)
    s = rng.normal(0, 5, shape)
    tau = 1.3
    v = oracle.implicit_sweep(s, eps, tau, grid.h, 2)
    e = eps[1, 1]
    ef = 2 * e[:-1] * e[1:] / (e[:-1] + e[1:])
    r = tau / grid.h ** 2
    m = n - 2
    ab = np.zeros((3, m))
    ab[0, 1:] = -r * ef[1:m]
    ab[1, :] = 1 + r * (ef[0:m] + ef[1:m + 1])
    ab[2, :-1] = -r * ef[1:m]
    rhs = s[1, 1, 1:-1].copy()
    rhs[0] += r * ef[0] * s[1, 1, 0]
    rhs[-1] += r * ef[m] * s[1, 1, -1]
    x = scipy.linalg.solve_banded((1, 1), ab, rhs)
    assert np.allclose(v[1, 1, 1:-1], x, rtol=1e-13, atol=1e-13)


# --------------------------------------------------------------------------
# nonlinear sub-step (Eqs. (ana1)-(ana3))

def _N(u, theta):
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    th = np.full(u.shape, theta)
    return oracle.nonlinear_substep(u, th, np.ones(u.shape, dtype=bool))


@pytest.mark.parametrize("theta", [1e-4, 0.05, 0.7, 3.0])
def test_nonlinear_closed_form_tanh(theta):
    # integral of dw / sinh w = ln |tanh(w/2)|  =>  tanh(w1/2) = e^{-2 theta} tanh(w0/2)
    u = np.concatenate([np.linspace(-30, 30, 241), [-5000.0, -800.0, 800.0, 5000.0]])
    w = _N(u, theta)
    ref = 2.0 * np.arctanh(np.exp(-2 * theta) * np.tanh(u / 2))
    assert np.allclose(w, ref, rtol=1e-11, atol=1e-12)


def test_nonlinear_matches_rk4_of_the_ode():
    kb2, alpha, dt = 1.7, 0.5, 0.2
    theta = kb2 * dt / (2 * alpha)
    for u0 in (-4.0, -0.7, 0.3, 2.5, 5.0):
        w = u0
        n = 20000
        hstep = dt / n
        f = lambda y: -kb2 / alpha * math.sinh(y)
        for _ in range(n):
            k1 = f(w)
            k2 = f(w + 0.5 * hstep * k1)
            k3 = f(w + 0.5 * hstep * k2)
            k4 = f(w + hstep * k3)
            w += hstep / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        assert _N(u0, theta)[0] == pytest.approx(w, rel=1e-10, abs=1e-12)


def test_nonlinear_semigroup_symmetry_identity():
    u = np.linspace(-12, 12, 97)
    a, b = 0.3, 1.1
    assert np.allclose(_N(_N(u, a), b), _N(u, a + b), rtol=1e-12, atol=1e-13)
    assert np.allclose(_N(-u, a), -_N(u, a), rtol=1e-13, atol=1e-14)
    assert _N(0.0, 2.0)[0] == 0.0
    z = oracle.nonlinear_substep(u, np.zeros_like(u), np.ones_like(u, dtype=bool))
    assert np.array_equal(z, u)
    th = 1e-6
    assert np.allclose(_N(u[:40] / 4, th), u[:40] / 4 - 2 * th * np.sinh(u[:40] / 4), rtol=1e-9, atol=1e-12)


def test_nonlinear_leaves_boundary_shell_alone():
    u = np.full((5, 5, 5), 3.0)
    th = np.full(u.shape, 0.5)
    interior = np.zeros(u.shape, dtype=bool)
    interior[1:-1, 1:-1, 1:-1] = True
    w = oracle.nonlinear_substep(u, th, interior)
    assert np.all(w[~interior] == 3.0) and np.all(w[interior] < 3.0)


# --------------------------------------------------------------------------
# whole steps: fixed points against dense solves (kbar = 0)

def _step_map_dense(pb, dt, alpha, scheme):
    """Affine step map u -> M u + c assembled from dense matrices."""
    tau = dt / alpha
    h = pb.grid.h
    N = pb.u0.size
    Ds = [_dense.dense_second_difference(pb.eps_node, h, ax, pb.face(ax))
          for ax in (2, 1, 0)]  # x, y, z
    rho = pb.rho.ravel()
    if scheme in ("LODIE2", "LODIE1"):
        A = [np.eye(N) - tau * D for D in Ds]
        Minv = np.linalg.solve(A[2], np.linalg.solve(A[1], np.linalg.solve(A[0], np.eye(N))))
        if scheme == "LODIE2":
            return Minv, Minv @ (tau * rho)
        return Minv, tau * rho
    if scheme in ("LODCN2", "LODCN1"):
        # (I - tau/2 D_d)^-1 (I + tau/2 D_d) per direction, x then y then z
        Minv = np.eye(N)
        for D in Ds:
            Minv = np.linalg.solve(np.eye(N) - 0.5 * tau * D, (np.eye(N) + 0.5 * tau * D) @ Minv)
        if scheme == "LODCN2":
            return Minv, Minv @ (tau * rho)
        return Minv, tau * rho
    if scheme in ("MAOSIE", "MAOSCN"):
        # kbar = 0: the flow is the identity; mean of three directional solves
        M = np.zeros((N, N))
        cv = np.zeros(N)
        for D in Ds:
            if scheme == "MAOSIE":
                Bi = np.linalg.inv(np.eye(N) - 3 * tau * D)
                E = np.eye(N)
            else:
                Bi = np.linalg.inv(np.eye(N) - 1.5 * tau * D)
                E = np.eye(N) + 1.5 * tau * D
            M += Bi @ E / 3.0
            cv += Bi @ (tau * rho) / 3.0
        return M, cv
    c = {"AOSIE1": (4.0, 0.0, 0.0), "AOSIE2": (4.0 / 3, 4.0 / 3, 4.0 / 3),
         "AOSCN1": (4.0, 0.0, 0.0), "AOSCN2": (4.0 / 3, 4.0 / 3, 4.0 / 3)}[scheme]
    M = np.eye(N) * 0.25
    cv = np.zeros(N)
    for D, cd in zip(Ds, c):
        if scheme.startswith("AOSIE"):
            Bi = np.linalg.inv(np.eye(N) - 4 * tau * D)
            E = np.eye(N)
        else:
            Bi = np.linalg.inv(np.eye(N) - 2 * tau * D)
            E = np.eye(N) + 2 * tau * D
        M += 0.25 * Bi @ E
        cv += 0.25 * Bi @ (cd * tau * rho)
    return M, cv


@pytest.mark.parametrize("scheme", ["LODIE2", "LODIE1", "AOSIE2", "AOSIE1", "LODCN1", "LODCN2",
                                    "AOSCN1", "AOSCN2", "MAOSIE", "MAOSCN"])
def test_linear_fixed_point_matches_dense_solve(scheme):
    grid = _tiny(9, 0.5)
    mol = _two_atoms()
    p = _params(scheme=scheme, ionic_molar=0.0, dt=0.1, alpha=1.0)
    pb = oracle.make_problem(mol, grid, p, "solvated")
    # MAOSCN: the stiffest modes decay by ~0.99 per step (Crank-Nicolson
    # factors near -1 in all three directions at once)
    u = oracle.run(pb, p.dt, p.alpha, 8000 if scheme == "MAOSCN" else 600, scheme)
    M, c = _step_map_dense(pb, p.dt, p.alpha, scheme)
    ud = _dense.affine_fixed_point(M, c, pb.u0.ravel(), _dense.interior_flags(pb.u0.shape))
    assert np.max(np.abs(u.ravel() - ud)) <= 1e-10 * np.max(np.abs(ud))


@pytest.mark.parametrize("scheme", ["LODIE2", "LODIE1", "AOSIE2", "LODCN1", "LODCN2", "AOSCN1",
                                    "AOSCN2", "MAOSIE", "MAOSCN"])
def test_one_step_matches_dense_map(scheme):
    grid = _tiny(8, 0.5, ny=9, nz=7)
    mol = _two_atoms()
    p = _params(scheme=scheme, ionic_molar=0.0, dt=0.7, alpha=0.5)
    pb = oracle.make_problem(mol, grid, p, "solvated")
    rng = np.random.default_rng(4)
    u = pb.u0.copy()
    u[1:-1, 1:-1, 1:-1] = rng.normal(0, 20, (5, 7, 6))
    u1 = oracle.run(pb, p.dt, p.alpha, 1, scheme, u_init=u)
    M, c = _step_map_dense(pb, p.dt, p.alpha, scheme)
    ud = M @ u.ravel() + c
    assert np.max(np.abs(u1.ravel() - ud)) <= 1e-11 * np.max(np.abs(ud))


def _steady(pb, dt, alpha, scheme, tol=1e-13, max_steps=20000):
    u = pb.u0.copy()
    for n in range(max_steps):
        un = oracle.run(pb, dt, alpha, 1, scheme, u_init=u)
        if np.max(np.abs(un - u)) < tol * np.max(np.abs(un)):
            return un
        u = un
    raise AssertionError("no steady state")


def test_lod_steady_state_converges_to_poisson_first_order_and_richardson_second():
    grid = _tiny(9, 0.5)
    mol = _two_atoms()
    p = _params(ionic_molar=0.0)
    pb = oracle.make_problem(mol, grid, p, "solvated")
    D = sum(_dense.dense_second_difference(pb.eps_node, grid.h, ax) for ax in range(3))
    I = _dense.interior_flags(pb.u0.shape)
    # discrete Poisson: -D u = rho inside, u = g on the shell
    ex = _dense.newton_npb(D, np.zeros(pb.u0.size), pb.rho.ravel(), pb.u0.ravel(), I)
    errs, sols = [], []
    for tau in (0.04, 0.02, 0.01):
        u = _steady(pb, tau, 1.0, "LODIE2")
        sols.append(u.ravel())
        errs.append(np.max(np.abs(u.ravel() - ex)))
    r1 = errs[0] / errs[1]
    r2 = errs[1] / errs[2]
    assert 1.7 < r1 < 2.4 and 1.7 < r2 < 2.4
    re1 = np.max(np.abs(oracle.richardson(sols[0], sols[1]) - ex))
    re2 = np.max(np.abs(oracle.richardson(sols[1], sols[2]) - ex))
    assert re1 < errs[1] / 3 and 3.0 < re1 / re2 < 5.0


@pytest.mark.parametrize("scheme", ["LODIE2", "LODIE1", "AOSIE2", "LODCN2", "AOSCN2", "MAOSIE"])
def test_nonlinear_steady_state_converges_to_discrete_npb(scheme):
    grid = _tiny(9, 0.5)
    mol = _two_atoms()
    p = _params(ionic_molar=2.0, eps_in=2.0, eps_out=20.0, scheme=scheme)
    pb = oracle.make_problem(mol, grid, p, "solvated")
    D = sum(_dense.dense_second_difference(pb.eps_node, grid.h, ax) for ax in range(3))
    I = _dense.interior_flags(pb.u0.shape)
    ex = _dense.newton_npb(D, pb.kbar2_node.ravel(), pb.rho.ravel(), pb.u0.ravel(), I)
    assert np.max(np.abs(pb.kbar2_node.ravel() * np.sinh(ex))) > 1.0   # nonlinearity matters
    errs, sols = [], []
    for tau in (0.02, 0.01):
        u = _steady(pb, tau, 1.0, scheme)
        sols.append(u.ravel())
        errs.append(np.max(np.abs(u.ravel() - ex)))
    assert 1.6 < errs[0] / errs[1] < 2.5
    re = np.max(np.abs(oracle.richardson(sols[0], sols[1]) - ex))
    assert re < 0.5 * errs[1]


# --------------------------------------------------------------------------
# the face rule by location (Sec. 3.1, text after Eq. (SpatialOperators))

def _three_atoms():
    return inputs.Molecule(xyz=np.array([[0.13, -0.21, 0.07], [-0.4, 0.35, 0.3],
                                         [0.61, 0.5, -0.45]]),
                           q=np.array([1.0, -0.6, 0.3]), radius=np.array([1.1, 0.8, 0.55]))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_face_solute_matches_brute_force(axis):
    grid = inputs.Grid(9, 8, 10, 0.3, (-1.3, -1.1, -1.45))
    mol = _three_atoms()
    F = oracle.face_solute(grid, mol.xyz, mol.radius, axis)
    n = [grid.nx, grid.ny, grid.nz]
    m = list(n)
    m[axis] -= 1
    assert F.shape == (m[2], m[1], m[0])
    for k in range(m[2]):
        for j in range(m[1]):
            for i in range(m[0]):
                idx = [i, j, k]
                p = [grid.origin[d] + float(idx[d]) * grid.h for d in range(3)]
                p[axis] = grid.origin[axis] + (float(idx[axis]) + 0.5) * grid.h
                inside = False
                for a in range(mol.xyz.shape[0]):
                    dx, dy, dz = (p[d] - mol.xyz[a, d] for d in range(3))
                    inside = inside or ((dx * dx + dy * dy) + dz * dz <= mol.radius[a] ** 2)
                assert F[k, j, i] == inside, (axis, i, j, k)
    assert F.any() and not F.all()


def _location_problem(grid, mol, **kw):
    p = _params(face_rule="location", **kw)
    pb = oracle.make_problem(mol, grid, p, "solvated")
    assert pb.faces is not None
    return p, pb


def test_location_faces_take_only_the_two_media_values_and_differ_from_harmonic():
    grid = _tiny(11, 0.35)
    mol = _three_atoms()
    p, pb = _location_problem(grid, mol)
    for ax in range(3):
        f = pb.faces[ax]
        assert set(np.unique(f)) <= {p.eps_in, p.eps_out}
        hm = oracle.face_eps(pb.eps_node, ax)
        same = (pb.eps_node.take(range(f.shape[ax]), axis=ax) ==
                pb.eps_node.take(range(1, f.shape[ax] + 1), axis=ax))
        # between two nodes of one medium both rules mostly agree; across
        # the surface the location rule never gives the harmonic value
        assert np.mean(f[same] == hm[same]) > 0.9
        assert not np.any(f[~same] == hm[~same])


def test_location_faces_euler_steady_state_is_the_dense_poisson_solution():
    grid = _tiny(9, 0.35, ny=8, nz=10)
    mol = _three_atoms()
    p, pb = _location_problem(grid, mol)
    D = sum(_dense.dense_second_difference(pb.eps_node, grid.h, ax, pb.faces[ax])
            for ax in range(3))
    I = _dense.interior_flags(pb.u0.shape)
    # linear: -D u = rho on the interior, u = g on the shell
    g = pb.u0.ravel()
    ex = g.copy()
    ex[I] = np.linalg.solve(-D[np.ix_(I, I)], pb.rho.ravel()[I] + D[np.ix_(I, ~I)] @ g[~I])
    u, n = _euler_steady(pb, _euler_tau(pb))
    assert np.max(np.abs(u.ravel() - ex)) <= 1e-10 * np.max(np.abs(ex))


@pytest.mark.parametrize("scheme", ["LODIE2", "AOSIE2", "LODCN2", "MAOSCN"])
def test_location_faces_one_step_matches_dense_map(scheme):
    grid = _tiny(8, 0.35, ny=9, nz=7)
    mol = _three_atoms()
    p, pb = _location_problem(grid, mol, scheme=scheme, dt=0.7, alpha=0.5)
    rng = np.random.default_rng(6)
    u = pb.u0.copy()
    u[1:-1, 1:-1, 1:-1] = rng.normal(0, 20, (5, 7, 6))
    u1 = oracle.run(pb, p.dt, p.alpha, 1, scheme, u_init=u)
    M, c = _step_map_dense(pb, p.dt, p.alpha, scheme)
    ud = M @ u.ravel() + c
    assert np.max(np.abs(u1.ravel() - ud)) <= 1e-11 * np.max(np.abs(ud))


# --------------------------------------------------------------------------
# explicit Euler (the reference solver of Sec. 5.2 and Sec. 5.4)

def test_euler_step_matches_a_node_by_node_operator():
    # brute force: every interior node's six neighbours, harmonic faces and
    # the sinh term written out with Python loops on a ragged tiny grid
    grid = _tiny(7, 0.4, ny=6, nz=8)
    mol = _two_atoms()
    p = _params(ionic_molar=1.5, eps_in=2.0, eps_out=30.0, dt=0.003, alpha=0.5)
    pb = oracle.make_problem(mol, grid, p, "solvated")
    rng = np.random.default_rng(9)
    u = pb.u0.copy()
    u[1:-1, 1:-1, 1:-1] = rng.normal(0, 1.5, (6, 4, 5))
    got = oracle.euler_step(u, pb, p.dt, p.alpha)
    tau, h = p.dt / p.alpha, grid.h
    e = pb.eps_node
    want = u.copy()
    nz, ny, nx = u.shape
    for k in range(1, nz - 1):
        for j in range(1, ny - 1):
            for i in range(1, nx - 1):
                acc = 0.0
                for dk, dj, di in ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0),
                                   (-1, 0, 0)):
                    en = e[k + dk, j + dj, i + di]
                    ef = 2.0 * e[k, j, i] * en / (e[k, j, i] + en)
                    acc += ef * (u[k + dk, j + dj, i + di] - u[k, j, i]) / (h * h)
                acc -= pb.kbar2_node[k, j, i] * math.sinh(u[k, j, i])
                acc += pb.rho[k, j, i]
                want[k, j, i] = u[k, j, i] + tau * acc
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    assert np.array_equal(got[~pb.interior], u[~pb.interior])


def _euler_steady(pb, tau, tol=1e-13, max_steps=40000):
    u = pb.u0.copy()
    for n in range(max_steps):
        un = oracle.euler_step(u, pb, tau, 1.0)
        if np.max(np.abs(un - u)) < tol * np.max(np.abs(un)):
            return un, n + 1
        u = un
    raise AssertionError("no steady state")


def _euler_tau(pb):
    # 0.9 of the explicit limit 2 / lambda_max, lambda_max <= 2 * sum of a
    # node's six face coefficients (Gershgorin)
    return 0.9 * 2.0 / (2.0 * 6.0 * float(np.max(pb.eps_node)) / pb.grid.h ** 2)


def test_euler_steady_state_is_the_direct_poisson_solution():
    # uniform eps, kbar = 0: no splitting error, so the Euler fixed point is
    # the discrete Poisson solution of the sine-transform solve itself
    grid = _tiny(11, 0.5, ny=9, nz=10)
    mol = _two_atoms()
    pb = oracle.make_problem(mol, grid, _params(), "vacuum")
    u, n = _euler_steady(pb, _euler_tau(pb))
    ex = oracle.poisson_direct(pb)
    assert np.max(np.abs(u - ex)) <= 1e-11 * np.max(np.abs(ex))


def test_euler_steady_state_is_the_discrete_npb_solution():
    # nonlinear, discontinuous eps: the Euler fixed point solves the discrete
    # NPB equations exactly (dense Newton), unlike the split schemes whose
    # steady states carry an O(dt) splitting error
    grid = _tiny(9, 0.5)
    mol = _two_atoms()
    p = _params(ionic_molar=2.0, eps_in=2.0, eps_out=20.0)
    pb = oracle.make_problem(mol, grid, p, "solvated")
    D = sum(_dense.dense_second_difference(pb.eps_node, grid.h, ax) for ax in range(3))
    I = _dense.interior_flags(pb.u0.shape)
    ex = _dense.newton_npb(D, pb.kbar2_node.ravel(), pb.rho.ravel(), pb.u0.ravel(), I)
    assert np.max(np.abs(pb.kbar2_node.ravel() * np.sinh(ex))) > 1.0
    # linearised limit: the sinh term adds up to kbar^2 cosh(u) to lambda_max
    lam = 2.0 * 6.0 * float(np.max(pb.eps_node)) / grid.h ** 2
    lam += float(np.max(pb.kbar2_node.ravel() * np.cosh(ex)))
    u, n = _euler_steady(pb, 0.9 * 2.0 / lam)
    assert np.max(np.abs(u.ravel() - ex)) <= 1e-10 * np.max(np.abs(ex))


def test_euler_is_unstable_just_above_the_explicit_limit():
    # uniform eps: lambda_max of the 7-point operator is known exactly, so
    # tau 2 % below 2 / lambda_max stays bounded and 2 % above grows
    grid = _tiny(9, 0.5)
    mol = _two_atoms()
    pb = oracle.make_problem(mol, grid, _params(), "vacuum")
    e, h, N = pb.eps_node.flat[0], grid.h, 7
    lam_max = 3 * (e / h ** 2) * 4.0 * math.sin(math.pi * N / (2.0 * (N + 1))) ** 2
    rng = np.random.default_rng(2)
    u0 = pb.u0.copy()
    u0[1:-1, 1:-1, 1:-1] += rng.normal(0, 1.0, (N, N, N))
    ex = oracle.poisson_direct(pb)
    dev0 = np.max(np.abs(u0 - ex))
    amp = {}
    for f in (0.98, 1.02):
        u = u0.copy()
        for _ in range(3000):
            u = oracle.euler_step(u, pb, f * 2.0 / lam_max, 1.0)
        amp[f] = np.max(np.abs(u - ex)) / dev0
    assert amp[0.98] < 1.0 and amp[1.02] > 1e6


# --------------------------------------------------------------------------
# source prefactor and energy

def test_vacuum_potential_approaches_coulomb_away_from_the_charge():
    # discrete Poisson solution of a unit charge in eps_in: compare with
    # l_B / (eps d) at nodes a few cells away (Eq. (RhoEq) prefactor).
    grid = inputs.cubic_grid(17, 0.5)
    mol = inputs.single_ion(1.0, 1.0)
    p = _params(eps_in=2.0, ionic_molar=0.0)
    pb = oracle.make_problem(mol, grid, p, "vacuum")
    u = _steady(pb, 0.02, 1.0, "LODIE2", tol=1e-12)
    u = oracle.richardson(_steady(pb, 0.04, 1.0, "LODIE2", tol=1e-12), u)
    lB = oracle.bjerrum_length(298.0)
    for (k, j, i) in [(8, 8, 12), (8, 11, 11), (5, 8, 8), (11, 11, 11)]:
        d = 0.5 * math.sqrt((i - 8) ** 2 + (j - 8) ** 2 + (k - 8) ** 2)
        assert u[k, j, i] == pytest.approx(lB / (2.0 * d), rel=0.05)


def test_uniform_medium_gives_exactly_zero_solvation_energy():
    w = inputs.small_globular(n_atoms=30, n=25, n_steps=3, richardson=True,
                              eps_in=4.0, eps_out=4.0, ionic_molar=0.0)
    r = oracle.solve(w.molecule, w.grid, w.params)
    assert r["dG"] == 0.0 and r["dG_plain"] == 0.0
    assert r["G_m"] == r["G_0"]


def test_linear_energy_scales_with_charge_squared():
    w = inputs.small_globular(n_atoms=30, n=25, n_steps=3, richardson=True, ionic_molar=0.0)
    r1 = oracle.solve(w.molecule, w.grid, w.params)
    mol2 = inputs.Molecule(xyz=w.molecule.xyz, q=2.5 * w.molecule.q, radius=w.molecule.radius)
    r2 = oracle.solve(mol2, w.grid, w.params)
    assert r2["dG"] == pytest.approx(6.25 * r1["dG"], rel=1e-12)


def test_born_energy_from_steady_states_with_richardson_and_vacuum():
    # Born: dG = -(332.06371 / (2 a)) (1/eps_in - 1/eps_out) = -81.978 kcal/mol.
    # Both media iterated to their LODIE2 steady state at tau and tau/2,
    # Richardson-combined (Eq. (rich)), energy by Eq. (deltaG3).
    born = -(332.06371 / 4.0) * (1.0 - 1.0 / 80.0)
    errs = []
    for n, h in ((17, 0.5), (33, 0.25)):
        grid = inputs.cubic_grid(n, h)
        p = _params(eps_in=1.0, eps_out=80.0, ionic_molar=0.0)
        G = []
        for medium in ("solvated", "vacuum"):
            pb = oracle.make_problem(inputs.single_ion(1.0, 2.0), grid, p, medium)
            u1 = _steady(pb, 0.2, 1.0, "LODIE2", tol=1e-11)
            u2 = _steady(pb, 0.1, 1.0, "LODIE2", tol=1e-11)
            G.append(oracle.energy(pb, oracle.richardson(u1, u2)))
        errs.append(abs((G[0] - G[1]) - born) / abs(born))
    assert errs[0] < 0.06 and errs[1] < 0.02
    assert errs[1] < 0.5 * errs[0]


def test_born_solvated_potential_outside_the_sphere_is_screened_coulomb():
    grid = inputs.cubic_grid(17, 0.5)
    p = _params(eps_in=1.0, eps_out=80.0, ionic_molar=0.0)
    pb = oracle.make_problem(inputs.single_ion(1.0, 2.0), grid, p, "solvated")
    u = oracle.richardson(_steady(pb, 0.02, 1.0, "LODIE2", tol=1e-11),
                          _steady(pb, 0.01, 1.0, "LODIE2", tol=1e-11))
    lB = oracle.bjerrum_length(298.0)
    for (k, j, i) in [(8, 8, 14), (8, 14, 8), (2, 8, 8), (8, 13, 13)]:
        r = 0.5 * math.sqrt((i - 8) ** 2 + (j - 8) ** 2 + (k - 8) ** 2)
        assert u[k, j, i] == pytest.approx(lB / (80.0 * r), rel=0.05)


def test_mirror_symmetry_of_a_centred_ion():
    grid = inputs.cubic_grid(15, 0.5)
    p = _params(ionic_molar=0.5, eps_in=1.0, eps_out=80.0, dt=0.3, n_steps=4)
    pb = oracle.make_problem(inputs.single_ion(1.0, 1.5), grid, p, "solvated")
    u = oracle.run(pb, p.dt, p.alpha, p.n_steps, "LODIE2")
    m = np.max(np.abs(u))
    for ax in range(3):
        assert np.max(np.abs(u - np.flip(u, axis=ax))) < 1e-12 * m


# --------------------------------------------------------------------------
# vacuum potential by the direct (sine-transform) Poisson solve, Sec. 5.1;
# Eq. (deltaG2) and the recovered potential of Sec. 5.4

def _vacuum_problem(nx=8, ny=9, nz=7, eps_in=2.0):
    grid = _tiny(nx, 0.5, ny=ny, nz=nz)
    p = _params(eps_in=eps_in, ionic_molar=0.0)
    return oracle.make_problem(_two_atoms(), grid, p, "vacuum")


def test_direct_poisson_matches_dense_solve_with_arbitrary_boundary_data():
    # non-cubic grid and random data on every face: a swapped axis, a
    # dropped face or a wrong eigenvalue fails this
    import dataclasses
    pb = _vacuum_problem()
    rng = np.random.default_rng(21)
    g = pb.u0.copy()
    B = oracle.boundary_shell(pb.grid)
    g[B] = rng.normal(0.0, 50.0, int(B.sum()))
    pb = dataclasses.replace(pb, u0=g)
    D = sum(_dense.dense_second_difference(pb.eps_node, pb.grid.h, ax) for ax in range(3))
    I = _dense.interior_flags(g.shape)
    # -D u = rho on interior rows, u = g on the shell
    ex = g.ravel().copy()
    ex[I] = np.linalg.solve(-D[np.ix_(I, I)], pb.rho.ravel()[I] + D[np.ix_(I, ~I)] @ g.ravel()[~I])
    u = oracle.poisson_direct(pb)
    assert np.max(np.abs(u.ravel() - ex)) <= 1e-11 * np.max(np.abs(ex))
    assert np.array_equal(u[B], g[B])


def test_direct_poisson_reproduces_discrete_harmonic_functions():
    # x^2 - y^2 + 2 x z - 3 z + 1 has a zero 7-point Laplacian: with no
    # charge and these Dirichlet values the interior must equal it
    import dataclasses
    pb = _vacuum_problem(9, 7, 8)
    grid = pb.grid
    Z, Y, X = np.meshgrid(*(oracle.axis_coords(grid, d) for d in (2, 1, 0)), indexing="ij")
    f = X ** 2 - Y ** 2 + 2.0 * X * Z - 3.0 * Z + 1.0
    g = np.where(oracle.boundary_shell(grid), f, 0.0)
    pb = dataclasses.replace(pb, u0=g, rho=np.zeros_like(g))
    u = oracle.poisson_direct(pb)
    assert np.max(np.abs(u - f)) <= 1e-12 * np.max(np.abs(f))


def test_direct_poisson_is_the_small_step_limit_of_the_vacuum_lod_run():
    pb = _vacuum_problem(9, 9, 9)
    ex = oracle.poisson_direct(pb)
    errs, sols = [], []
    for tau in (0.04, 0.02, 0.01):
        u = _steady(pb, tau, 1.0, "LODIE2")
        sols.append(u)
        errs.append(np.max(np.abs(u - ex)))
    assert 1.7 < errs[0] / errs[1] < 2.4 and 1.7 < errs[1] / errs[2] < 2.4
    assert np.max(np.abs(oracle.richardson(sols[1], sols[2]) - ex)) < errs[2] / 3


def test_recovered_potential_reproduces_the_re_v_energy():
    # (1/2) sum Q (phi_rec - phi_0^FFT) = (1/2) sum Q (phi_m - phi_0^LOD):
    # the reading phi_m - phi_0^LOD + phi_0^FFT of the recovery formula
    w = inputs.small_globular(seed=5, n_atoms=30, n=25, n_steps=4, richardson=True)
    r = oracle.solve(w.molecule, w.grid, w.params, want_fields=True, vacuum_direct=True)
    lhs = 0.5 * float(np.sum(r["Q"] * (r["phi_rec"] - r["phi_0_direct"])))
    assert lhs == pytest.approx(r["dG"], rel=1e-11)
    d2 = 0.5 * float(np.sum(r["Q"] * (r["phi_m"] - r["phi_0_direct"])))
    assert r["dG_direct"] == pytest.approx(d2, rel=1e-12)
    # on the shell the recovered potential is the solvated Dirichlet data
    B = oracle.boundary_shell(w.grid)
    scale = np.max(np.abs(r["phi_0_direct"]))
    assert np.max(np.abs(r["phi_rec"][B] - r["phi_m"][B])) <= 1e-13 * scale


# --------------------------------------------------------------------------
# Crank-Nicolson sub-steps (Eqs. (LODCN1_2)-(LODCN1_4))

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_explicit_half_matches_dense_operator(axis):
    grid = _tiny(8, 0.5, ny=9, nz=7)
    p = _params(eps_in=2.0, eps_out=80.0)
    pb = oracle.make_problem(_two_atoms(), grid, p, "solvated")
    rng = np.random.default_rng(7 + axis)
    s = rng.normal(0.0, 10.0, pb.u0.shape)
    D = _dense.dense_second_difference(pb.eps_node, grid.h, axis)
    got = oracle.explicit_half(s, pb.eps_node, 0.3, grid.h, axis)
    ref = s.ravel() + 0.3 * (D @ s.ravel())
    assert np.max(np.abs(got.ravel() - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_cn_sweep_amplifies_an_eigenmode_by_the_crank_nicolson_factor():
    # constant eps, zero Dirichlet data: sin(pi m i / (n - 1)) along x is an
    # eigenvector of delta_x^2 with eigenvalue -(eps/h^2) 4 sin^2(pi m / (2 (n - 1)));
    # one sub-step multiplies it by (1 - c lam) / (1 + c lam), c = tau / 2
    n, h, eps, tau, m = 17, 0.5, 3.0, 0.8, 5
    grid = _tiny(n, h, ny=6, nz=5)
    eps_node = np.full((5, 6, n), eps)
    i = np.arange(n)
    mode = np.sin(np.pi * m * i / (n - 1))
    s = np.zeros((5, 6, n))
    s[1:-1, 1:-1, :] = mode
    lam = (eps / h ** 2) * 4.0 * np.sin(np.pi * m / (2.0 * (n - 1))) ** 2
    g = (1.0 - 0.5 * tau * lam) / (1.0 + 0.5 * tau * lam)
    v = oracle.cn_sweep(s, eps_node, tau, h, axis=2)
    assert np.max(np.abs(v[1:-1, 1:-1, :] - g * s[1:-1, 1:-1, :])) <= 1e-13
    assert abs(g) < 1.0 and g < 0.0   # a stiff mode: damped with a sign flip


# --------------------------------------------------------------------------
# the analytic benchmark of Sec. 4.1 (charged cavity) against the paper's
# printed spatial-convergence errors (Tables LODspat, AOSIEspat, MAOSspat)

def _sphere_errors(h, scheme, face_rule="harmonic"):
    b = inputs.sphere_benchmark(h)
    pb = oracle.problem_from_fields(b.grid, b.solute, b.eps_in, b.eps_out, b.kbar_sq, b.rho, b.u0,
                                    face_rule=face_rule)
    dt = h * h / 20.0
    u = oracle.run(pb, dt, 1.0, int(round(10.0 / dt)), scheme)
    e = (u - b.exact)[b.valid]
    ex = b.exact[b.valid]
    return (float(np.sqrt(np.sum(e * e) / np.sum(ex * ex))),
            float(np.max(np.abs(e)) / np.max(np.abs(ex))))


def test_sphere_benchmark_fields_are_the_analytic_problem():
    # the exact field is continuous across r = R; the initial field meets
    # the Dirichlet data on the shell and carries the H term inside
    b = inputs.sphere_benchmark(0.25, H=20.0)
    n = b.grid.nx
    c = n // 2
    x = np.array([b.grid.origin[0] + i * b.grid.h for i in range(n)])
    onR = np.argmin(np.abs(x - 1.0))
    assert b.exact[c, c, onR] == pytest.approx(1.0 / 80.0, rel=1e-12)
    B = oracle.boundary_shell(b.grid)
    assert np.array_equal(b.u0[B], b.exact[B])
    assert b.u0[c, c, c] == 20.0 and b.rho[c, c, c] == pytest.approx(4 * math.pi / 0.25 ** 3)


@pytest.mark.parametrize("scheme,key", [("LODIE2", "LODIE"), ("LODCN2", "LODCN"),
                                        ("AOSIE2", "AOSIE2"), ("MAOSIE", "MAOSIE")])
def test_sphere_spatial_errors_match_the_paper_table(scheme, key):
    # h = 0.5 and 0.25 (Delta t = h^2 / 20, T = 10): the relative L2 and Linf
    # errors against the analytic solution agree with the printed values to
    # within 30 % (measured: within 26 %).  Parity at the printed digits is not expected: the paper
    # sets eps at half points from an MSMS-derived surface, here it is the
    # harmonic mean of nodal values, which matters most at the coarsest h
    # (h = 1 is left out for that reason).
    ref = json.load(open(os.path.join(GOLDEN, "paper_sphere_spatial.json")))
    for h in (0.5, 0.25):
        l2, linf = _sphere_errors(h, scheme)
        i = ref["h"].index(h)
        assert l2 == pytest.approx(ref[key]["L2"][i], rel=0.3), (h, l2)
        assert linf == pytest.approx(ref[key]["Linf"][i], rel=0.3), (h, linf)


@pytest.mark.parametrize("scheme,key", [("LODIE2", "LODIE"), ("LODCN2", "LODCN"),
                                        ("MAOSCN", "MAOSCN"), ("AOSCN1", "AOSCN1"),
                                        ("AOSCN2", "AOSCN2"), ("AOSIE2", "AOSIE2"),
                                        ("MAOSIE", "MAOSIE")])
def test_sphere_spatial_errors_with_the_location_rule_reproduce_the_paper_table(scheme, key):
    # with eps at each half point by its own location (the paper's rule),
    # the printed errors come back at every h down to the coarsest: the LOD
    # schemes, AOSCN1, AOSCN2 and MAOSCN to the printed 3 digits (at h = 1
    # AOSCN1/2 and MAOSCN to 3 digits too, LODIE/LODCN L2 within 3 %), the
    # implicit-Euler additive family (AOSIE2, MAOSIE) within 2 % for h <= 0.5
    # only: at h = 1 it sits about a third below the printed row under every
    # reading tried (see the design notes)
    ref = json.load(open(os.path.join(GOLDEN, "paper_sphere_spatial.json")))
    exact3 = key in ("LODIE", "LODCN", "MAOSCN", "AOSCN1", "AOSCN2")
    for h in ((1.0, 0.5, 0.25) if exact3 else (0.5, 0.25)):
        l2, linf = _sphere_errors(h, scheme, "location")
        i = ref["h"].index(h)
        tol = (0.03 if h == 1.0 else 0.006) if exact3 else 0.02
        assert l2 == pytest.approx(ref[key]["L2"][i], rel=tol), (h, l2)
        assert linf == pytest.approx(ref[key]["Linf"][i], rel=max(tol, 0.006)), (h, linf)
