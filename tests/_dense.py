"""Brute-force dense reference machinery for pinning the oracle on tiny grids.

Every matrix here is assembled node by node from the definitions in the
paper (central differences with dielectric at half points, Eq.
(SpatialOperators); Dirichlet rows are identity rows), independently of the
oracle's line solver, and solved with numpy.linalg.
"""
import numpy as np


def harmonic(a, b):
    return 2.0 * a * b / (a + b)


def _is_interior(idx, shape):
    return all(1 <= idx[d] <= shape[d] - 2 for d in range(3))


def dense_second_difference(eps_node, h, axis, faces=None):
    """Matrix D_axis over all nodes (zyx-flattened): rows of interior nodes
    hold h^-2 (e+ (v+ - v) + e- (v- - v)); other rows are zero.  e+- are
    harmonic means of the nodal values, or read from `faces` (eps at the
    half point between a node and its successor along the axis, stored at
    the node's index) when given."""
    shape = eps_node.shape
    N = eps_node.size
    D = np.zeros((N, N))
    lin = np.arange(N).reshape(shape)
    for k in range(shape[0]):
        for j in range(shape[1]):
            for i in range(shape[2]):
                idx = [k, j, i]
                if not _is_interior(idx, shape):
                    continue
                p = lin[k, j, i]
                up = list(idx)
                dn = list(idx)
                up[axis] += 1
                dn[axis] -= 1
                if faces is None:
                    e_up = harmonic(eps_node[k, j, i], eps_node[tuple(up)])
                    e_dn = harmonic(eps_node[k, j, i], eps_node[tuple(dn)])
                else:
                    e_up = faces[tuple(idx)]
                    e_dn = faces[tuple(dn)]
                D[p, lin[tuple(up)]] += e_up / h ** 2
                D[p, lin[tuple(dn)]] += e_dn / h ** 2
                D[p, p] -= (e_up + e_dn) / h ** 2
    return D


def interior_flags(shape):
    f = np.zeros(shape, dtype=bool)
    f[1:-1, 1:-1, 1:-1] = True
    return f.ravel()


def affine_fixed_point(Mmap, cvec, g_full, interior):
    """Fixed point of u -> M u + c with the non-interior values held at g."""
    I = interior
    B = ~interior
    A = np.eye(I.sum()) - Mmap[np.ix_(I, I)]
    rhs = Mmap[np.ix_(I, B)] @ g_full[B] + cvec[I]
    u = g_full.copy()
    u[I] = np.linalg.solve(A, rhs)
    return u


def newton_npb(D, kbar2, rho, g_full, interior, iters=60):
    """Discrete NPB on the interior: -D u + kbar2 sinh(u) = rho, u = g on the
    boundary (dense Newton)."""
    I = interior
    u = g_full.copy()
    u[I] = 0.0
    for _ in range(iters):
        F = -(D @ u) + kbar2 * np.sinh(u) - rho
        J = -D[np.ix_(I, I)] + np.diag(kbar2[I] * np.cosh(u[I]))
        du = np.linalg.solve(J, -F[I])
        u[I] += du
        if np.max(np.abs(du)) < 1e-14 * max(1.0, np.max(np.abs(u))):
            break
    return u
