"""Error norms against exact fields (test infrastructure only).

The relative errors of the paper's convergence study (Sec. 4.1, eq. (errors)):
L2 and H1-seminorm of the velocity error and L2 of the pressure error, each
divided by the same norm of the exact field, integrated with a conical-product
(collapsed Gauss-Jacobi) rule of high degree.
"""
import numpy as np
from scipy.special import roots_jacobi


def _gj01(n, alpha):
    """n-point Gauss-Jacobi rule on [0,1] for the weight (1-u)^alpha."""
    x, w = roots_jacobi(n, alpha, 0.0)
    return (1.0 + x) / 2.0, w / 2.0 ** (alpha + 1)


def tet_rule(n=4):
    """Conical-product rule on the unit simplex with n^3 points, exact for
    polynomials of degree 2n-1.  Returns barycentric coordinates [q][4] and
    weights summing to 1/6."""
    u1, w1 = _gj01(n, 2.0)
    u2, w2 = _gj01(n, 1.0)
    u3, w3 = _gj01(n, 0.0)
    pts, wts = [], []
    for a, wa in zip(u1, w1):
        for b, wb in zip(u2, w2):
            for c, wc in zip(u3, w3):
                x1 = a
                x2 = b * (1.0 - a)
                x3 = c * (1.0 - a) * (1.0 - b)
                pts.append([1.0 - x1 - x2 - x3, x1, x2, x3])
                wts.append(wa * wb * wc)
    return np.array(pts), np.array(wts)


def p1_errors(coords, tets, u_h, p_h, exact, t, nq=4):
    """Relative errors (e_L2^u, e_H1^u, e_L2^p) of P1 nodal fields against `exact`
    (an object with velocity, grad and pressure methods) at time t."""
    lam, w = tet_rule(nq)
    X = coords[tets]                                               # [nt][4][3]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    Jinv = np.linalg.inv(J)
    det = np.abs(np.linalg.det(J))
    grads = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)   # [nt][4][3]
    U = u_h[tets]                                                  # [nt][4][3]
    P = p_h[tets]
    gradU = np.einsum("eac,eaj->ecj", U, grads)                   # [nt][3][3]
    eu = nu = eg = ng = ep = npp = 0.0
    for q in range(len(w)):
        xq = np.einsum("a,eac->ec", lam[q], X)
        uq = np.einsum("a,eac->ec", lam[q], U)
        pq = P @ lam[q]
        ue = exact.velocity(xq, t)
        ge = exact.grad(xq, t)
        pe = exact.pressure(xq, t)
        wq = w[q] * det
        eu += np.sum(wq * np.sum((uq - ue) ** 2, axis=1))
        nu += np.sum(wq * np.sum(ue ** 2, axis=1))
        eg += np.sum(wq * np.sum((gradU - ge) ** 2, axis=(1, 2)))
        ng += np.sum(wq * np.sum(ge ** 2, axis=(1, 2)))
        ep += np.sum(wq * (pq - pe) ** 2)
        npp += np.sum(wq * pe ** 2)
    return np.sqrt(eu / nu), np.sqrt(eg / ng), np.sqrt(ep / npp)


def p2_errors(coords, tets, edge_of_tet, u_h, p_h, exact, t, nq=4):
    """Relative errors (e_L2^u, e_H1^u, e_L2^p) of a P2 velocity (nodal values at the
    vertices, then at the edges indexed by edge_of_tet [nt][6]) and a P1 pressure."""
    lam, w = tet_rule(nq)
    nv = coords.shape[0]
    X = coords[tets]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    Jinv = np.linalg.inv(J)
    det = np.abs(np.linalg.det(J))
    dl = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)      # [nt][4][3]
    nodes = np.concatenate([tets, nv + edge_of_tet], axis=1)
    U = u_h[nodes]                                                             # [nt][10][3]
    P = p_h[tets]
    E = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    eu = nu = eg = ng = ep = npp = 0.0
    for q in range(len(w)):
        L = lam[q]
        phi = np.array([L[a] * (2 * L[a] - 1) for a in range(4)] + [4 * L[i] * L[j] for i, j in E])
        dphi = np.concatenate([(4 * L[:4, None] - 1)[None, :, :] * dl,
                               np.stack([4 * (L[i] * dl[:, j] + L[j] * dl[:, i]) for i, j in E], axis=1)], axis=1)
        xq = np.einsum("a,eac->ec", L, X)
        uq = np.einsum("a,eac->ec", phi, U)
        gq = np.einsum("eac,eaj->ecj", U, dphi)
        pq = P @ L
        ue, ge, pe = exact.velocity(xq, t), exact.grad(xq, t), exact.pressure(xq, t)
        wq = w[q] * det
        eu += np.sum(wq * np.sum((uq - ue) ** 2, axis=1))
        nu += np.sum(wq * np.sum(ue ** 2, axis=1))
        eg += np.sum(wq * np.sum((gq - ge) ** 2, axis=(1, 2)))
        ng += np.sum(wq * np.sum(ge ** 2, axis=(1, 2)))
        ep += np.sum(wq * (pq - pe) ** 2)
        npp += np.sum(wq * pe ** 2)
    return np.sqrt(eu / nu), np.sqrt(eg / ng), np.sqrt(ep / npp)
