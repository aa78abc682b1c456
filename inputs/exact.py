"""Closed-form fields of the verification problems (problem data, not solver code).

* Beltrami flow (Ethier and Steinman 1994), the exact Navier-Stokes solution the
  paper uses for software verification (its Appendix A), parametrised by a, d,
  density rho and viscosity mu; forcing is zero.
* Affine patch fields (constant, Couette, stagnation) whose discrete solution is
  exact on any P1 mesh.

Gradients use the convention grad(u)[i][j] = d u_i / d x_j.  The Neumann datum
for the gradient-gradient diffusion form is the traction (mu grad u - p I) n.
"""
import numpy as np


def _bx(x, y, z, a, d):
    """x-component of the Beltrami velocity without the -a e^{-d^2 nu t} factor,
    and its partial derivatives."""
    eax, eaz = np.exp(a * x), np.exp(a * z)
    s1, c1 = np.sin(a * y + d * z), np.cos(a * y + d * z)
    s2, c2 = np.sin(a * x + d * y), np.cos(a * x + d * y)
    val = eax * s1 + eaz * c2
    dx = a * eax * s1 - a * eaz * s2
    dy = a * eax * c1 - d * eaz * s2
    dz = d * eax * c1 + a * eaz * c2
    return val, dx, dy, dz


class Beltrami:
    """u, p, grad u of the Beltrami flow on arbitrary points X [n][3] at time t."""

    def __init__(self, a=np.pi / 4, d=np.pi / 2, rho=1.0, mu=0.01):
        self.a, self.d, self.rho, self.mu = a, d, rho, mu
        self.nu = mu / rho

    def _amp(self, t):
        return -self.a * np.exp(-self.d * self.d * self.nu * t)

    def velocity(self, X, t):
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        A = self._amp(t)
        ux = _bx(x, y, z, self.a, self.d)[0]
        uy = _bx(y, z, x, self.a, self.d)[0]
        uz = _bx(z, x, y, self.a, self.d)[0]
        return A * np.stack([ux, uy, uz], axis=1)

    def grad(self, X, t):
        """[n][3][3] with G[:, i, j] = d u_i / d x_j."""
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        A = self._amp(t)
        G = np.empty((X.shape[0], 3, 3))
        _, dx, dy, dz = _bx(x, y, z, self.a, self.d)
        G[:, 0, 0], G[:, 0, 1], G[:, 0, 2] = dx, dy, dz
        # u_y(x,y,z) = bx(y,z,x): d/dy -> first slot, d/dz -> second, d/dx -> third
        _, d1, d2, d3 = _bx(y, z, x, self.a, self.d)
        G[:, 1, 1], G[:, 1, 2], G[:, 1, 0] = d1, d2, d3
        _, d1, d2, d3 = _bx(z, x, y, self.a, self.d)
        G[:, 2, 2], G[:, 2, 0], G[:, 2, 1] = d1, d2, d3
        return A * G

    def pressure(self, X, t):
        a, d = self.a, self.d
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        br = (np.exp(2 * a * x) + np.exp(2 * a * y) + np.exp(2 * a * z)
              + 2 * np.sin(a * x + d * y) * np.cos(a * z + d * x) * np.exp(a * (y + z))
              + 2 * np.sin(a * y + d * z) * np.cos(a * x + d * y) * np.exp(a * (z + x))
              + 2 * np.sin(a * z + d * x) * np.cos(a * y + d * z) * np.exp(a * (x + y)))
        return -0.5 * a * a * self.rho * br * np.exp(-2 * d * d * self.nu * t)

    def traction(self, X, t, normal):
        """(mu grad u - p I) n for a constant outward normal n."""
        n = np.asarray(normal, float)
        return self.mu * np.einsum("kij,j->ki", self.grad(X, t), n) - self.pressure(X, t)[:, None] * n[None, :]


class Affine:
    """u = u0 + L x (L constant 3x3), p = p0 + q.x; forcing f = rho (u.grad) u + grad p
    makes it a steady Navier-Stokes solution (Laplacian of an affine field is 0)."""

    def __init__(self, L, u0=(0, 0, 0), q=(0, 0, 0), p0=0.0, rho=1.0, mu=0.01):
        self.L = np.asarray(L, float)
        self.u0 = np.asarray(u0, float)
        self.q = np.asarray(q, float)
        self.p0, self.rho, self.mu = float(p0), rho, mu

    def velocity(self, X, t=0.0):
        return self.u0[None, :] + X @ self.L.T

    def grad(self, X, t=0.0):
        return np.broadcast_to(self.L, (X.shape[0], 3, 3)).copy()

    def pressure(self, X, t=0.0):
        return self.p0 + X @ self.q

    def forcing(self, X, t=0.0):
        u = self.velocity(X)
        return self.rho * (u @ self.L.T) + self.q[None, :]

    def traction(self, X, t, normal):
        n = np.asarray(normal, float)
        return self.mu * np.einsum("kij,j->ki", self.grad(X), n) - self.pressure(X)[:, None] * n[None, :]


def couette(rho=1.0, mu=0.01):
    return Affine([[0, 1, 0], [0, 0, 0], [0, 0, 0]], rho=rho, mu=mu)


def stagnation(rho=1.0, mu=0.01):
    return Affine([[1, 0, 0], [0, -1, 0], [0, 0, 0]], rho=rho, mu=mu)


def constant_flow(u0=(0.3, -0.2, 0.1), rho=1.0, mu=0.01):
    return Affine(np.zeros((3, 3)), u0=u0, rho=rho, mu=mu)


def poiseuille_peak(peak, radius):
    """Centreline velocity of a parabolic profile with peak `peak` (used only to
    convert the configs' peak velocity into the unit-flow-rate amplitude)."""
    return peak * np.pi * radius * radius / 2.0
