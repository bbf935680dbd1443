"""Independent definitions used to pin the oracle (test helpers only).

Nothing here shares code with the oracle or the GPU path.

* ``energy_matrix_form``: the discrete energy E_h of sec. 2 written in the
  paper's matrix form, 1/2(-k1 p^T D p - k1 q^T D q - k2 u^T D u + v^T v
  + mu^2 u^T u) - g (p^2 + q^2)^T u, with D the periodic central-difference
  Laplacian assembled as a Kronecker sum of the 1-D second-difference matrix.
  The oracle writes E_h with squared forward differences instead; the two
  agree by summation by parts.  The function is analytic in its arguments, so
  complex-step differentiation gives exact-to-rounding gradients.

* ``dp_avf_point_solve``: one pointwise DP-AVF update obtained by solving the
  defining equation (eq. dp-avf-i) with Newton's method:
      (y_new - y_old)/tau = J * int_0^1 grad_{y} E_h(... y^theta ...) dtheta,
  where the integrand follows the dual-partition rule of eq. dp-avf (the
  variable earlier in the variable order enters with its new value, the later
  one with its old value), the gradient is a complex-step derivative of
  ``energy_matrix_form`` and the theta-integral is 3-point Gauss-Legendre,
  exact for the polynomial integrand (degree <= 2 in theta).
"""
from __future__ import annotations

import numpy as np

# Gauss-Legendre nodes/weights on [0, 1]
_GL_X = 0.5 + 0.5 * np.array([-np.sqrt(3.0 / 5.0), 0.0, np.sqrt(3.0 / 5.0)])
_GL_W = 0.5 * np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])


def laplacian_matrix(dim: int, n: int, h: float) -> np.ndarray:
    """Periodic central-difference Laplacian on n^dim points (C order)."""
    D2 = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    D2[0, -1] += 1.0
    D2[-1, 0] += 1.0
    D2 /= h * h
    I = np.eye(n)
    D = np.zeros((n ** dim, n ** dim))
    for a in range(dim):
        term = np.array([[1.0]])
        for b in range(dim):
            term = np.kron(term, D2 if a == b else I)
        D = D + term
    return D


def energy_matrix_form(D, h, dim, k1, k2, mu, g, p, q, u, v):
    """h^dim * E_h in the matrix form of sec. 2 (p, q, u, v flat, maybe complex)."""
    E = 0.5 * (-k1 * (p @ (D @ p)) - k1 * (q @ (D @ q)) - k2 * (u @ (D @ u)) + v @ v
               + mu * mu * (u @ u)) - g * ((p * p + q * q) @ u)
    return h ** dim * E


class PointProblem:
    """A flat state plus the parameters; gradients by complex step."""

    def __init__(self, dim, n, h, k1, k2, mu, g, P, Q, U, V):
        self.dim, self.n, self.h = dim, n, h
        self.k = (k1, k2, mu, g)
        self.D = laplacian_matrix(dim, n, h)
        self.z = {"p": P.ravel().astype(np.complex128), "q": Q.ravel().astype(np.complex128),
                  "u": U.ravel().astype(np.complex128), "v": V.ravel().astype(np.complex128)}

    def E(self, z):
        return energy_matrix_form(self.D, self.h, self.dim, *self.k, z["p"], z["q"], z["u"], z["v"])

    def dE(self, z, var, i, step=1e-30):
        zz = {k: a.copy() for k, a in z.items()}
        zz[var][i] += 1j * step
        # E is h^dim * E_h; the scheme uses the gradient of E_h itself
        return self.E(zz).imag / step / self.h ** self.dim


def dp_avf_point_solve(pp: PointProblem, tau: float, i: int, pair: str, adjoint: bool,
                       iters: int = 60):
    """Solve the DP-AVF equation for one point and one variable pair.

    pair == "psi": y = (p_i, q_i) with J = [[0, 1/2], [-1/2, 0]];
    pair == "uv":  y = (u_i, v_i) with J = [[0, 1], [-1, 0]].
    The base variable order is p > q > u > v, the adjoint order v > u > q > p
    (sec. 3.2).  Returns the new (y1, y2)."""
    a, b = ("p", "q") if pair == "psi" else ("u", "v")
    scale = 0.5 if pair == "psi" else 1.0
    first, second = (b, a) if adjoint else (a, b)
    y_old = np.array([pp.z[a][i].real, pp.z[b][i].real])

    def F(y):
        new = {a: y[0], b: y[1]}
        old = {a: y_old[0], b: y_old[1]}
        grads = {}
        for var in (a, b):
            other = b if var == a else a
            # the other variable of the pair: new value if it comes earlier in the order
            other_val = new[other] if other == first else old[other]
            acc = 0.0
            for th, w in zip(_GL_X, _GL_W):
                z = {k: arr.copy() for k, arr in pp.z.items()}
                z[var][i] = th * new[var] + (1.0 - th) * old[var]
                z[other][i] = other_val
                acc += w * pp.dE(z, var, i)
            grads[var] = acc
        # J grad: d/dt a = scale * grad_b, d/dt b = -scale * grad_a
        r0 = (y[0] - y_old[0]) / tau - scale * grads[b]
        r1 = (y[1] - y_old[1]) / tau + scale * grads[a]
        return np.array([r0, r1])

    y = y_old.copy()
    for _ in range(iters):
        f = F(y)
        J = np.empty((2, 2))
        for c in range(2):
            e = np.zeros(2)
            e[c] = 1e-6 * max(1.0, abs(y[c]))
            J[:, c] = (F(y + e) - F(y - e)) / (2 * e[c])
        dy = np.linalg.solve(J, -f)
        y = y + dy
        if np.all(np.abs(dy) <= 1e-17 * np.maximum(1.0, np.abs(y))):
            break
    return y
