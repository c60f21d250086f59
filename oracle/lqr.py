"""Closed forms for the linear-quadratic case (test infrastructure only).

For x_{i+1} = Ad x_i + Bd v_i (Ad = I + dt A, Bd = dt B) and the per-step cost of
Algorithm 1, S(v) = sum_{i=1..T} x_i^T Q x_i + x_T^T Qf x_T + sum_i 1/2 v_i^T R v_i,
the cost is quadratic in the stacked controls: S(v) = 1/2 v^T H v + g^T v + c.

* ``batch_lqr`` solves it by least squares; ``riccati_lqr`` by the textbook backward
  Riccati recursion (a cross-check of the former).
* ``expected_update`` is the K -> infinity limit of one MPPI iteration: with
  du ~ N(0, nu Sigma) and the likelihood-ratio cost of Section III-C, the weighted
  law of v = U + du is Gaussian with precision P = (Sigma^-1 - R/lam)/nu + H/lam and
  mean P^-1 [ (Sigma^-1 - R/lam) U / nu - g / lam ].  With the noise-cost coupling
  R = lam Sigma^-1 of Section II this is the LQR optimum -H^-1 g in one iteration;
  without it, the LQR optimum is the fixed point of the iteration.
"""
import numpy as np


def discrete(A, B, dt):
    n = A.shape[0]
    return np.eye(n) + dt * A, dt * B


def stacked(A, B, dt, T):
    """X = Phi x0 + Gam V with X = (x_1..x_T), V = (v_0..v_{T-1})."""
    Ad, Bd = discrete(A, B, dt)
    n, m = Bd.shape
    Phi = np.zeros((T * n, n))
    Gam = np.zeros((T * n, T * m))
    P = np.eye(n)
    for i in range(T):
        P = Ad @ P
        Phi[i * n:(i + 1) * n] = P
        for j in range(i + 1):
            Gam[i * n:(i + 1) * n, j * m:(j + 1) * m] = np.linalg.matrix_power(Ad, i - j) @ Bd
    return Phi, Gam


def quadratic_form(A, B, Q, Qf, R, dt, T, x0):
    """H, g of S(v) = 1/2 v^T H v + g^T v + c."""
    n = A.shape[0]
    Phi, Gam = stacked(A, B, dt, T)
    Qb = np.kron(np.eye(T), Q)
    Qb[(T - 1) * n:, (T - 1) * n:] += Qf
    Rb = np.kron(np.eye(T), R)
    H = 2.0 * Gam.T @ Qb @ Gam + Rb
    g = 2.0 * Gam.T @ Qb @ Phi @ x0
    return H, g


def batch_lqr(A, B, Q, Qf, R, dt, T, x0):
    H, g = quadratic_form(A, B, Q, Qf, R, dt, T, x0)
    m = B.shape[1]
    return np.linalg.solve(H, -g).reshape(T, m)


def riccati_lqr(A, B, Q, Qf, R, dt, T, x0):
    """Backward Riccati recursion for min sum_i [x_{i+1}^T Q x_{i+1} + 1/2 v_i^T R v_i] + x_T^T Qf x_T."""
    Ad, Bd = discrete(A, B, dt)
    P = Q + Qf               # cost-to-go weight of x_T
    gains = []
    for i in reversed(range(T)):
        Kg = np.linalg.solve(R + 2.0 * Bd.T @ P @ Bd, 2.0 * Bd.T @ P @ Ad)
        gains.append(Kg)
        Acl = Ad - Bd @ Kg
        P_next = 0.5 * Kg.T @ R @ Kg + Acl.T @ P @ Acl
        P = P_next + (Q if i > 0 else 0.0)
    gains.reverse()
    x = np.asarray(x0, float)
    U = []
    for Kg in gains:
        u = -Kg @ x
        U.append(u)
        x = Ad @ x + Bd @ u
    return np.asarray(U)


def expected_update(A, B, Q, Qf, R, dt, T, x0, U, sigma, nu, lam):
    """K -> infinity limit of one MPPI iteration from U (see module docstring)."""
    H, g = quadratic_form(A, B, Q, Qf, R, dt, T, x0)
    Si = np.kron(np.eye(T), np.linalg.inv(sigma))
    Rb = np.kron(np.eye(T), R)
    D = (Si - Rb / lam) / nu
    P = D + H / lam
    mean = np.linalg.solve(P, D @ np.ravel(U) - g / lam)
    return mean.reshape(U.shape)
