"""Butcher tableaux of classical explicit Runge-Kutta methods (inputs shared
by the oracle tests and the GPU tests): name -> (A, b, c, order).

Euler; Heun (explicit trapezoid); explicit midpoint; Kutta's third-order
method; the classical RK4; Kutta's 3/8 rule (Hairer, Norsett, Wanner,
Solving ODEs I, Sec. II.1)."""
import numpy as np

TABLEAUX = {
    "euler": ([[0.0]], [1.0], [0.0], 1),
    "heun": ([[0.0, 0.0], [1.0, 0.0]], [0.5, 0.5], [0.0, 1.0], 2),
    "midpoint": ([[0.0, 0.0], [0.5, 0.0]], [0.0, 1.0], [0.0, 0.5], 2),
    "rk3": ([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [-1.0, 2.0, 0.0]], [1 / 6, 2 / 3, 1 / 6], [0.0, 0.5, 1.0], 3),
    "rk4": ([[0.0, 0.0, 0.0, 0.0], [0.5, 0.0, 0.0, 0.0], [0.0, 0.5, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0]],
            [1 / 6, 1 / 3, 1 / 3, 1 / 6], [0.0, 0.5, 0.5, 1.0], 4),
    "rk38": ([[0.0, 0.0, 0.0, 0.0], [1 / 3, 0.0, 0.0, 0.0], [-1 / 3, 1.0, 0.0, 0.0], [1.0, -1.0, 1.0, 0.0]],
             [1 / 8, 3 / 8, 3 / 8, 1 / 8], [0.0, 1 / 3, 2 / 3, 1.0], 4),
}


def tableau(name):
    A, b, c, p = TABLEAUX[name]
    return np.array(A, dtype=np.float64), np.array(b, dtype=np.float64), np.array(c, dtype=np.float64), p


def stability_matrix(name, Z):
    """R(Z) = I + sum_k (b^T A^(k-1) 1) Z^k: one step of the method applied to
    y' = Z y / h (exact expansion for an explicit method, whose A is
    nilpotent)."""
    A, b, c, _ = tableau(name)
    s = b.shape[0]
    R = np.eye(Z.shape[0])
    Ak = np.eye(s)
    Zk = np.eye(Z.shape[0])
    for k in range(1, s + 1):
        Zk = Zk @ Z
        R = R + (b @ Ak @ np.ones(s)) * Zk
        Ak = Ak @ A
    return R
