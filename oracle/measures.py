"""Approximation measures and circular statistics (Sec. 4.2).

TEST INFRASTRUCTURE: see the package docstring.  All with rho = 0.95 unless
given; C is the orthonormal DCT (see `matrices.dct_matrix`).
"""

from __future__ import annotations

import math

import numpy as np

from .matrices import approx_matrix, dct_matrix


def covariance(rho: float = 0.95, n: int = 8) -> np.ndarray:
    """R_x[i, j] = rho^|i-j| (Sec. 4.2)."""
    i = np.arange(n)
    return rho ** np.abs(i[:, None] - i[None, :]).astype(np.float64)


def total_error_energy(c_hat: np.ndarray) -> float:
    """epsilon = pi ||C - C_hat||_F^2 (Sec. 4.2.1)."""
    d = dct_matrix() - c_hat
    return math.pi * float(np.sum(d * d))


def mse(c_hat: np.ndarray, rho: float = 0.95) -> float:
    """MSE = (1/8) tr((C - C_hat) R_x (C - C_hat)^T) (Sec. 4.2.2)."""
    d = dct_matrix() - c_hat
    return float(np.trace(d @ covariance(rho) @ d.T)) / 8.0


def coding_gain(c_hat: np.ndarray, rho: float = 0.95) -> float:
    """C_g for orthogonal transforms (Sec. 4.2.3): r_ii = diag(C_hat R_x C_hat^T),
    10 log10( mean(r_ii) / (prod(r_ii ||c_i||^2))^(1/8) )."""
    r = np.diag(c_hat @ covariance(rho) @ c_hat.T)
    nrm = np.sum(c_hat * c_hat, axis=1)
    return 10.0 * math.log10(float(np.mean(r)) / float(np.prod(r * nrm)) ** 0.125)


def unified_coding_gain(c_hat: np.ndarray, rho: float = 0.95) -> float:
    """Unified coding gain C_g* (Sec. 4.2.3):
    10 log10 prod_i 1/(A_i B_i)^(1/8), A_i = su[(c_i c_i^T) o R_x],
    B_i = ||g_i||^2 with g_i^T the i-th ROW of C_hat^-1 (literal reading)."""
    rx = covariance(rho)
    g = np.linalg.inv(c_hat)
    total = 0.0
    for i in range(8):
        ci = c_hat[i]
        a = float(np.sum(np.outer(ci, ci) * rx))
        b = float(np.sum(g[i] * g[i]))
        total += -math.log10(a * b) / 8.0
    return 10.0 * total


def transform_efficiency(c_hat: np.ndarray, rho: float = 0.95) -> float:
    """eta = sum|r_ii| / sum|r_ij| * 100 with R_y = C_hat R_x C_hat^T (Sec. 4.2.4)."""
    ry = c_hat @ covariance(rho) @ c_hat.T
    return float(np.sum(np.abs(np.diag(ry))) / np.sum(np.abs(ry)) * 100.0)


def angle(u: np.ndarray, v: np.ndarray) -> float:
    """angle(u, v) = arccos(<u, v> / (||u|| ||v||)) (Sec. 3.3)."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    c = float(np.dot(u, v) / (np.linalg.norm(u) * np.linalg.norm(v)))
    return math.acos(max(-1.0, min(1.0, c)))


def row_angles_to_e1(m: np.ndarray) -> np.ndarray:
    """theta_k = angle(m_k / ||m_k||, q), q = [1, 0, ..., 0] (Sec. 4.2.5)."""
    q = np.zeros(8)
    q[0] = 1.0
    return np.array([angle(row, q) for row in np.asarray(m, dtype=np.float64)])


def circular_mean(theta: np.ndarray) -> float:
    """Circular mean by the case analysis of Sec. 4.2.5 (radians)."""
    c = float(np.sum(np.cos(theta)))
    s = float(np.sum(np.sin(theta)))
    if c > 0 and s >= 0:
        return math.atan(s / c)
    if c == 0 and s > 0:
        return math.pi / 2
    if c < 0:
        return math.atan(s / c) + math.pi
    if c >= 0 and s < 0:
        return math.atan(s / c) + 2 * math.pi if c != 0 else 3 * math.pi / 2
    raise ValueError("circular mean undefined for C = S = 0")


def circular_variance(theta: np.ndarray) -> float:
    """V = 1 - sqrt(C^2 + S^2) / 8 (Sec. 4.2.5)."""
    c = float(np.sum(np.cos(theta)))
    s = float(np.sum(np.sin(theta)))
    return 1.0 - math.sqrt(c * c + s * s) / 8.0


def modified_mean_circular_difference(theta_c: np.ndarray, theta_t: np.ndarray) -> float:
    """D_mod = (1/8) sum_i (pi - |pi - |theta_ci - theta_ti||) (Sec. 4.2.5)."""
    d = np.abs(np.asarray(theta_c) - np.asarray(theta_t))
    return float(np.mean(math.pi - np.abs(math.pi - d)))


def mean_circular_difference(theta_c: np.ndarray, theta_t: np.ndarray) -> float:
    """D-bar over all 64 pairs (Sec. 4.2.5)."""
    d = np.abs(np.asarray(theta_c)[:, None] - np.asarray(theta_t)[None, :])
    return float(np.mean(math.pi - np.abs(math.pi - d)))


def measures(t: np.ndarray, rho: float = 0.95) -> dict:
    """The four figures of merit of Sec. 4.3's measures table for C_hat = S T."""
    c_hat = approx_matrix(t)
    return {"eps": total_error_energy(c_hat), "mse": mse(c_hat, rho),
            "cg_star": unified_coding_gain(c_hat, rho),
            "eta": transform_efficiency(c_hat, rho)}


def dct_measures(rho: float = 0.95) -> dict:
    c = dct_matrix()
    return {"eps": total_error_energy(c), "mse": mse(c, rho),
            "cg_star": unified_coding_gain(c, rho), "eta": transform_efficiency(c, rho)}


def circular_stats(m: np.ndarray) -> dict:
    """theta-bar (degrees), V and D_mod against the DCT rows (radians)."""
    th_t = row_angles_to_e1(m)
    th_c = row_angles_to_e1(dct_matrix())
    return {"theta_bar_deg": math.degrees(circular_mean(th_t)),
            "V": circular_variance(th_t),
            "D_mod": modified_mean_circular_difference(th_c, th_t)}
