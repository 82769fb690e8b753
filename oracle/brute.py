"""NumPy brute-force form of the filter step, for tiny cubes.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Written independently of
oracle.c as a cross-check: instead of index clamping it pads the cube with a
copy of its own faces (so every difference across a face is zero, the
reflecting boundary) and forms the six neighbour differences with shifted
views, Eq. 7 of Section 3.3 for the intensity weight and the per-edge
Perona-Malik weights for the other two forms.
"""
import numpy as np


def _weights(cond, d, kr):
    if cond == "pm_exp":
        return np.exp(-(d / kr) ** 2)
    if cond == "pm_rational":
        return 1.0 / (1.0 + (d / kr) ** 2)
    return np.ones_like(d)


def step(I, cond, K, rho, tau, C):
    """One synchronous step on an FP64 array of shape (nz, ny, nx)."""
    P = np.pad(I, 1, mode="edge")
    core = P[1:-1, 1:-1, 1:-1]
    kr = K * rho
    # (shifted neighbour view, axis weight); array axes are (z, y, x)
    nbrs = [
        (P[1:-1, 1:-1, 2:], C[0]), (P[1:-1, 1:-1, :-2], C[0]),
        (P[1:-1, 2:, 1:-1], C[1]), (P[1:-1, :-2, 1:-1], C[1]),
        (P[2:, 1:-1, 1:-1], C[2]), (P[:-2, 1:-1, 1:-1], C[2]),
    ]
    acc = np.zeros_like(core)
    for Nb, c in nbrs:
        d = Nb - core
        acc = acc + c * _weights(cond, d, kr) * d
    if cond == "intensity":
        return core + tau * acc / (1.0 + core ** 2 / kr ** 2)
    return core + tau * acc


def run(I0, cond="pm_exp", K=2.0, tau=1.0 / 16, n_iter=1, C=(1.0, 1.0, 1.0), rms=None):
    I = np.asarray(I0, dtype=np.float64)
    rho = float(np.sqrt(np.mean(I * I))) if rms is None else float(rms)
    for _ in range(n_iter):
        I = step(I, cond, K, rho, tau, C)
    return I, rho
