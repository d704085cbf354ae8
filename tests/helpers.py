"""Input preparation and norms shared by the tests (no discretisation arithmetic)."""
import numpy as np


def to_conservative(rho, v, p, gamma=1.4):
    """Primitive -> conservative input preparation (rho, rho v, p/(gamma-1) + rho|v|^2/2)."""
    rho = np.asarray(rho, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    return np.concatenate([rho[..., None], rho[..., None] * v,
                           (p / (gamma - 1) + 0.5 * rho * (v * v).sum(-1))[..., None]], axis=-1)


def rel_per_var(R, Rref, E):
    """max|R-Rref|/max|Rref| for each of the 5 variables of a uniform-order layout."""
    A = np.asarray(R).reshape(E, 5, -1)
    B = np.asarray(Rref).reshape(E, 5, -1)
    return np.abs(A - B).max(axis=(0, 2)) / np.maximum(np.abs(B).max(axis=(0, 2)), 1e-300)


def quad_weights_uniform(w, E):
    """w_i w_j w_k for every node of E elements of one order, layout [e][k][j][i] flattened."""
    n = len(w)
    wk = (w[:, None, None] * w[None, :, None] * w[None, None, :]).reshape(-1)
    return np.tile(wk, E)
