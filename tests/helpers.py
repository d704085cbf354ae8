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


# FP64 parity gate.  Two FP64 evaluations of the split-form residual that round differently
# disagree at the rounding level of its cancelling sums, so the bar is set by the oracle's own
# FP64 error e64 (its double build against its long-double build on the same input): the GPU
# must lie within max(floor |ref|, GATE e64) of the long-double result, per conserved variable.
# GATE = 2: the GPU may round at most twice as badly as the plain FP64 oracle.
GATE = 2.0


def parity_log(name, **fields):
    """Append one JSON record of a parity comparison to $PARITY_LOG (when set)."""
    import json
    import os
    path = os.environ.get("PARITY_LOG")
    if not path:
        return
    rec = {"case": name}
    for k, v in fields.items():
        rec[k] = np.asarray(v).tolist() if isinstance(v, np.ndarray) else v
    with open(path, "a") as f:
        f.write(json.dumps(rec) + "\n")


def gate_ok(name, eg, e64, scale, floor=1e-12):
    """True when every variable's GPU error eg lies within max(floor scale, GATE e64); logs the
    errors relative to the scale and the ratio eg / e64."""
    eg, e64, scale = (np.asarray(x, dtype=np.float64) for x in (eg, e64, scale))
    tol = np.maximum(floor * scale, GATE * e64)
    ratio = eg / np.maximum(e64, 1e-300)
    parity_log(name, gpu_rel=eg / np.maximum(scale, 1e-300), fp64_rel=e64 / np.maximum(scale, 1e-300),
               ratio=ratio, ok=bool(np.all(eg <= tol)))
    return bool(np.all(eg <= tol))


# Stated tolerances of the FP32-bulk path: relative L-inf per conserved variable (rho, rho v1-3,
# rho e) of the FP32-bulk result against FP64 (the oracle, or the oracle-checked FP64 GPU path),
# about twice the largest error measured on each workload.  The error is set by FP32 rounding of
# the O(1) convective and pressure fluxes, whose sums cancel to the residual: it grows with the
# ratio of the flux terms (~1/h) to the residual, i.e. with resolution and with 1/Ma^2.
#   SMALL  Taylor-Green vortex Ma 0.1 up to 8^3 elements at N = 4 and 4^3 up to N = 7
#          (measured at most 2.8e-6, 1.25e-4, 1.10e-4, 1.8e-5, 1.6e-5);
#   C2     the 32^3, N = 4 benchmark mesh (measured 1.1e-5, 3.5e-4, 3.5e-4, 6.5e-5, 4.8e-5);
#   C5     the 64^3, N = 5 mesh (measured 3.7e-5, 1.33e-3, 1.32e-3, 2.3e-4, 1.9e-4);
#   MIXED  mixed orders 2..6, isentropic vortex Ma 0.5 up to 24^3 elements (measured 8.9e-6,
#          1.06e-5, 1.0e-5, 2.6e-5, 8.4e-6).
FP32_TOL = {
    "small": np.array([6e-6, 2.5e-4, 2.5e-4, 2.5e-4, 4e-5]),
    "c2": np.array([2.5e-5, 8e-4, 8e-4, 8e-4, 1e-4]),
    "c5": np.array([8e-5, 2.7e-3, 2.7e-3, 2.7e-3, 4e-4]),
    "mixed": np.array([2e-5, 2.5e-5, 2.5e-5, 6e-5, 2e-5]),
}
