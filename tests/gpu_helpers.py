"""Shared helpers for the GPU parity tests: run the oracle and the HIP path on
the same seeded problem and compare."""
import numpy as np

import oracle

ORACLE_TO_GPU = {"phi1": 0, "psi": 1, "ReC": 2, "ImC": 3, "ReB": 4, "ImB": 5, "phase": 6}


def oracle_planes(U):
    """Oracle state [7][nth][nx][nz] -> dict by plane name."""
    return {name: U[i] for name, i in ORACLE_TO_GPU.items()}


def gpu_planes(solver):
    return {k: v.detach().double().cpu().numpy() for k, v in solver.planes().items()}


def rounded_oracle_state(U, dtype):
    """The oracle state as the GPU would store it (planes rounded to the grid
    dtype, psi kept in double), back in float64 oracle layout."""
    out = U.copy()
    if dtype == "f32":
        for name, i in ORACLE_TO_GPU.items():
            if name != "psi":
                out[i] = U[i].astype(np.float32).astype(np.float64)
    return out


def plane_scale(O, name):
    """Scale of the error of state plane `name`: the larger of its own and
    Im B's maximum (C and B share the beam's scale), pi for the phase plane
    (its errors are angles)."""
    if name == "phase":
        return np.pi
    return max(np.abs(O[name]).max(), np.abs(O["ImB"]).max())


def rel_err(a, b, scale=None):
    scale = np.abs(b).max() if scale is None else scale
    return np.abs(a - b).max() / max(scale, 1e-300)


def log(msg):
    print(msg, flush=True)
