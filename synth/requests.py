"""Seeded request stream of the serving workload.

Request i (seed = base + i) draws, from numpy default_rng(base + i):
geometry kind (overlapping spheres or thresholded Gaussian random field, 50/50),
box side N uniform over {32, 48, 64, 96, 128}, porosity uniform on
[0.15, 0.6], and a sphere radius uniform over {2, ..., 6} voxels or a
correlation length uniform on [4, 12] voxels; the geometry itself is generated
with seed base + i.  Every request is a unit force along x, solved with the
SIMPLE preconditioner in mixed precision to tol 1e-8.
"""

from __future__ import annotations

import numpy as np

from .geometry import grf, spheres

SIDES = (32, 48, 64, 96, 128)


def request_params(i: int, base: int = 1000) -> dict:
    rng = np.random.default_rng(base + i)
    kind = "spheres" if rng.integers(2) == 0 else "grf"
    N = int(SIDES[rng.integers(len(SIDES))])
    phi = float(rng.uniform(0.15, 0.6))
    p = {"index": i, "seed": base + i, "kind": kind, "N": N, "porosity": phi}
    if kind == "spheres":
        p["radius"] = int(rng.integers(2, 7))
    else:
        p["corr_len"] = float(rng.uniform(4.0, 12.0))
    return p


def request_mask(p: dict) -> np.ndarray:
    if p["kind"] == "spheres":
        return spheres(p["N"], float(p["radius"]), p["porosity"], p["seed"])
    return grf(p["N"], p["corr_len"], p["porosity"], p["seed"])


def make_request(i: int, base: int = 1000):
    """(params, mask) of request i."""
    p = request_params(i, base)
    return p, request_mask(p)
