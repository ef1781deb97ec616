"""Write oracle_trajectories_64.json (default) or oracle_trajectories_128.json
(`--size 128`): the CPU oracle's outer CG trajectories on 64^3 geometries and on
the 128^3 sphere pack r=6 porosity 0.5, for GPU parity tests at sizes the
oracle needs minutes per solve for (too slow to run inside the GPU test suite).

Calls only `oracle/` and the seeded input generators of `synth/`.  For each
case the oracle solves twice, with inner tolerances 1e-12 (the GPU's) and
1e-11; the iterations before the first one at which the two runs' alpha or
beta differ by more than 1e-7 (relative) form the "rounding horizon": up to
there the trajectory is fixed by the method, beyond it by the rounding of the
inner solves (late CG coefficients are sensitive to perturbations, the
classical loss of orthogonality).  Stored per case: outer count, k_hat, the
alpha, beta, k_hat and relative-residual columns up to the horizon, the
extreme Ritz values of the tridiagonal built from those iterations and from
all of them (Lanczos, Sec. 4.1.2), and a hash of the mask.

    python tests/golden/make_oracle_trajectories.py [--size 128]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import grf, spheres  # noqa: E402

HORIZON_RTOL = 1e-7

CASES = {
    64: [
        # (name, generator call, preconditioners)
        ("spheres N=64 r=4 phi=0.5 seed=11", lambda: spheres(64, 4.0, 0.5, 11), ("simple", "uzawa")),
        ("grf N=64 corr=4 phi=0.35 seed=12", lambda: grf(64, 4.0, 0.35, 12), ("simple", "uzawa")),
    ],
    128: [
        ("spheres N=128 r=6 phi=0.5 seed=0", lambda: spheres(128, 6.0, 0.5, 0), ("simple",)),
    ],
}


def mask_hash(m):
    return hashlib.sha256(np.ascontiguousarray(m, dtype=np.uint8).tobytes()).hexdigest()[:16]


def horizon(ha, hb):
    k = min(len(ha), len(hb))
    for j in range(k):
        da = abs(ha[j, 5] - hb[j, 5]) / abs(ha[j, 5])
        last = j == k - 1
        db = 0.0 if last else abs(ha[j, 6] - hb[j, 6]) / abs(ha[j, 6])
        if da > HORIZON_RTOL or db > HORIZON_RTOL:
            return j
    return k


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=64, choices=sorted(CASES))
    size = ap.parse_args().size
    out_path = os.path.join(HERE, f"oracle_trajectories_{size}.json")
    out = {"source": "written by tests/golden/make_oracle_trajectories.py from the CPU oracle (FP64, Jacobi-PCG "
                     "inner solves); force (1, 0, 0), outer tol 1e-8 on ||r||/||r0||",
           "horizon_rtol": HORIZON_RTOL, "cases": []}
    for name, gen, pcs in CASES[size]:
        m = gen()
        o = oracle.Oracle(m, (1.0, 0.0, 0.0))
        for pc in pcs:
            pid = oracle.SIMPLE if pc == "simple" else oracle.UZAWA
            t0 = time.perf_counter()
            a = o.solve(pid, tol=1e-8, eps_A=1e-12, eps_S=1e-12)
            b = o.solve(pid, tol=1e-8, eps_A=1e-11, eps_S=1e-11)
            ha, hb = a["hist"], b["hist"]
            hz = horizon(ha, hb)
            pre = oracle.lanczos_ritz(ha[:hz, 5], ha[:hz, 6]) if hz > 0 else np.zeros(0)
            case = {
                "name": name, "precond": pc, "mask_sha256_16": mask_hash(m), "N": int(m.shape[0]),
                "outer_iters": a["outer_iters"], "outer_iters_eps11": b["outer_iters"],
                "k_hat": a["k_hat"], "k_hat_eps11": b["k_hat"],
                "horizon": hz,
                "alpha": ha[:hz, 5].tolist(), "beta": ha[:hz, 6].tolist(),
                "k_col": ha[:hz, 2].tolist(), "rel": ha[:hz, 0].tolist(),
                "ritz_prefix": [float(pre.min()), float(pre.max())] if hz > 0 else None,
                "ritz": [float(a["ritz"].min()), float(a["ritz"].max())],
                "ritz_eps11": [float(b["ritz"].min()), float(b["ritz"].max())],
                "components_kept": o.ncomp_kept,
            }
            out["cases"].append(case)
            print(f"{name} {pc}: outer {a['outer_iters']}/{b['outer_iters']} horizon {hz} "
                  f"k {a['k_hat']:.14e} ({time.perf_counter() - t0:.0f} s)", flush=True)
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
