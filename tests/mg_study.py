"""CPU study of the inner solves' multigrid cycle (not collected by pytest).

Runs PCG with a scipy model of the V-cycle on the SIMPLE matrix and on the
three planes of A, built from the oracle's assembled matrices, to compare the
library's cycle with variants it does not build: Gauss-Seidel smoothing on
more levels, and coarse levels whose 2x2x2 aggregates are split into their
connected pieces (so disconnected pores are not merged).  Every variant uses
the library's level rule (halve while the side is even, at least 2 and above
512 nodes), the library's damping (0.9), coarse-correction scales (1.7 for the
SIMPLE matrix, 1.5 for A) and 8 coarsest sweeps, so only the smoother or the
aggregation differs.  PCG stops on ||D^-1 r|| / ||D^-1 r0|| < 1e-12, as the
inner solves do; the right-hand side is seeded noise (mean-free for the
SIMPLE matrix).

    python tests/mg_study.py            # writes profiles/multigrid_cpu_study.md
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OMEGA, SWEEPS, TILED_MIN_SIDE, TOL = 0.9, 8, 64, 1e-12
# name: (level-0 smoother, coarse smoother, split coarse aggregates, deeper levels)
VARIANTS = {
    "library cycle": ("jacobi", "gs<64", False, False),
    "Jacobi everywhere (mg_coarse_gs=0)": ("jacobi", "jacobi", False, False),
    "Gauss-Seidel on every coarse level (mg_coarse_gs=2)": ("jacobi", "gs", False, False),
    "Gauss-Seidel on level 0 too (not built)": ("gs", "gs<64", False, False),
    "split aggregates on the coarse levels (not built)": ("jacobi", "gs<64", True, False),
    "split aggregates, levels continued while above 512 unknowns (not built)": ("jacobi", "gs<64", True, True),
}


def level_sides(N):
    ns, n = [N], N
    while n % 2 == 0 and n // 2 >= 2 and n ** 3 > 512:
        n //= 2
        ns.append(n)
    return ns


def hierarchy(A0, pos, N, split, deep=False):
    """Levels [(side, A, 1/D, black mask)] over the unknowns, and prolongations.
    pos: grid positions (i + n (j + n k)) of the level-0 unknowns.  deep: keep
    halving while the side is even and a level holds more than 512 unknowns
    (split aggregates leave more than the structured rule counts)."""
    levels, Ps = [], []
    A = A0.tocsr()
    ns = level_sides(N)
    if deep:
        ns, n = [N], N
        while n % 2 == 0 and n // 2 >= 2:
            n //= 2
            ns.append(n)
    for l, n in enumerate(ns):
        i, j, k = pos % n, (pos // n) % n, pos // (n * n)
        d = A.diagonal()
        inv = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
        levels.append((n, A, inv, ((i + j + k) & 1).astype(bool)))
        if l + 1 == len(ns) or (deep and A.shape[0] <= 512):
            break
        h = n // 2
        block = (i // 2) + h * ((j // 2) + h * (k // 2))
        if split and l >= 1:
            # connected pieces of each block: couplings inside the block only
            C = A.tocoo()
            inside = (block[C.row] == block[C.col]) & (C.row != C.col) & (C.data != 0)
            G = sp.csr_matrix((np.ones(int(inside.sum())), (C.row[inside], C.col[inside])), shape=A.shape)
            _, agg = csg.connected_components(G, directed=False)
        else:
            _, agg = np.unique(block, return_inverse=True)
        nc = int(agg.max()) + 1
        P = sp.csr_matrix((np.ones(A.shape[0]), (np.arange(A.shape[0]), agg)), shape=(A.shape[0], nc))
        cpos = np.zeros(nc, dtype=np.int64)
        cpos[agg] = block                       # an aggregate's block coordinates on the next level
        Ps.append(P)
        A = (P.T @ A @ P).tocsr()
        pos = cpos
    return levels, Ps


def relax(A, inv, x, b, mask):
    """Each node of `mask` (no two of them coupled) solves its own row."""
    off = A - sp.diags(A.diagonal())
    y = x.copy()
    y[mask] = (inv * (b - off @ x))[mask]
    return y


def cycle(levels, Ps, b, level0, coarse, scale, l=0):
    n, A, inv, black = levels[l]
    if l == len(levels) - 1:
        x = OMEGA * inv * b
        for _ in range(SWEEPS - 1):
            x = x + OMEGA * inv * (b - A @ x)
        return x
    kind = level0 if l == 0 else ("gs" if coarse == "gs" or (coarse == "gs<64" and n < TILED_MIN_SIDE) else "jacobi")
    if kind == "gs":
        x = relax(A, inv, relax(A, inv, np.zeros_like(b), b, ~black), b, black)
    else:
        x = OMEGA * inv * b
    x = x + scale * (Ps[l] @ cycle(levels, Ps, Ps[l].T @ (b - A @ x), level0, coarse, scale, l + 1))
    if kind == "gs":
        return relax(A, inv, relax(A, inv, x, b, black), b, ~black)
    return x + OMEGA * inv * (b - A @ x)


def pcg(A, b, M, maxit=5000):
    dinv = 1.0 / A.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    r0 = np.linalg.norm(dinv * r)
    for it in range(1, maxit + 1):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(dinv * r) / r0 < TOL:
            return it
        z = M(r)
        rz2 = r @ z
        p = z + (rz2 / rz) * p
        rz = rz2
    return -1


def operators(mask):
    """SIMPLE matrix over the unknown cells and A over the unknown faces of each plane."""
    import oracle
    o = oracle.Oracle(mask)
    N = mask.shape[0]
    fpos, cpos = o.unknowns()
    A = o.csr("A")
    B = o.csr("B")
    S = (B @ sp.diags(1.0 / A.diagonal()) @ B.T).tocsr()
    planes = []
    for p in range(3):
        sel = np.nonzero(fpos // N ** 3 == p)[0]
        planes.append((A[sel][:, sel].tocsr(), fpos[sel] - p * N ** 3))
    return N, (S, cpos), planes


def study(cases, out=None, with_A=("sph128", "tight128")):
    from synth import grf, spheres
    gens = {"sph128": ("128^3 spheres r=6 porosity 0.5 (the benchmark)", lambda: spheres(128, 6.0, 0.5, 0)),
            "tight128": ("128^3 spheres r=3 porosity 0.2", lambda: spheres(128, 3.0, 0.2, 0)),
            "grf128": ("128^3 GRF corr length 8 porosity 0.2", lambda: grf(128, 8.0, 0.2, 0))}
    rows = []
    for name in cases:
        desc, gen = gens[name]
        N, (S, cpos), planes = operators(gen())
        rng = np.random.default_rng(0)
        bS = rng.standard_normal(S.shape[0])
        bS -= bS.mean()
        bA = [rng.standard_normal(Ap.shape[0]) for Ap, _ in planes]
        Ablk = sp.block_diag([Ap for Ap, _ in planes]).tocsr()
        for vname, (level0, coarse, split, deep) in VARIANTS.items():
            t = time.time()
            lv, Ps = hierarchy(S, cpos, N, split, deep)
            its_S = pcg(S, bS, lambda r: cycle(lv, Ps, r, level0, coarse, 1.7))
            its_A = None
            if name in with_A:
                hier = [hierarchy(Ap, pos, N, split, deep) for Ap, pos in planes]
                cuts = np.cumsum([0] + [Ap.shape[0] for Ap, _ in planes])

                def MA(r):
                    return np.concatenate([cycle(h[0], h[1], r[cuts[q]:cuts[q + 1]], level0, coarse, 1.5)
                                           for q, h in enumerate(hier)])
                its_A = pcg(Ablk, np.concatenate(bA), MA)
            rows.append((desc, vname, [L[1].shape[0] for L in lv], its_S, its_A))
            print(f"{desc} | {vname}: SIMPLE {its_S}, A {its_A} ({time.time() - t:.0f} s)", flush=True)
    if out:
        L = ["# Multigrid cycle variants on the CPU: PCG iterations of the inner solves", "",
             "Command (repository root): `python tests/mg_study.py`", "",
             "scipy model of the inner solves' V-cycle on the oracle's assembled SIMPLE matrix and the three planes",
             "of A; the library's level rule, damping 0.9, scales 1.7 (SIMPLE) and 1.5 (A), 8 coarsest sweeps;",
             "PCG to ||D^-1 r|| / ||D^-1 r0|| < 1e-12 from seeded noise. 'not built': variants the GPU library",
             "does not implement.", "",
             "| Geometry | Cycle | unknowns per level (SIMPLE matrix) | SIMPLE iterations | A iterations |",
             "|---|---|---|---|---|"]
        for desc, vname, sizes, its_S, its_A in rows:
            L.append(f"| {desc} | {vname} | {sizes} | {its_S} | {'' if its_A is None else its_A} |")
        with open(out, "w") as fh:
            fh.write("\n".join(L) + "\n")
    return rows


if __name__ == "__main__":
    import oracle
    oracle.build(force=False)
    study(["sph128", "tight128", "grf128"], out=os.path.join(ROOT, "profiles", "multigrid_cpu_study.md"))
