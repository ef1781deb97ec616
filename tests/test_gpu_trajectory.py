"""GPU parity of the outer CG trajectory, not only of its end point.

The outer loop's coefficients alpha_k, beta_k, the permeability of the
recursive velocity at every iteration and the Lanczos estimate built from the
coefficients (Sec. 4.1.2, Ritz values of the CG tridiagonal) are compared
with the CPU oracle's.  Late CG coefficients depend on the rounding of the
inner solves (loss of orthogonality), so the comparison runs over the
"rounding horizon": the iterations before the first one at which the oracle's
own coefficients move by more than 1e-7 when its inner tolerance goes from
1e-12 to 1e-11 (ten times the inner error the GPU and the oracle leave).  Up to there the trajectory is fixed by the method and the GPU
must agree to 1e-6; beyond it, only the outer count (within one) and the
permeability (1e-6) are compared.  The Ritz values in the report must be the
extreme eigenvalues of the tridiagonal of the GPU's own coefficients.

Also here: the S-operator test hook against the oracle's operators, and the
2D square arrays of Sec. 4.2.1 run through the 3D library as boxes made of
copies of the image along z (the exact 3D solution is the 2D one), against
the 2D code that reproduces the paper's table of the 2D sweep.
"""

import json
import os
import sys

import numpy as np
import pytest

import oracle
from oracle.spectral2d import schur_pcg_2d, squares_2d
from synth import grf, spheres

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
HORIZON_RTOL = 1e-7
TRAJ_TOL = 1e-6


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_05266_amd as P
    P.load()
    return P


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def horizon(ha, hb, rtol=HORIZON_RTOL):
    """First iteration at which two trajectories' alpha or beta differ by more than rtol."""
    k = min(len(ha), len(hb))
    for j in range(k):
        if abs(ha[j, 5] - hb[j, 5]) > rtol * abs(ha[j, 5]):
            return j
        if j < k - 1 and abs(ha[j, 6] - hb[j, 6]) > rtol * abs(ha[j, 6]):
            return j
    return k


def ritz_extremes(alpha, beta):
    r = oracle.lanczos_ritz(alpha, beta)
    return float(r.min()), float(r.max())


def check_report_ritz(rep, hist):
    """The report's Ritz values are the extremes of T_k from its own coefficients."""
    lo, hi = ritz_extremes(hist[:, 5], hist[:, 6])
    assert rep["ritz_min"] == pytest.approx(lo, rel=1e-9)
    assert rep["ritz_max"] == pytest.approx(hi, rel=1e-9)
    assert rep["cond_est"] == pytest.approx(hi / lo, rel=2e-9)


def check_prefix(hist, alpha, beta, kcol, hz):
    """alpha, beta and k_hat of the first hz iterations agree with the oracle's."""
    n = min(hz, hist.shape[0])
    assert n > 0
    a = hist[:n, 5]
    np.testing.assert_allclose(a, alpha[:n], rtol=TRAJ_TOL, atol=0)
    m = min(n, hist.shape[0] - 1)   # the last row's beta is 0 when the loop stopped there
    np.testing.assert_allclose(hist[:m, 6], beta[:m], rtol=TRAJ_TOL, atol=0)
    np.testing.assert_allclose(hist[:n, 2], kcol[:n], rtol=TRAJ_TOL, atol=0)
    # the Ritz extremes of the tridiagonal over those iterations
    if n >= 2:
        g = ritz_extremes(a, hist[:n, 6])
        o = ritz_extremes(alpha[:n], beta[:n])
        assert g[0] == pytest.approx(o[0], rel=TRAJ_TOL)
        assert g[1] == pytest.approx(o[1], rel=TRAJ_TOL)
    return n


SMALL = [("spheres 24 r=4 phi=0.7 seed=0", lambda: spheres(24, 4.0, 0.7, 0)),
         ("spheres 24 r=4 phi=0.7 seed=1", lambda: spheres(24, 4.0, 0.7, 1)),
         ("spheres 37 r=2 phi=0.3 seed=4", lambda: spheres(37, 2.0, 0.3, 4))]


@pytest.mark.parametrize("case", range(len(SMALL)))
@pytest.mark.parametrize("pc", ["simple", "uzawa"])
def test_trajectory_against_oracle(P, case, pc):
    name, gen = SMALL[case]
    m = gen()
    pid = oracle.SIMPLE if pc == "simple" else oracle.UZAWA
    o = oracle.Oracle(m, (1.0, 0.0, 0.0))
    ra = o.solve(pid, tol=1e-8, eps_A=1e-12, eps_S=1e-12)
    rb = o.solve(pid, tol=1e-8, eps_A=1e-11, eps_S=1e-11)
    hz = horizon(ra["hist"], rb["hist"])
    gpid = P.STOKES_SIMPLE if pc == "simple" else P.STOKES_UZAWA
    with P.Stokes(m, (1.0, 0.0, 0.0)) as s:
        rep = s.solve(gpid, 1e-8)
        hist = s.history()
    say(f"[trajectory] {name} {pc}: outer gpu {rep['outer_iters']} oracle {ra['outer_iters']} horizon {hz} "
        f"cond gpu {rep['cond_est']:.6g} oracle {ra['cond_est']:.6g}")
    assert rep["status"] == 0
    assert abs(rep["outer_iters"] - ra["outer_iters"]) <= 1
    assert rep["k_hat"] == pytest.approx(ra["k_hat"], rel=1e-6)
    check_report_ritz(rep, hist)
    h = ra["hist"]
    n = check_prefix(hist, h[:, 5], h[:, 6], h[:, 2], hz)
    # the horizon is not trivially short: the comparison covers real iterations
    assert n >= min(10, ra["outer_iters"])


def _golden64():
    with open(os.path.join(HERE, "golden", "oracle_trajectories_64.json")) as f:
        return json.load(f)


GOLDEN_GEN = {"spheres N=64 r=4 phi=0.5 seed=11": lambda: spheres(64, 4.0, 0.5, 11),
              "grf N=64 corr=4 phi=0.35 seed=12": lambda: grf(64, 4.0, 0.35, 12)}


@pytest.mark.parametrize("idx", range(4))
def test_trajectory_64_against_stored_oracle(P, idx):
    """64^3: the tiled 64-wide columns and three multigrid levels are reached.
    The oracle's trajectories are stored by tests/golden/make_oracle_trajectories.py."""
    import hashlib
    case = _golden64()["cases"][idx]
    m = GOLDEN_GEN[case["name"]]()
    assert hashlib.sha256(np.ascontiguousarray(m).tobytes()).hexdigest()[:16] == case["mask_sha256_16"]
    gpid = P.STOKES_SIMPLE if case["precond"] == "simple" else P.STOKES_UZAWA
    with P.Stokes(m, (1.0, 0.0, 0.0)) as s:
        info = s.info()
        rep = s.solve(gpid, 1e-8)
        hist = s.history()
    say(f"[trajectory 64] {case['name']} {case['precond']}: outer gpu {rep['outer_iters']} oracle "
        f"{case['outer_iters']} horizon {case['horizon']} k gpu {rep['k_hat']:.14e} oracle {case['k_hat']:.14e}")
    assert info["mg_levels_S"] == 3 and info["mg_levels_A"] == 3
    assert rep["status"] == 0
    assert abs(rep["outer_iters"] - case["outer_iters"]) <= 1
    assert rep["k_hat"] == pytest.approx(case["k_hat"], rel=1e-6)
    check_report_ritz(rep, hist)
    n = check_prefix(hist, np.array(case["alpha"]), np.array(case["beta"]), np.array(case["k_col"]),
                     case["horizon"])
    assert n >= 10


def test_trajectory_128_against_stored_oracle(P):
    """128^3 sphere pack r=6 porosity 0.5 (the benchmark-size pack; four multigrid
    levels, one visit of level 1): outer count, k_hat and the CG coefficients up
    to the rounding horizon against the oracle's trajectory stored by
    tests/golden/make_oracle_trajectories.py --size 128 (the oracle needs about
    forty minutes per solve there)."""
    import hashlib
    with open(os.path.join(HERE, "golden", "oracle_trajectories_128.json")) as f:
        case = json.load(f)["cases"][0]
    m = spheres(128, 6.0, 0.5, 0)
    assert hashlib.sha256(np.ascontiguousarray(m).tobytes()).hexdigest()[:16] == case["mask_sha256_16"]
    with P.Stokes(m, (1.0, 0.0, 0.0)) as s:
        info = s.info()
        rep = s.solve(P.STOKES_SIMPLE, 1e-8)
        hist = s.history()
    say(f"[trajectory 128] {case['name']} {case['precond']}: outer gpu {rep['outer_iters']} oracle "
        f"{case['outer_iters']} horizon {case['horizon']} k gpu {rep['k_hat']:.14e} oracle {case['k_hat']:.14e}")
    assert info["mg_levels_S"] == 4 and info["mg_levels_A"] == 4
    assert rep["status"] == 0
    assert abs(rep["outer_iters"] - case["outer_iters"]) <= 1
    assert rep["k_hat"] == pytest.approx(case["k_hat"], rel=1e-6)
    check_report_ritz(rep, hist)
    n = check_prefix(hist, np.array(case["alpha"]), np.array(case["beta"]), np.array(case["k_col"]),
                     case["horizon"])
    assert n >= 10


def test_S_operator_hook_against_oracle(P):
    """STOKES_OP_S (B A^-1 B^T p with an inner solve at eps_A) against the oracle's
    B, B^T and inner A solve, on a multi-component geometry."""
    from synth import random_cell_field
    m = grf(40, 3.0, 0.35, 7)
    o = oracle.Oracle(m, (1.0, 0.0, 0.0))
    p = random_cell_field(40, 3)
    bt = o.apply(oracle.OP_BT, p)
    x, _ = o.inner_solve(0, bt, eps=1e-13)
    ref = o.apply(oracle.OP_B, x)
    with P.Stokes(m, (1.0, 0.0, 0.0)) as s:
        s.set_option("eps_A", 1e-13)
        got = s.apply(P.STOKES_OP_S, p)
    scale = np.abs(ref).max()
    say(f"[S hook] max |gpu - oracle| / max |oracle| = {np.abs(got - ref).max() / scale:.3e}")
    assert np.abs(got - ref).max() <= 1e-9 * scale


def extruded(m2):
    n = m2.shape[0]
    return np.ascontiguousarray(np.broadcast_to(m2[None, :, :], (n, n, n)))


@pytest.mark.parametrize("n_avg", [4, 8])
@pytest.mark.parametrize("pc", ["uzawa", "simple"])
def test_extruded_2d_squares_128(P, n_avg, pc):
    """4 x 4 randomly shifted squares in cells of 32 pixels (Sec. 4.2.1), copied along
    z into a 128^3 box, multigrid inner solves on the GPU; against the 2D outer PCG
    with exact inner solves at the paper's 2D stopping rule (1e-3 on ||r||/||r0||)
    and at 1e-8.  In 3D the SIMPLE matrix sees diag(A) = 6 + t, so the 2D reference
    uses that diagonal (diag_offset 2).  At 1e-3 the outer counts must be equal.  A
    1e-8 solve runs past the rounding horizon (module docstring), where the count
    depends on the inner solves' rounding (the oracle's own count moves by one when
    its inner tolerance goes from 1e-12 to 1e-10), so there the counts may differ by
    3 % (at least one) and the permeabilities must agree to 1e-6."""
    m2 = squares_2d(4, 32, n_avg, 2, seed=n_avg)
    m3 = extruded(m2)
    gpid = P.STOKES_SIMPLE if pc == "simple" else P.STOKES_UZAWA
    for tol in (1e-3, 1e-8):
        k2, perm2, _ = schur_pcg_2d(m2, pc, tol=tol, diag_offset=2.0 if pc == "simple" else 0.0)
        with P.Stokes(m3, (1.0, 0.0, 0.0), true_velocity=1) as s:
            info = s.info()
            rep = s.solve(gpid, tol)
        say(f"[extruded squares] n_avg={n_avg} {pc} tol={tol}: outer gpu {rep['outer_iters']} 2d {k2} "
            f"k_vox gpu {rep['k_vox']:.12e} 2d {perm2:.12e}")
        assert info["mg_levels_S"] >= 3 and info["mg_levels_A"] >= 3
        assert rep["status"] == 0
        assert abs(rep["outer_iters"] - k2) <= (0 if tol > 1e-6 else max(1, int(0.03 * k2)))
        assert rep["k_vox"] == pytest.approx(perm2, rel=1e-6)
        assert abs(rep["mean_u"][2]) < 1e-12 * rep["mean_u"][0]
