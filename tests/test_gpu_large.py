"""The large workloads at their full sizes, checked where the oracle can check
them: residual rows of the discrete system evaluated one by one by the oracle
at sampled faces and cells (no matrix at these sizes is assembled), the
permeability re-derived from the returned velocity, and the mixed-precision
permeability against the FP64 GPU solve of the same geometry (bar 1e-4).

- 256^3 overlapping spheres r = 3, porosity 0.2 (surface-to-volume above the
  paper's range; ~43 k components, one conducts), SIMPLE, mixed and FP64;
- 512^3 Gaussian random field, correlation length 8, porosity 0.15, SIMPLE,
  mixed (about two minutes; marked `long`, which selects it but does not skip it).
"""

import sys

import numpy as np
import pytest

import oracle
from synth import grf, spheres

pytestmark = pytest.mark.gpu

TOL = 1e-8


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


def check_solution(s, rep, light, rng, nface=400000, ncell=200000):
    """Sampled oracle residual rows and the flux average of the returned fields."""
    N = s.N
    p, u = s.fields()
    fpos = rng.integers(0, 3 * N ** 3, nface)
    cpos = rng.integers(0, N ** 3, ncell)
    rf, rc = oracle.sample_residuals(light, u, p, fpos, cpos)
    act, fl = ~np.isnan(rf), ~np.isnan(rc)
    rms_f, rms_c = np.sqrt(np.mean(rf[act] ** 2)), np.sqrt(np.mean(rc[fl] ** 2))
    nc = int(light.nfluid)
    say(f"    sampled {act.sum()} faces: momentum rms {rms_f:.2e}; {fl.sum()} cells: continuity rms {rms_c:.2e} "
        f"(reported ||Bu||/sqrt(cells) {rep['div_norm'] / np.sqrt(nc):.2e})")
    assert act.sum() > 1000 and fl.sum() > 1000
    # momentum: the velocity solves A u = f - B^T p far below the outer tolerance
    assert rms_f < TOL
    # continuity: ||B u|| meets the outer tolerance, and the sampled rows agree with it
    assert rep["div_norm"] <= 1.01 * TOL * rep["r0_norm"]
    assert rms_c <= 2.0 * rep["div_norm"] / np.sqrt(nc)
    # permeability = N^-3 sum of the x-velocity over the box, over N^2
    assert rep["k_hat"] == pytest.approx(u[0].sum() / N ** 3 / N ** 2, rel=1e-12)


def test_tight_spheres_256_mixed_and_fp64(P):
    m = spheres(256, 3.0, 0.2, 0)
    say("[large] spheres 256^3 r=3 porosity 0.2 seed 0")
    light = oracle.Oracle(m, assemble=False)
    assert light.ncomp_all > 10000 and light.ncomp_kept == 1
    rng = np.random.default_rng(5)
    with P.Stokes(m) as s:
        s.set_option("precision", 1)
        rm = s.solve(P.STOKES_SIMPLE, TOL)
        say(f"    mixed k={rm['k_hat']:.14e} outer={rm['outer_iters']} t={rm['seconds']:.1f}s")
        assert rm["status"] == 0
        check_solution(s, rm, light, rng)
        s.set_option("precision", 0)
        r64 = s.solve(P.STOKES_SIMPLE, TOL)
        say(f"    fp64  k={r64['k_hat']:.14e} outer={r64['outer_iters']} t={r64['seconds']:.1f}s")
        assert r64["status"] == 0
        check_solution(s, r64, light, rng)
    # level 1 (128^3) is visited twice by the SIMPLE matrix's cycle (estimate 1.62 < 1.8)
    assert rm["flags"] & P.STOKES_FLAG_MG_TWO_VISITS and r64["flags"] & P.STOKES_FLAG_MG_TWO_VISITS
    assert abs(rm["k_hat"] - r64["k_hat"]) <= 1e-4 * r64["k_hat"]
    assert abs(rm["outer_iters"] - r64["outer_iters"]) <= 10


def test_spheres_224_partial_coarse_tiles(P):
    """224^3: the first coarse level (112^3) runs the tiled coarse kernels on
    64-wide columns whose second tile runs past the level's edge."""
    m = spheres(224, 4.0, 0.4, 3)
    say("[large] spheres 224^3 r=4 porosity 0.4 seed 3")
    light = oracle.Oracle(m, assemble=False)
    with P.Stokes(m, precision=1) as s:
        assert s.info()["mg_levels_S"] == 5
        r = s.solve(P.STOKES_SIMPLE, TOL)
        say(f"    mixed k={r['k_hat']:.14e} outer={r['outer_iters']} t={r['seconds']:.1f}s")
        assert r["status"] == 0
        check_solution(s, r, light, np.random.default_rng(7))
        s.set_option("precision", 0)
        r64 = s.solve(P.STOKES_SIMPLE, TOL)
        assert r64["status"] == 0
    # level 1 (112^3) is below the two-visit side: one visit
    assert not (r["flags"] & P.STOKES_FLAG_MG_TWO_VISITS)
    assert abs(r["k_hat"] - r64["k_hat"]) <= 1e-4 * r64["k_hat"]


@pytest.mark.long
def test_grf_512_mixed(P):
    m = grf(512, 8.0, 0.15, 0)
    say("[large] GRF 512^3 corr length 8 porosity 0.15 seed 0")
    light = oracle.Oracle(m, assemble=False)
    with P.Stokes(m, precision=1, progress=40) as s:
        r = s.solve(P.STOKES_SIMPLE, TOL)
        say(f"    mixed k={r['k_hat']:.14e} outer={r['outer_iters']} t={r['seconds']:.1f}s")
        assert r["status"] == 0
        # two visits of level 1, with the corrections below it scaled 1.3 (the estimate
        # with 1.7 is 3.29, with 1.3 1.64)
        assert r["flags"] & P.STOKES_FLAG_MG_TWO_VISITS
        check_solution(s, r, light, np.random.default_rng(6))
