"""GPU parity of the Schur solve with a given right-hand side g = B xi
(stokes_solve_rhs): the random-consistent-RHS runs of the slit-stack
workload, whose outer counts are read against the surface-to-volume ratio.
g is formed by the oracle's B from a seeded face field and handed to both
sides; outer counts (within one) and the pressure (per-component zero mean,
1e-6 relative) are compared."""

import sys

import numpy as np
import pytest

import oracle
from synth import random_face_field, slits, spheres

pytestmark = pytest.mark.gpu


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


CASES = [("slits 48 W=3,4,6 walls normal to y", lambda: slits(48, [3, 4, 6], axis=1)),
         ("slits 64 W=8 walls normal to y", lambda: slits(64, 8, axis=1)),
         ("spheres 40 r=3 phi=0.5", lambda: spheres(40, 3.0, 0.5, 11))]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("pc", ["uzawa", "simple"])
def test_given_rhs_against_oracle(P, case, pc):
    name, gen = CASES[case]
    m = gen()
    N = m.shape[0]
    o = oracle.Oracle(m, (1.0, 0.0, 0.0))
    g = o.apply(oracle.OP_B, random_face_field(N, 7 + case))
    pid = oracle.SIMPLE if pc == "simple" else oracle.UZAWA
    ref = o.solve(pid, tol=1e-8, g=g)
    with P.Stokes(m, (1.0, 0.0, 0.0)) as s:
        rep = s.solve_rhs(g, pc, 1e-8)
        p, u = s.fields()
    say(f"[given rhs] {name} {pc}: outer gpu {rep['outer_iters']} oracle {ref['outer_iters']} "
        f"comps {rep['n_components_kept']}")
    assert rep["status"] == 0 and ref["status"] == 0
    assert rep["outer_iters"] > 0
    assert abs(rep["outer_iters"] - ref["outer_iters"]) <= 1
    scale = np.abs(ref["p"]).max()
    assert np.abs(p - ref["p"]).max() <= 1e-6 * scale
    assert rep["r0_norm"] == pytest.approx(ref["r0"], rel=1e-12)
    # the velocity of the loop is -A^-1 B^T p: its divergence is -g + (residual)
    bu = o.apply(oracle.OP_B, u)
    assert np.abs(bu + g).max() <= 1e-6 * np.abs(g).max()


def test_given_rhs_refused_where_not_built(P):
    from paper_2307_05266_amd.stokes import StokesError
    m = spheres(16, 2.0, 0.5, 3)
    with P.Stokes(m, precision=1) as s:
        with pytest.raises(StokesError) as e:
            s.solve_rhs(np.zeros((16, 16, 16)))
        assert e.value.status == P.STOKES_E_STATE
