"""CPU checks of the two-visit multigrid cycle on the scipy model that the GPU
V-cycle is compared with element by element (tests/test_gpu_multigrid.py).

The second visit of level 1 cycles on the residual the first leaves and adds
its result: on level 1 that is the operator 2 B1 - B1 A1 B1 (B1: the cycle from
level 1 down, A1: the level-1 Galerkin operator), whose eigenvalues relative to
A1 are 1 - (1 - mu)^2 for the eigenvalues mu of B1 A1.  Checked here on a small
sphere pack with dense matrices: the model's two-visit level-1 operator equals
that product form, its eigenvalues follow the relation, and the whole two-visit
cycle is symmetric and positive definite on the range of the SIMPLE matrix when
max mu < 2 (the condition the library's set-up estimate tests)."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth import spheres
from test_gpu_multigrid import SCALE_S, cycle, embed, hierarchy, mg_plan

N = 20   # levels 20 -> 10 -> 5: level 1 is not the coarsest


@pytest.fixture(scope="module")
def model():
    m = spheres(N, 3.0, 0.45, 4)
    o = oracle.Oracle(m)
    n3 = N ** 3
    _, cpos = o.unknowns()
    B = o.csr("B")
    dA = o.csr("A").diagonal()
    Sh = embed((B @ sp.diags(1.0 / dA) @ B.T).tocsr(), cpos, n3)
    lv, Ps = hierarchy(Sh, mg_plan(N, 1))
    assert [x[0] for x in lv] == [20, 10, 5]
    return Sh, cpos, lv, Ps


def dense_op(f, idx, n):
    """Matrix of a linear map restricted to the coordinates idx (columns = images of unit vectors)."""
    M = np.zeros((len(idx), len(idx)))
    for j, c in enumerate(idx):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, j] = f(e)[idx]
    return M


def test_second_visit_is_2B_minus_BAB(model):
    _, _, lv, Ps = model
    n1, A1, inv1 = lv[1]
    idx = np.nonzero(inv1 > 0)[0]
    B1 = dense_op(lambda b: cycle(lv, Ps, b, 1, SCALE_S, l=1), idx, n1 ** 3)
    A = A1.toarray()[np.ix_(idx, idx)]

    def two(b):
        # the model's second visit, as the V-cycle test applies it inside level 0
        x = cycle(lv, Ps, b, 1, SCALE_S, l=1)
        w = np.where(inv1 > 0, b - A1 @ x, 0.0)
        return x + cycle(lv, Ps, w, 1, SCALE_S, l=1)

    M1 = dense_op(two, idx, n1 ** 3)
    ref = 2.0 * B1 - B1 @ A @ B1
    assert np.abs(M1 - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(B1 - B1.T).max() <= 1e-12 * np.abs(B1).max()        # the level-1 cycle is symmetric
    # eigenvalues relative to A1 (on its range): 1 - (1 - mu)^2
    mu = np.sort(np.linalg.eigvals(B1 @ A).real)
    nu = np.sort(np.linalg.eigvals(M1 @ A).real)
    assert np.allclose(np.sort(1.0 - (1.0 - mu) ** 2), nu, atol=1e-9)
    assert mu.max() < 2.0


def test_two_visit_cycle_is_spd_on_the_range(model):
    Sh, cpos, lv, Ps = model
    n3 = N ** 3
    M = dense_op(lambda b: cycle(lv, Ps, b, 1, SCALE_S, visits=2), cpos, n3)
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    S = Sh.toarray()[np.ix_(cpos, cpos)]
    # on the range of the singular SIMPLE matrix: eigenvalues of M S are real and positive
    lam = np.linalg.eigvals(M @ S).real
    big = np.abs(lam) > 1e-10 * np.abs(lam).max()
    assert (lam[big] > 0).all()
