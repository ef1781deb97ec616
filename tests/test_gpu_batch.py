"""Batched contexts (stokes_setup_batch): several geometries of one size in one
context, every kernel launch advancing all of them.  Each member's result must be
bitwise the same as when it is solved alone (a batch of one) and whatever the
order of the members, and must match the CPU oracle to the mixed-precision bar.
"""

import sys

import numpy as np
import pytest

import oracle
from synth import grf, slits, spheres

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-4


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


def members32():
    return [spheres(32, 3.0, 0.5, 1), grf(32, 4.0, 0.35, 2), spheres(32, 2.0, 0.3, 3),
            slits(32, [3, 5, 7], axis=2),           # several conducting components, g along x exact
            spheres(32, 4.0, 0.7, 5), grf(32, 6.0, 0.45, 6)]


KEYS = ("status", "flags", "outer_iters", "inner_A_iters", "inner_S_iters", "k_hat", "k_vox", "rel_res",
        "div_norm", "r0_norm", "cond_est")


def same_report(a, b):
    for k in KEYS:
        va, vb = a[k], b[k]
        if isinstance(va, float) and np.isnan(va) and np.isnan(vb):
            continue
        assert va == vb, (k, va, vb)


@pytest.mark.parametrize("pc", ["simple", "uzawa"])
def test_member_alone_equals_member_in_batch(P, pc):
    masks = members32()
    with P.StokesBatch(masks) as b:
        reps = b.solve(pc, 1e-8)
        fields = [b.result(m, fields=True) for m in range(len(masks))]
    for m, mask in enumerate(masks):
        with P.StokesBatch([mask]) as one:
            r1 = one.solve(pc, 1e-8)[0]
            _, p1, u1 = one.result(0, fields=True)
        say(f"[batch] {pc} member {m}: outer {reps[m]['outer_iters']} k_hat {reps[m]['k_hat']:.15e} "
            f"alone {r1['k_hat']:.15e}")
        same_report(reps[m], r1)
        assert np.array_equal(fields[m][1], p1) and np.array_equal(fields[m][2], u1)


def test_member_order_does_not_matter(P):
    masks = members32()
    order = [4, 1, 5, 0, 3, 2]
    with P.StokesBatch(masks) as b:
        a = b.solve("simple", 1e-8)
    with P.StokesBatch([masks[i] for i in order]) as b:
        c = b.solve("simple", 1e-8)
    for j, i in enumerate(order):
        same_report(a[i], c[j])


def test_batch_members_against_oracle(P):
    masks = members32()
    with P.StokesBatch(masks) as b:
        reps = b.solve("simple", 1e-8)
        us = [b.result(m, fields=True)[2] for m in range(len(masks))]
    for m, mask in enumerate(masks):
        ref = oracle.Oracle(mask, (1.0, 0.0, 0.0)).solve(oracle.SIMPLE, tol=1e-8)
        rel = abs(reps[m]["k_hat"] - ref["k_hat"]) / abs(ref["k_hat"])
        say(f"[batch vs oracle] member {m}: k gpu {reps[m]['k_hat']:.12e} oracle {ref['k_hat']:.12e} rel {rel:.2e}")
        assert reps[m]["status"] == 0
        assert rel <= MIXED_TOL
        assert np.abs(us[m] - ref["u"]).max() <= MIXED_TOL * np.abs(ref["u"]).max()
    # the slit member: channels along the force, g = 0, no outer step
    assert reps[3]["outer_iters"] == 0 and reps[3]["flags"] & P.STOKES_FLAG_ZERO_RHS


def test_batch_with_a_member_without_flow(P):
    """A member whose fluid does not conduct along the force has k = 0 exactly and
    does not disturb the others."""
    masks = [spheres(24, 3.0, 0.5, 7), slits(24, 4, axis=0), spheres(24, 3.0, 0.5, 8)]
    with P.StokesBatch(masks) as b:
        reps = b.solve("simple", 1e-8)
    assert reps[1]["k_hat"] == 0.0 and reps[1]["flags"] & P.STOKES_FLAG_NO_FLOW
    for m in (0, 2):
        with P.StokesBatch([masks[m]]) as one:
            same_report(reps[m], one.solve("simple", 1e-8)[0])


def test_batch_sizes_with_hierarchy_and_limits(P):
    """48^3 and 64^3 members (deeper hierarchies, 64-wide tiles); a batch of the
    maximum size; refused operations."""
    from paper_2307_05266_amd.stokes import StokesError
    for N in (48, 64):
        masks = [spheres(N, 3.0, 0.45, 10 + i) for i in range(3)]
        with P.StokesBatch(masks) as b:
            reps = b.solve("simple", 1e-8)
        with P.StokesBatch([masks[1]]) as one:
            same_report(reps[1], one.solve("simple", 1e-8)[0])
    masks = [spheres(16, 2.0, 0.5, 100 + i) for i in range(32)]
    with P.StokesBatch(masks) as b:
        reps = b.solve("simple", 1e-8)
        assert all(r["status"] == 0 for r in reps)
        with pytest.raises(StokesError):
            b.set_option("precision", 0)
        import torch
        x = torch.zeros(3 * 16 ** 3, dtype=torch.float64, device="cuda")
        with pytest.raises(StokesError):
            P.stokes_apply_device(b._ctx, P.STOKES_OP_A, x, x)
    with P.StokesBatch([masks[31]]) as one:
        same_report(reps[31], one.solve("simple", 1e-8)[0])
    with pytest.raises(StokesError):
        P.StokesBatch([spheres(16, 2.0, 0.5, 0)] * 33)
