"""The entry point that allocates nothing, stokes_apply_device_noalloc, called
through the C ABI and compared bitwise with stokes_apply_device (same kernels,
scratch in the library's fixed device array instead of the context's work
vectors): on two calls in a row, the second on a smaller box, with several
components (per-component partial sums in the scratch) and with one, plus the
size limit and the operators it does not take."""

import sys

import numpy as np
import pytest

from synth import slits, spheres

pytestmark = pytest.mark.gpu

OPS = ["A", "B", "BT", "SHAT", "DIAG_A", "DIAG_SHAT", "PROJECT"]


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


def _compare_all_ops(P, mask, keep_all, seed):
    import torch

    from paper_2307_05266_amd.stokes import _op_shapes
    N = mask.shape[0]
    gen = torch.Generator().manual_seed(seed)
    with P.Stokes(mask, (1.0, 0.0, 0.0), keep_all=keep_all) as s:
        say(f"[no-alloc] N={N} keep_all={keep_all} components kept={s.info()['ncomp_kept']}")
        for name in OPS:
            op = getattr(P, "STOKES_OP_" + name)
            nin, nout, _ = _op_shapes(op, N)
            # unmasked random input: entries off the unknowns must be ignored
            x = torch.randn(nin, dtype=torch.float64, generator=gen).cuda()
            ref = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
            out = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
            s.apply_device(op, x, ref)
            s.apply_device_noalloc(op, x, out)
            torch.cuda.synchronize()
            assert not torch.isnan(ref).any(), name
            assert torch.equal(out, ref), f"{name} at N={N}"
            assert torch.count_nonzero(out) > 0, name
        # the projection in place (in == out)
        x = torch.randn(N ** 3, dtype=torch.float64, generator=gen).cuda()
        ref = torch.empty_like(x)
        s.apply_device(P.STOKES_OP_PROJECT, x, ref)
        s.apply_device_noalloc(P.STOKES_OP_PROJECT, x, x)
        torch.cuda.synchronize()
        assert torch.equal(x, ref)


def test_noalloc_matches_apply_device_twice_smaller_second(P):
    # several kept components (one per channel), then a smaller one-component box
    _compare_all_ops(P, slits(48, [4, 6, 9], axis=1), True, 1)
    _compare_all_ops(P, spheres(24, 4.0, 0.7, 0), False, 2)
    # and back up, after the smaller call left its values in the array
    _compare_all_ops(P, spheres(40, 3.0, 0.5, 3), False, 3)


def test_noalloc_limit_and_unsupported_ops(P):
    import torch
    N = 112   # 3 N^3 doubles exceed 32 MiB; N^3 doubles do not
    mask = spheres(N, 6.0, 0.6, 4)
    with P.Stokes(mask, (1.0, 0.0, 0.0)) as s:
        x = torch.ones(3 * N ** 3, dtype=torch.float64, device="cuda")
        out = torch.full((3 * N ** 3,), 7.0, dtype=torch.float64, device="cuda")
        st = s.apply_device_noalloc(P.STOKES_OP_A, x, out, ok=(P.STOKES_E_LIMIT,))
        assert st == P.STOKES_E_LIMIT
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())          # no device work was done
        # B^T at the same size fits, and matches the existing entry point
        p = torch.randn(N ** 3, dtype=torch.float64).cuda()
        ref = torch.empty(3 * N ** 3, dtype=torch.float64, device="cuda")
        s.apply_device(P.STOKES_OP_BT, p, ref)
        s.apply_device_noalloc(P.STOKES_OP_BT, p, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        for op in (P.STOKES_OP_S, P.STOKES_OP_MG_SHAT, P.STOKES_OP_MG_A, 99, -1):
            st = s.apply_device_noalloc(op, p, out[:N ** 3], ok=(P.STOKES_E_ARG,))
            assert st == P.STOKES_E_ARG
