"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Operators are compared element by element on seeded inputs over a zoo of
masks and sizes that span several sweep tiles and ragged tails.  Solves are
compared on permeability (1e-6 relative, FP64), fields and outer iteration
counts.  At the benchmark size (128^3) the solution is checked through
properties that hold at any size, evaluated with the oracle's own operators.
"""

import sys

import numpy as np
import pytest

import oracle
from synth import grf, random_cell_field, random_face_field, slits, spheres
from synth.geometry import channel_widths

pytestmark = pytest.mark.gpu

K_TOL = 1e-6          # FP64 permeability parity
OP_TOL = 1e-13        # operator parity, relative to the largest output entry


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


ZOO_NAMES = ["allfluid_5", "random_2", "random_3", "random_5", "random_33_p85", "random_24_p40", "spheres_24",
             "spheres_70", "slits_33_x", "slits_40_z", "grf_64", "spheres_128"]
_ZOO = {}


def zoo(name):
    if name in _ZOO:
        return _ZOO[name]
    seed = ZOO_NAMES.index(name)
    rng = np.random.default_rng(seed)
    if name == "allfluid_5":
        m = np.ones((5, 5, 5), np.uint8)
    elif name.startswith("random_"):
        parts = name.split("_")
        N = int(parts[1])
        phi = float(parts[2][1:]) / 100 if len(parts) > 2 else 0.6
        m = (rng.random((N, N, N)) < phi).astype(np.uint8)
    elif name == "spheres_24":
        m = spheres(24, 4.0, 0.7, 0)
    elif name == "spheres_70":
        m = spheres(70, 3.0, 0.4, 1)
    elif name == "slits_33_x":
        m = slits(33, [3, 5], axis=0)
    elif name == "slits_40_z":
        m = slits(40, 4, axis=2)
    elif name == "grf_64":
        m = grf(64, 4.0, 0.3, 2)
    elif name == "spheres_128":
        m = spheres(128, 6.0, 0.5, 0)
    _ZOO[name] = m
    return m


@pytest.mark.parametrize("name", ZOO_NAMES)
@pytest.mark.parametrize("keep_all", [False, True])
def test_operator_parity(P, name, keep_all):
    m = zoo(name)
    N = m.shape[0]
    force = (0.0, 1.0, 0.0) if "slits_33_x" in name else (1.0, 0.0, 0.0)
    if "slits_40_z" in name:
        force = (1.0, 0.3, 0.0)
    say(f"[operator parity] {name} N={N} keep_all={keep_all}")
    o = oracle.Oracle(m, force, strip=not keep_all)
    s = P.Stokes(m, force, keep_all=keep_all)
    try:
        info = s.info()
        assert info["nfluid"] == o.nfluid and info["ncomp_kept"] == o.ncomp_kept
        u = random_face_field(N, 11)
        p = random_cell_field(N, 12)
        checks = [
            (P.STOKES_OP_A, oracle.OP_A, u),
            (P.STOKES_OP_B, oracle.OP_B, u),
            (P.STOKES_OP_BT, oracle.OP_BT, p),
            (P.STOKES_OP_SHAT, oracle.OP_SHAT, p),
            (P.STOKES_OP_DIAG_A, oracle.OP_DIAG_A, None),
            (P.STOKES_OP_DIAG_SHAT, oracle.OP_DIAG_SHAT, None),
            (P.STOKES_OP_PROJECT, oracle.OP_PROJECT, p),
        ]
        for gop, oop, x in checks:
            got = s.apply(gop, x)
            ref = o.apply(oop, x)
            scale = max(np.abs(ref).max(), 1e-300)
            err = np.abs(got - ref).max() / scale
            assert err <= OP_TOL, (name, gop, err)
            # entries that are not unknowns are exactly zero
            assert np.all(got[ref == 0] == 0) or oop == oracle.OP_PROJECT
    finally:
        s.close()


def test_operator_bitwise_repeatable(P):
    m = zoo("spheres_70")
    s = P.Stokes(m)
    try:
        u = random_face_field(70, 3)
        a = s.apply(P.STOKES_OP_A, u)
        b = s.apply(P.STOKES_OP_A, u)
        assert np.array_equal(a, b)
    finally:
        s.close()


def test_apply_device_matches_host(P):
    import torch
    m = zoo("spheres_24")
    N = 24
    s = P.Stokes(m)
    try:
        u = random_face_field(N, 5)
        host = s.apply(P.STOKES_OP_A, u)
        dev_in = torch.tensor(u.reshape(-1), dtype=torch.float64, device="cuda")
        dev_out = torch.empty_like(dev_in)
        s.apply_device(P.STOKES_OP_A, dev_in, dev_out)
        torch.cuda.synchronize()
        assert np.array_equal(dev_out.cpu().numpy().reshape(host.shape), host)
    finally:
        s.close()


# ---------------------------------------------------------------------------
# Solver parity
# ---------------------------------------------------------------------------
def compare_solve(P, m, force, pc, tol=1e-8, fields=True, iters_slack=1):
    o = oracle.Oracle(m, force)
    ref = o.solve(pc, tol=tol)
    with P.Stokes(m, force) as s:
        rep = s.solve(pc, tol=tol)
        p, u = s.fields()
        hist = s.history()
    assert rep["status"] == 0, rep
    say(f"    k gpu={rep['k_hat']:.14e} oracle={ref['k_hat']:.14e} outer {rep['outer_iters']}/{ref['outer_iters']} "
        f"inner A {rep['inner_A_iters']}/{ref['inner_A']} S {rep['inner_S_iters']}/{ref['inner_S']}")
    if ref["k_hat"] == 0.0:
        assert rep["k_hat"] == 0.0
    else:
        assert abs(rep["k_hat"] - ref["k_hat"]) <= K_TOL * abs(ref["k_hat"])
    assert abs(rep["outer_iters"] - ref["outer_iters"]) <= iters_slack
    if fields and ref["k_hat"] != 0.0:
        us = np.abs(ref["u"]).max()
        assert np.abs(u - ref["u"]).max() <= 1e-5 * us
        ps = max(np.abs(ref["p"]).max(), 1e-30)
        assert np.abs(p - ref["p"]).max() <= 1e-5 * ps + 1e-12
    # history: residuals decrease to the tolerance, k per iteration converges
    if rep["outer_iters"] > 0:
        assert hist.shape[0] == rep["outer_iters"]
        assert hist[-1, 0] < tol
        assert abs(hist[-1, 2] - rep["k_hat"]) <= 1e-12 * abs(rep["k_hat"])
    return rep, ref


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("pc", ["uzawa", "simple"])
def test_solve_spheres_24(P, seed, pc):
    """24^3 periodic box, overlapping spheres of radius 4 until porosity 0.7."""
    say(f"[solve] spheres 24^3 r=4 phi=0.7 seed={seed} {pc}")
    m = spheres(24, 4.0, 0.7, seed)
    pcid = P.STOKES_SIMPLE if pc == "simple" else P.STOKES_UZAWA
    compare_solve(P, m, (1.0, 0.0, 0.0), pcid)


@pytest.mark.parametrize("pc", ["uzawa", "simple"])
def test_solve_tight_spheres_ragged(P, pc):
    """Tight packing (high surface-to-volume) on a size that is not a multiple of the tile."""
    say(f"[solve] spheres 37^3 r=2 phi=0.3 {pc}")
    m = spheres(37, 2.0, 0.3, 4)
    pcid = P.STOKES_SIMPLE if pc == "simple" else P.STOKES_UZAWA
    compare_solve(P, m, (1.0, 0.0, 0.0), pcid)


def test_solve_grf_multicomponent_oblique(P):
    """Thresholded Gaussian field, oblique force, several conducting components."""
    say("[solve] grf 40^3 oblique force")
    m = grf(40, 3.0, 0.3, 5)
    force = (0.3, 0.0, 1.0)
    o = oracle.Oracle(m, force)
    say(f"    components kept {o.ncomp_kept} of {o.ncomp_all}")
    compare_solve(P, m, force, P.STOKES_SIMPLE)


def test_solve_slits_many_components(P):
    """Oblique force on a slit stack: one conducting component per channel,
    linear pressure per channel, closed-form flux."""
    say("[solve] slits 48^3 oblique, many components")
    N = 48
    m = slits(N, [3, 4, 6], axis=1)
    force = (1.0, 0.5, 0.0)
    rep, ref = compare_solve(P, m, force, P.STOKES_SIMPLE)
    ws = channel_widths(N, [3, 4, 6])
    kx = sum(w * (w * w + 2) / 12.0 for w in ws) / N
    assert rep["mean_u"][0] == pytest.approx(kx, rel=1e-9)
    assert abs(rep["mean_u"][1]) < 1e-10


@pytest.mark.parametrize("axis,fdir", [(1, 0), (0, 2), (2, 1)])
def test_slit_closed_form_gpu(P, axis, fdir):
    """Plane Poiseuille flux W (W^2 + 2)/12 per channel; g = 0 so no outer step."""
    say(f"[solve] slit closed form axis={axis} force={fdir}")
    N = 36
    m = slits(N, [4, 7], axis=axis)
    f = [0.0, 0.0, 0.0]
    f[fdir] = 1.0
    with P.Stokes(m, f) as s:
        rep = s.solve(P.STOKES_SIMPLE, 1e-8)
    ws = channel_widths(N, [4, 7])
    assert rep["outer_iters"] == 0 and rep["flags"] & 0x2
    assert rep["k_vox"] == pytest.approx(sum(w * (w * w + 2) / 12.0 for w in ws) / N, rel=1e-11)


@pytest.mark.parametrize("W", [4, 16, 32])
@pytest.mark.parametrize("precision", [0, 1])
def test_slit_stack_128_along_channels(P, W, precision):
    """128^3 slit stack, 2-voxel walls, force along the channels, multigrid on both
    inner solves: g = B A^-1 f is zero in exact arithmetic; the computed one sits at
    the inner solve's error, below the floor, so no outer step is taken and the
    flux is the plane Poiseuille closed form W (W^2 + 2)/12 per channel."""
    N = 128
    say(f"[slit stack 128] W={W} along the channels precision={precision}")
    m = slits(N, W, axis=1)
    ws = channel_widths(N, W)
    for pc in (P.STOKES_SIMPLE, P.STOKES_UZAWA):
        with P.Stokes(m, (1.0, 0.0, 0.0), precision=precision) as s:
            info = s.info()
            assert info["mg_levels_S"] >= 3 and info["mg_levels_A"] >= 3
            rep = s.solve(pc, 1e-8)
        say(f"    pc={pc} outer={rep['outer_iters']} r0={rep['r0_norm']:.3e} flags={rep['flags']} "
            f"k_vox={rep['k_vox']:.15e}")
        assert rep["status"] == 0
        assert rep["outer_iters"] == 0 and rep["flags"] & P.STOKES_FLAG_ZERO_RHS
        assert rep["k_vox"] == pytest.approx(sum(w * (w * w + 2) / 12.0 for w in ws) / N, rel=1e-9)
        assert abs(rep["mean_u"][1]) == 0.0 and abs(rep["mean_u"][2]) == 0.0


@pytest.mark.parametrize("W", [4, 16])
def test_slit_stack_128_oblique(P, W):
    """128^3 slit stack with the force (1, 0.5, 0): the exact solution has u_y = 0,
    a pressure rising by f_y per voxel across each channel, and the channel flux
    of the closed form; multigrid on both inner solves."""
    N = 128
    say(f"[slit stack 128] W={W} oblique force")
    m = slits(N, W, axis=1)
    ws = channel_widths(N, W)
    with P.Stokes(m, (1.0, 0.5, 0.0)) as s:
        rep = s.solve(P.STOKES_SIMPLE, 1e-8)
        p, u = s.fields()
    say(f"    outer={rep['outer_iters']} innerA={rep['inner_A_iters']} innerS={rep['inner_S_iters']} "
        f"mean_u={rep['mean_u']}")
    assert rep["status"] == 0 and rep["outer_iters"] > 0
    assert rep["mean_u"][0] == pytest.approx(sum(w * (w * w + 2) / 12.0 for w in ws) / N, rel=1e-8)
    # pressure steps of f_y across every active y-face (B^T p = f_y where u_y = 0)
    fl = m.astype(bool)
    act_y = fl & np.roll(fl, 1, axis=1)
    dp = (p - np.roll(p, 1, axis=1))[act_y]
    assert np.abs(dp - 0.5).max() < 1e-6
    assert np.abs(u[1]).max() < 1e-6 * np.abs(u[0]).max()


def test_no_flow_geometry(P):
    """Force normal to all walls: no conducting fluid, k = 0 exactly, no device solve."""
    m = slits(16, 4, axis=0)
    with P.Stokes(m, (1.0, 0.0, 0.0)) as s:
        rep = s.solve(P.STOKES_UZAWA, 1e-8)
        assert rep["k_hat"] == 0.0 and rep["flags"] & 0x1
        assert s.permeability() == 0.0


@pytest.mark.parametrize("N", [2, 3])
def test_tiny_boxes(P, N):
    rng = np.random.default_rng(N)
    m = (rng.random((N, N, N)) < 0.75).astype(np.uint8)
    m[0, 0, :] = 1
    for pc in (P.STOKES_UZAWA, P.STOKES_SIMPLE):
        compare_solve(P, m, (1.0, 0.0, 0.0), pc, tol=1e-10)


def test_state_and_argument_errors(P):
    from paper_2307_05266_amd.stokes import StokesError
    m = spheres(16, 2.0, 0.6, 0)
    with P.Stokes(m) as s:
        with pytest.raises(StokesError) as e:
            s.permeability()
        assert e.value.status == -5
        with pytest.raises(StokesError):
            s.solve(P.STOKES_SIMPLE, tol=-1.0)
        with pytest.raises(StokesError):
            s.set_option("no_such_option", 1.0)


def test_not_converged_is_reported(P):
    """A tiny outer cap: the solve returns the last iterate with NOT_CONVERGED."""
    m = spheres(24, 3.0, 0.5, 1)
    with P.Stokes(m) as s:
        s.set_option("max_outer", 2)
        rep = s.solve(P.STOKES_UZAWA, 1e-12)
        assert rep["status"] == 1 and rep["outer_iters"] == 2
        assert s.permeability() > 0.0


def test_solve_repeatable_bitwise(P):
    m = spheres(32, 3.0, 0.5, 7)
    with P.Stokes(m) as s:
        a = s.solve(P.STOKES_SIMPLE, 1e-8)
        pa, ua = s.fields()
        b = s.solve(P.STOKES_SIMPLE, 1e-8)
        pb, ub = s.fields()
    assert a["k_hat"] == b["k_hat"] and a["outer_iters"] == b["outer_iters"]
    assert np.array_equal(ua, ub) and np.array_equal(pa, pb)


def test_preconditioned_stop_norm(P):
    """Algorithm 1's own stopping test on ||z|| / ||z0||."""
    m = spheres(24, 3.0, 0.45, 2)
    o = oracle.Oracle(m)
    ref = o.solve(oracle.SIMPLE, tol=1e-6, stop_prec=True)
    with P.Stokes(m) as s:
        s.set_option("stop_prec", 1)
        rep = s.solve(P.STOKES_SIMPLE, 1e-6)
    assert abs(rep["outer_iters"] - ref["outer_iters"]) <= 1
    assert rep["rel_res_prec"] < 1e-6


def test_true_velocity_option(P):
    m = spheres(24, 3.0, 0.5, 3)
    o = oracle.Oracle(m)
    ref = o.solve(oracle.SIMPLE, tol=1e-8, true_u=True)
    with P.Stokes(m) as s:
        s.set_option("true_velocity", 1)
        rep = s.solve(P.STOKES_SIMPLE, 1e-8)
    assert rep["k_hat"] == pytest.approx(ref["k_hat_true"], rel=1e-6)
    assert rep["div_norm"] <= 1e-7 * ref["r0"]


# ---------------------------------------------------------------------------
# Benchmark size: 128^3 spheres r = 6, porosity 0.5 (launch configuration of the
# benchmark), checked through the discrete equations with the oracle's operators.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pc", ["simple", "uzawa"])
def test_full_size_solution_satisfies_equations(P, pc):
    say(f"[full size] spheres 128^3 r=6 phi=0.5 seed=0 {pc}")
    N = 128
    m = zoo("spheres_128")
    pcid = P.STOKES_SIMPLE if pc == "simple" else P.STOKES_UZAWA
    with P.Stokes(m) as s:
        rep = s.solve(pcid, 1e-8)
        p, u = s.fields()
    say(f"    k={rep['k_hat']:.12e} outer={rep['outer_iters']} innerA={rep['inner_A_iters']} "
        f"innerS={rep['inner_S_iters']} t={rep['seconds']:.2f}s cond={rep['cond_est']:.3g}")
    assert rep["status"] == 0
    o = oracle.Oracle(m)
    # momentum: A u + B^T p = f on active faces
    Au = o.apply(oracle.OP_A, u)
    BTp = o.apply(oracle.OP_BT, p)
    diagA = o.apply(oracle.OP_DIAG_A, None)
    f = np.zeros_like(diagA)
    f[0] = (diagA[0] > 0).astype(np.float64)          # unit force along x on active x-faces
    res = Au + BTp - f
    assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(f)
    # continuity: ||B u|| <= tol ||g||
    Bu = o.apply(oracle.OP_B, u)
    assert np.linalg.norm(Bu) <= 1.01e-8 * rep["r0_norm"]
    # energy identity f.u = u.A u and the flux average
    fu = u[0].sum()
    assert fu == pytest.approx(float(np.dot(u.ravel(), Au.ravel())), rel=1e-8)
    assert rep["k_vox"] == pytest.approx(fu / N ** 3, rel=1e-12)
    # pressure has zero mean on every kept component
    fl, comp = o.masks()
    for c in range(o.ncomp_kept):
        assert abs(p[comp == c].mean()) < 1e-10 * max(np.abs(p).max(), 1.0)


# 10: one coarse level, columns wider than the box; 36: the last column of
# 32-wide tiles runs past the box edge (wrapped lanes feed the periodic ring)
@pytest.mark.parametrize("N,seed", [(10, 1), (24, 3), (36, 2), (48, 5)])
def test_multigrid_and_jacobi_inner_solves_agree(P, N, seed):
    """The SIMPLE inner solve with the multigrid preconditioner (default) and with
    Jacobi reach the same outer trajectory: same outer count (+-1), same k."""
    m = spheres(N, 3.0 if N > 10 else 1.5, 0.45, seed)
    with P.Stokes(m) as s:
        s.set_option("mg", 0)
        s.set_option("mg_A", 0)
        a = s.solve(P.STOKES_SIMPLE, 1e-8)
        s.set_option("mg", 1)
        s.set_option("mg_A", 1)
        b = s.solve(P.STOKES_SIMPLE, 1e-8)
        info = s.info()
    say(f"    jacobi: outer={a['outer_iters']} innerA={a['inner_A_iters']} innerS={a['inner_S_iters']}  "
        f"mg: outer={b['outer_iters']} innerA={b['inner_A_iters']} innerS={b['inner_S_iters']}  "
        f"levels S={info['mg_levels_S']} A={info['mg_levels_A']}")
    assert abs(a["outer_iters"] - b["outer_iters"]) <= 1
    assert abs(a["k_hat"] - b["k_hat"]) <= 1e-7 * abs(a["k_hat"])
    # halving stops at an odd side; the coarsest level must fit one workgroup
    # (n^3 <= 2048 for the SIMPLE matrix, 3 n^3 <= 2048 for A's three planes)
    n = N
    while n % 2 == 0 and n // 2 >= 2 and n ** 3 > 512:
        n //= 2
    assert info["mg_levels_S"] == (0 if n == N or n ** 3 > 2048 else (N // n).bit_length() - 1)
    assert info["mg_levels_A"] == (0 if n == N or 3 * n ** 3 > 2048 else (N // n).bit_length() - 1)
    assert info["mg_levels_S"] > 0
    assert b["inner_S_iters"] < a["inner_S_iters"]
    if info["mg_levels_A"] > 0:
        assert b["inner_A_iters"] < a["inner_A_iters"]
    else:
        assert b["inner_A_iters"] == a["inner_A_iters"]


def test_kernel_timing_counts_every_kind(P):
    """Sampled HIP-event timing covers every kernel the inner solves launch:
    with multigrid the direction, stencil, fused update + restriction and
    level-0 smoothing kernels (the SIMPLE matrix's in their pipelined FP64 forms
    by default, the plain forms with mg_pipe=0); with Jacobi the direction,
    stencil and update kernels.  Bytes per launch follow the per-voxel byte
    model."""
    from paper_2307_05266_amd.stokes import KERNEL_NAMES
    N = 32
    per_voxel = [73, 49, 145, 32, 17, 56, 28, 52, 18, 26, 148, 58, 97, 33, 51, 19, 34]
    assert len(KERNEL_NAMES) == len(per_voxel)
    with P.Stokes(spheres(N, 3.0, 0.5, 1)) as s:
        for mg, pipe, launched in [(1, 1, {7, 10, 12, 14, 15, 16}), (1, 0, {7, 9, 10, 11, 12, 13}),
                                   (0, 1, {0, 1, 2, 3, 4, 5})]:
            s.set_option("mg", mg)
            s.set_option("mg_A", mg)
            s.set_option("mg_pipe", pipe)
            s.set_option("fuse_dir_A", 1)
            s.set_option("kernel_timing", 1)
            s.solve(P.STOKES_SIMPLE, 1e-8)
            for kind, name in enumerate(KERNEL_NAMES):
                ms, n, nbytes = s.kernel_timing(kind)
                say(f"    mg={mg} pipe={pipe} {name}: {n} launches {ms:.3f} ms")
                assert (n > 0 and ms > 0.0) == (kind in launched), name
                assert nbytes == per_voxel[kind] * N ** 3
                assert s.kernel_timing(kind)[1] == 0   # reset by the read
        with pytest.raises(P.StokesError):
            s.kernel_timing(len(KERNEL_NAMES))


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_matches_eager_launches(P, precision):
    """Inner iterations replayed from captured HIP graphs give bitwise the same
    solve as kernel-by-kernel launches, on every replay (three solves in a row,
    with eager work and host synchronisation between them), and with timed eager
    iterations mixed into the replays."""
    m = spheres(32, 3.0, 0.5, 11)
    with P.Stokes(m, precision=precision) as s:
        s.set_option("graphs", 0)
        ref = s.solve(P.STOKES_SIMPLE, 1e-8)
        p0, u0 = s.fields()
        s.set_option("graphs", 1)
        for rep in range(3):
            r = s.solve(P.STOKES_SIMPLE, 1e-8)
            p1, u1 = s.fields()
            assert r["outer_iters"] == ref["outer_iters"]
            assert r["inner_A_iters"] == ref["inner_A_iters"] and r["inner_S_iters"] == ref["inner_S_iters"]
            assert r["k_hat"] == ref["k_hat"]
            assert np.array_equal(p1, p0) and np.array_equal(u1, u0)
        s.set_option("kernel_timing", 3)
        r = s.solve(P.STOKES_SIMPLE, 1e-8)
        assert r["k_hat"] == ref["k_hat"]
        # the SIMPLE direction + stencil kernel was timed (pipelined form in FP64)
        assert s.kernel_timing(16 if precision == 0 else 13)[1] > 0


def test_fused_direction_matches_separate_kernels(P):
    """Forming the direction inside the stencil kernel (double-buffered
    direction) or in a separate pointwise kernel gives bitwise the same solve."""
    m = spheres(40, 3.0, 0.45, 12)
    out = {}
    with P.Stokes(m) as s:
        for fa, fs in [(1, 1), (0, 0), (1, 0), (0, 1)]:
            s.set_option("fuse_dir_A", fa)
            s.set_option("fuse_dir_S", fs)
            r = s.solve(P.STOKES_SIMPLE, 1e-8)
            p, u = s.fields()
            out[(fa, fs)] = (r["k_hat"], r["inner_A_iters"], r["inner_S_iters"], p, u)
    ref = out[(1, 1)]
    for key, val in out.items():
        assert val[:3] == ref[:3], key
        assert np.array_equal(val[3], ref[3]) and np.array_equal(val[4], ref[4]), key


@pytest.mark.parametrize("N", [40, 64, 112])
def test_pipelined_level0_sweeps_match_plain(P, N):
    """The FP64 SIMPLE solve's level-0 sweeps with their loads issued a plane
    ahead (option mg_pipe, default on) give bitwise the same solve as the plain
    forms: 32-wide columns with two-plane runs (N = 40), 64-wide columns (64)
    and 64-wide tiles running past the box edge (112)."""
    m = spheres(N, 4.0, 0.45, 30 + N)
    out = {}
    with P.Stokes(m) as s:
        for pipe in (1, 0):
            s.set_option("mg_pipe", pipe)
            r = s.solve(P.STOKES_SIMPLE, 1e-8)
            p, u = s.fields()
            out[pipe] = (r["k_hat"], r["outer_iters"], r["inner_A_iters"], r["inner_S_iters"], p, u)
    say(f"    N={N}: k={out[1][0]:.15e} outer={out[1][1]} inner S={out[1][3]}")
    assert out[1][:4] == out[0][:4]
    assert np.array_equal(out[1][4], out[0][4]) and np.array_equal(out[1][5], out[0][5])


@pytest.mark.parametrize("pc", ["simple", "uzawa"])
def test_partial_wide_tiles_112(P, pc):
    """N = 112: 64-wide columns whose second tile runs past the box edge (wrapped
    lanes, the row-pair sum of the restriction through LDS), multigrid on both
    inner solves.  Multigrid and Jacobi reach the same solution, and it satisfies
    the discrete equations built by the oracle."""
    N = 112
    m = spheres(N, 5.0, 0.5, 21)
    pcid = P.STOKES_SIMPLE if pc == "simple" else P.STOKES_UZAWA
    with P.Stokes(m) as s:
        info = s.info()
        assert info["mg_levels_S"] == 4 and info["mg_levels_A"] == 4
        r = s.solve(pcid, 1e-8)
        p, u = s.fields()
        s.set_option("mg", 0)
        s.set_option("mg_A", 0)
        rj = s.solve(pcid, 1e-8)
    say(f"    {pc}: mg k={r['k_hat']:.14e} outer={r['outer_iters']}  jacobi k={rj['k_hat']:.14e} outer={rj['outer_iters']}")
    assert r["status"] == 0 and rj["status"] == 0
    assert abs(r["k_hat"] - rj["k_hat"]) <= 1e-7 * abs(rj["k_hat"])
    assert abs(r["outer_iters"] - rj["outer_iters"]) <= 1
    o = oracle.Oracle(m)
    dA = o.apply(oracle.OP_DIAG_A, None)
    f = np.zeros_like(dA)
    f[0] = (dA[0] > 0).astype(np.float64)
    res = o.apply(oracle.OP_A, u) + o.apply(oracle.OP_BT, p) - f
    assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(f)
    assert np.linalg.norm(o.apply(oracle.OP_B, u)) <= 1.01e-8 * r["r0_norm"]
