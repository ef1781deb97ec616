"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a closed form of the discrete
problem, an invariant of the operators, a textbook special case, a library
routine on a special case, or brute force on tiny inputs.  Together they are
chosen so that a dropped term, a wrong sign, a wrong neighbour index or a
wrong wall rule in the oracle fails at least one of them.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle
from synth import slits, spheres
from synth.geometry import channel_widths

TIGHT = dict(tol=1e-11, eps_A=1e-13, eps_S=1e-13)


def slit_kvox(N, widths):
    """Plane Poiseuille flow between voxel walls with the mirrored-ghost wall rule:
    the discrete profile is u_j = (W^2 + 1)/8 - (j - (W+1)/2)^2 / 2, whose sum over
    a channel is W (W^2 + 2) / 12; the box mean is the sum over channels / N."""
    return sum(w * (w * w + 2) / 12.0 for w in widths) / N


# --------------------------------------------------------------------------
# P1: plane Poiseuille flow in slits, every wall orientation and tangential force
# --------------------------------------------------------------------------
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("widths", [[4], [3, 6, 5]])
def test_slit_closed_form(oracle_mod, axis, widths):
    N = 16
    m = slits(N, widths, axis=axis)
    ws = channel_widths(N, widths)
    for fdir in range(3):
        if fdir == axis:
            continue
        f = [0.0, 0.0, 0.0]
        f[fdir] = 1.0
        for pc in (oracle.UZAWA, oracle.SIMPLE):
            r = oracle.Oracle(m, f).solve(pc, **TIGHT)
            assert r["status"] == 0
            # g = B A^{-1} f vanishes exactly: no outer iteration is needed
            assert r["outer_iters"] == 0
            assert r["k_vox"] == pytest.approx(slit_kvox(N, ws), rel=1e-11)
            # the other velocity components stay zero
            for c in range(3):
                if c != fdir:
                    assert np.abs(r["u"][c]).max() == 0.0


def test_slit_wall_rule_is_not_drop_all(oracle_mod):
    """The alternative rule (dropping the wall neighbour, wall a full voxel away)
    would give W (W+1)(W+2)/12 per channel; make sure the two are told apart."""
    N, W = 12, 4
    r = oracle.Oracle(slits(N, W), (1, 0, 0)).solve(oracle.UZAWA, **TIGHT)
    ws = channel_widths(N, W)
    drop_all = sum(w * (w + 1) * (w + 2) / 12.0 for w in ws) / N
    assert abs(r["k_vox"] - drop_all) > 0.1 * drop_all


# --------------------------------------------------------------------------
# Rectangular duct: exact discrete solution by eigen-expansion of the 1D
# ghost-Dirichlet second difference (eigenpairs 4 sin^2(pi m / 2W),
# sin(pi m (j - 1/2) / W)); checks the corner faces with two wall neighbours.
# --------------------------------------------------------------------------
def duct_flux(Wy, Wz):
    def eig(W):
        j = np.arange(1, W + 1)
        m = np.arange(1, W + 1)
        phi = np.sin(np.pi * np.outer(m, j - 0.5) / W)          # (m, j)
        lam = 4 * np.sin(np.pi * m / (2 * W)) ** 2
        return lam, phi
    ly, py = eig(Wy)
    lz, pz = eig(Wz)
    sy = py.sum(1) ** 2 / (py ** 2).sum(1)
    sz = pz.sum(1) ** 2 / (pz ** 2).sum(1)
    return float((np.outer(sy, sz) / (ly[:, None] + lz[None, :])).sum())


@pytest.mark.parametrize("Wy,Wz,flow", [(5, 3, 0), (4, 6, 1), (3, 3, 2)])
def test_rectangular_duct_closed_form(oracle_mod, Wy, Wz, flow):
    N = 9
    m = np.zeros((N, N, N), dtype=np.uint8)
    # duct along `flow`; cross-section spans two other axes starting at index 2
    ax = [a for a in range(3) if a != flow]
    sl = [slice(None)] * 3
    sl[2 - ax[0]] = slice(2, 2 + Wy)
    sl[2 - ax[1]] = slice(2, 2 + Wz)
    m[tuple(sl)] = 1
    f = [0.0, 0.0, 0.0]
    f[flow] = 1.0
    r = oracle.Oracle(m, f).solve(oracle.SIMPLE, **TIGHT)
    assert r["outer_iters"] == 0
    assert r["k_vox"] == pytest.approx(duct_flux(Wy, Wz) / N ** 2, rel=1e-11)


# --------------------------------------------------------------------------
# P2 / P3: oblique and wall-normal forces on slits
# --------------------------------------------------------------------------
def test_oblique_force_slit(oracle_mod):
    N, W = 12, 4
    m = slits(N, W, axis=1)
    ws = channel_widths(N, W)
    f = (1.0, 0.5, 0.0)
    for pc in (oracle.UZAWA, oracle.SIMPLE):
        r = oracle.Oracle(m, f).solve(pc, **TIGHT)
        assert r["status"] == 0
        # u_y vanishes and u_x is the Poiseuille profile of the x-component of f
        assert np.abs(r["u"][1]).max() < 1e-9
        assert r["mean_u"][0] == pytest.approx(slit_kvox(N, ws), rel=1e-9)
        # the y-force is held by a linear pressure: p_X - p_{X-e_y} = 0.5 inside a channel
        p = r["p"]
        gy = p[:, 3:2 + W, :] - p[:, 2:1 + W, :]
        assert np.allclose(gy, 0.5, atol=1e-8)


def test_wall_normal_force_slit_no_flow(oracle_mod):
    """Force normal to the walls: no channel winds along it, all fluid is removed and
    the permeability is exactly zero."""
    m = slits(12, 4, axis=1)
    o = oracle.Oracle(m, (0, 1, 0))
    assert o.ncomp_kept == 0 and o.nfluid == 0
    r = o.solve(oracle.SIMPLE)
    assert r["k_hat"] == 0.0 and r["outer_iters"] == 0


# --------------------------------------------------------------------------
# Dense helpers (tiny grids): full KKT system from the oracle's matrices
# --------------------------------------------------------------------------
def dense_ops(o):
    A = o.csr("A").toarray()
    B = o.csr("B").toarray()
    BT = o.csr("BT").toarray()
    return A, B, BT


def random_mask(N, seed, phi=0.6):
    rng = np.random.default_rng(seed)
    return (rng.random((N, N, N)) < phi).astype(np.uint8)


# --------------------------------------------------------------------------
# P5: B^T (built from its own rule) is exactly the transpose of B
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,seed", [(2, 0), (3, 1), (5, 2), (6, 3)])
def test_adjointness(oracle_mod, N, seed):
    o = oracle.Oracle(random_mask(N, seed), (1, 0, 0), strip=False)
    B, BT = o.csr("B"), o.csr("BT")
    assert (B.T - BT).count_nonzero() == 0
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((3, N, N, N))
    p = rng.standard_normal((N, N, N))
    Bu = o.apply(oracle.OP_B, u)
    BTp = o.apply(oracle.OP_BT, p)
    assert np.dot(Bu.ravel(), p.ravel()) == pytest.approx(np.dot(u.ravel(), BTp.ravel()), rel=1e-12)


# --------------------------------------------------------------------------
# P6: A symmetric, SPD with walls; the wall-free box gives three copies of the
# periodic 7-point Laplacian with eigenvalues sum_d 4 sin^2(pi m_d / N)
# --------------------------------------------------------------------------
def test_A_all_fluid_is_periodic_laplacian(oracle_mod):
    N = 4
    o = oracle.Oracle(np.ones((N, N, N), np.uint8), (1, 0, 0))
    A = o.csr("A").toarray()
    assert o.nf == 3 * N ** 3
    m = np.arange(N)
    s = 4 * np.sin(np.pi * m / N) ** 2
    lap = (s[:, None, None] + s[None, :, None] + s[None, None, :]).ravel()
    expect = np.sort(np.concatenate([lap, lap, lap]))
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), expect, atol=1e-12)


@pytest.mark.parametrize("N,seed", [(4, 0), (5, 1), (6, 2)])
def test_A_symmetric_positive_definite(oracle_mod, N, seed):
    o = oracle.Oracle(random_mask(N, seed, 0.7), (1, 0, 0), strip=False)
    A = o.csr("A")
    assert abs(A - A.T).max() == 0
    assert np.linalg.eigvalsh(A.toarray()).min() > 1e-8
    # weak diagonal dominance: off-diagonal row sums never exceed the diagonal
    Ad = A.toarray()
    off = np.abs(Ad).sum(1) - np.abs(np.diag(Ad))
    assert np.all(off <= np.diag(Ad))


# --------------------------------------------------------------------------
# P7 / P8: spectrum of S in [0, 1]; the wall-free box has S = I - 11^T/N^3
# --------------------------------------------------------------------------
def test_S_wall_free_box(oracle_mod):
    N = 4
    o = oracle.Oracle(np.ones((N, N, N), np.uint8), (1, 0, 0))
    A, B, BT = dense_ops(o)
    S = B @ np.linalg.pinv(A) @ BT
    n = N ** 3
    assert np.allclose(S, np.eye(n) - np.ones((n, n)) / n, atol=1e-10)


@pytest.mark.parametrize("N,seed", [(5, 4), (6, 5)])
def test_S_spectrum_in_unit_interval(oracle_mod, N, seed):
    o = oracle.Oracle(random_mask(N, seed, 0.75), (1, 0, 0), strip=False)
    A, B, BT = dense_ops(o)
    S = B @ np.linalg.solve(A, BT)
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.min() > -1e-10 and ev.max() < 1 + 1e-10
    # nullity = number of fluid components (constants on each)
    assert int(np.sum(ev < 1e-9)) == o.ncomp_kept
    # the no-slip walls create eigenvalues below one, and some remain exactly one
    assert ev.max() == pytest.approx(1.0, abs=1e-9)


# --------------------------------------------------------------------------
# P9: SIMPLE bound, spec(Shat^+ S) on range(B) within [1/2, 1/lambda_min(D^-1 A)]
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,seed", [(5, 6), (6, 7)])
def test_simple_spectral_bound(oracle_mod, N, seed):
    o = oracle.Oracle(random_mask(N, seed, 0.75), (1, 0, 0), strip=False)
    A, B, BT = dense_ops(o)
    D = np.diag(A)
    S = B @ np.linalg.solve(A, BT)
    Sh = B @ (BT / D[:, None])
    w, V = np.linalg.eigh(Sh)
    keep = w > 1e-10
    Vr = V[:, keep] / np.sqrt(w[keep])
    ev = np.linalg.eigvalsh(Vr.T @ S @ Vr)
    lmin = np.linalg.eigvals(A / D[:, None]).real.min()
    assert ev.min() >= 0.5 - 1e-10
    assert ev.max() <= 1.0 / lmin + 1e-10
    # the oracle's SIMPLE operator and its diagonal match B diag(A)^-1 B^T
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((N, N, N))
    _, cp = o.unknowns()
    y = o.apply(oracle.OP_SHAT, x).ravel()[cp]
    assert np.allclose(y, Sh @ x.ravel()[cp], atol=1e-12)
    dS = o.apply(oracle.OP_DIAG_SHAT, None).ravel()[cp]
    assert np.allclose(dS, np.diag(Sh), atol=1e-14)


# --------------------------------------------------------------------------
# P10: the iterative solve agrees with a direct solve of the coupled system
# --------------------------------------------------------------------------
def kkt_direct(o):
    """Direct solve of [[A, B^T], [B, 0]] [u; p] = [f; 0] with one pressure per
    component fixed by an extra zero-mean row (least squares on the consistent
    system), returning dense u and component-centred dense p."""
    N = o.N
    A, B, BT = o.csr("A"), o.csr("B"), o.csr("BT")
    fp, cp = o.unknowns()
    f = np.array([o.force[pos // N ** 3] for pos in fp])
    _, comp = o.masks()
    K = o.ncomp_kept
    C = sp.csr_matrix((np.ones(o.nc), (comp.ravel()[cp], np.arange(o.nc))), shape=(K, o.nc))
    M = sp.bmat([[A, BT, None], [B, None, C.T], [None, C, None]], format="csc")
    rhs = np.concatenate([f, np.zeros(o.nc), np.zeros(K)])
    sol = sp.linalg.spsolve(M, rhs)
    u = np.zeros(3 * N ** 3)
    u[fp] = sol[:o.nf]
    p = np.zeros(N ** 3)
    p[cp] = sol[o.nf:o.nf + o.nc]
    return u.reshape(3, N, N, N), p.reshape(N, N, N), sol[o.nf + o.nc:]


@pytest.mark.parametrize("N,seed,force", [(6, 0, (1, 0, 0)), (8, 1, (0, 0, 1)),
                                         (12, 2, (1, 0.5, 0.25))])
def test_iterative_matches_direct(oracle_mod, N, seed, force):
    m = spheres(N, 1.6, 0.55, seed)
    o = oracle.Oracle(m, force)
    if o.nfluid == 0:
        pytest.skip("no conducting fluid for this seed")
    u_ref, p_ref, lagr = kkt_direct(o)
    assert np.abs(lagr).max() < 1e-10       # the system is consistent
    for pc in (oracle.UZAWA, oracle.SIMPLE):
        r = o.solve(pc, **TIGHT)
        assert r["status"] == 0
        scale = np.abs(u_ref).max()
        assert np.abs(r["u"] - u_ref).max() < 1e-8 * scale
        assert np.abs(r["p"] - p_ref).max() < 1e-8 * max(np.abs(p_ref).max(), 1.0)
        k_ref = float(np.dot(np.asarray(force), u_ref.reshape(3, -1).mean(1))) \
            / float(np.dot(force, force)) / N ** 2
        assert r["k_hat"] == pytest.approx(k_ref, rel=1e-9)


# --------------------------------------------------------------------------
# P4: a component that does not wind along the force carries no flow, so
# removing it is exact (direct solve on the full, unstripped system)
# --------------------------------------------------------------------------
def test_closed_pocket_stripping_exact(oracle_mod):
    N = 8
    m = np.zeros((N, N, N), np.uint8)
    m[1:4, 1:4, :] = 1                  # a duct along x: winds in x
    m[5:7, 5:7, 2:6] = 1                # a closed pocket
    m[5:7, 1:3, :] = 1                  # a second duct along x
    m[1:3, 5:7, 3] = 1                  # a plate that winds in y only
    m[1:3, :, 5] = 1
    o_full = oracle.Oracle(m, (1, 0, 0), strip=False)
    o_cut = oracle.Oracle(m, (1, 0, 0), strip=True)
    assert o_full.ncomp_kept == 4 and o_cut.ncomp_kept == 2
    u_full, _, lagr = kkt_direct(o_full)
    assert np.abs(lagr).max() < 1e-10
    r = o_cut.solve(oracle.SIMPLE, **TIGHT)
    assert np.abs(r["u"] - u_full).max() < 1e-9 * np.abs(u_full).max()
    # velocity in the non-conducting parts is zero in the full solve
    fl_cut, _ = o_cut.masks()
    removed = (m == 1) & (fl_cut == 0)
    for c in range(3):
        assert np.abs(u_full[c][removed]).max() < 1e-10


# --------------------------------------------------------------------------
# P11 / P12: energy identity and divergence along the iteration
# --------------------------------------------------------------------------
def test_energy_identity_and_divergence(oracle_mod):
    N = 12
    m = spheres(N, 2.0, 0.5, 3)
    o = oracle.Oracle(m, (1, 0, 0))
    r = o.solve(oracle.SIMPLE, **TIGHT)
    u = r["u"]
    Au = o.apply(oracle.OP_A, u)
    fu = u[0].sum()                      # f = e_x on every active face
    assert fu == pytest.approx(float(np.dot(u.ravel(), Au.ravel())), rel=1e-9)
    assert r["k_vox"] == pytest.approx(fu / N ** 3, rel=1e-12)
    # B u_k = r_k: the recursive velocity ends divergence-free to the tolerance
    assert r["div_norm"] < 1e-9 * r["r0"]


# --------------------------------------------------------------------------
# Zero right-hand side: ||g||^2 <= f . A^{-1} f (dense algebra), and the floor
# zero_rhs_factor * eps_A * sqrt(f . u0) separates channels along the force
# (exact g = 0) from geometries with a real pressure, however small
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,seed,phi", [(5, 1, 0.7), (6, 2, 0.8), (7, 3, 0.6)])
def test_rhs_energy_bound(oracle_mod, N, seed, phi):
    """S = B A^-1 B^T has no eigenvalue above 1, so ||g||^2 <= g^T S^+ g <= f^T A^-1 f;
    checked with dense matrices and a dense solve, independently of the oracle's CG."""
    o = oracle.Oracle(random_mask(N, seed, phi), (1, 0.3, 0))
    A, B, BT = dense_ops(o)
    fp, _ = o.unknowns()
    f = np.array([o.force[pos // N ** 3] for pos in fp])
    u0 = np.linalg.solve(A, f)
    g = B @ u0
    _, comp = o.masks()
    _, cp = o.unknowns()
    lab = comp.ravel()[cp]
    for q in range(o.ncomp_kept):           # the projected g (zero mean per component)
        g[lab == q] -= g[lab == q].mean()
    S = B @ np.linalg.solve(A, BT)
    gSg = g @ np.linalg.lstsq(S, g, rcond=1e-12)[0]
    assert g @ g <= gSg * (1 + 1e-10) + 1e-14
    assert gSg <= (f @ u0) * (1 + 1e-10)
    r = o.solve(oracle.SIMPLE, **TIGHT)
    assert r["r0"] == pytest.approx(np.linalg.norm(g), rel=1e-9)
    assert r["f_dot_u0"] == pytest.approx(f @ u0, rel=1e-10)
    assert not r["zero_rhs"] and r["r0"] > 1e-4 * np.sqrt(r["f_dot_u0"])


def test_zero_rhs_floor_separates_channels_from_bumps(oracle_mod):
    """Slits with the force along the channels have g = 0 exactly; one solid voxel
    in a channel gives a small real g that stays far above the floor."""
    N = 16
    m = slits(N, [6, 4], axis=1)
    r = oracle.Oracle(m, (1, 0, 0)).solve(oracle.SIMPLE, **TIGHT)
    assert r["zero_rhs"] and r["outer_iters"] == 0 and r["r0"] == 0.0
    ws = channel_widths(N, [6, 4])
    assert r["k_vox"] == pytest.approx(slit_kvox(N, ws), rel=1e-11)
    mb = m.copy()
    fl = np.argwhere(mb == 1)
    k, j, i = fl[len(fl) // 2]
    mb[k, j, i] = 0
    rb = oracle.Oracle(mb, (1, 0, 0)).solve(oracle.SIMPLE, **TIGHT)
    assert not rb["zero_rhs"] and rb["outer_iters"] > 0
    ratio = rb["r0"] / np.sqrt(rb["f_dot_u0"])
    assert 1e3 * 1e-13 * 1e4 < ratio < 1.0
    assert rb["k_vox"] < r["k_vox"]


# --------------------------------------------------------------------------
# P13: Lanczos Ritz values from the CG coefficients bracket the spectrum
# --------------------------------------------------------------------------
def test_lanczos_extreme_eigenvalues(oracle_mod):
    """Ritz values of the CG tridiagonal lie in the spectrum's hull, and the extreme
    ones approach the extreme eigenvalues that the right-hand side g excites (CG
    only sees the eigen-components present in its starting residual)."""
    N = 6
    m = random_mask(N, 11, 0.8)
    o = oracle.Oracle(m, (1, 0, 0))
    A, B, BT = dense_ops(o)
    S = B @ np.linalg.solve(A, BT)
    w, V = np.linalg.eigh(0.5 * (S + S.T))
    fp, _ = o.unknowns()
    f = np.array([o.force[pos // N ** 3] for pos in fp])
    coef = V.T @ (B @ np.linalg.solve(A, f))
    present = w[np.abs(coef) > 1e-10 * np.abs(coef).max()]
    r = o.solve(oracle.UZAWA, tol=1e-13, eps_A=1e-14)
    ritz = r["ritz"]
    assert ritz.min() == pytest.approx(present.min(), rel=1e-8)
    assert present.max() * (1 - 1e-2) <= ritz.max() <= present.max() * (1 + 1e-10)
    assert ritz.max() <= w.max() * (1 + 1e-10) and w.max() == pytest.approx(1.0, abs=1e-9)
    assert r["cond_est"] == pytest.approx(ritz.max() / ritz.min())


# --------------------------------------------------------------------------
# Invariances: translation, mirror with reversed force, axis permutation
# --------------------------------------------------------------------------
def test_symmetry_invariances(oracle_mod):
    N = 10
    m = spheres(N, 1.8, 0.55, 7)
    k0 = oracle.Oracle(m, (1, 0, 0)).solve(oracle.SIMPLE, **TIGHT)["k_hat"]
    # translation
    mt = np.roll(m, (3, -2, 5), axis=(0, 1, 2))
    assert oracle.Oracle(mt, (1, 0, 0)).solve(oracle.SIMPLE, **TIGHT)["k_hat"] == pytest.approx(k0, rel=1e-9)
    # mirror in x (array axis 2) with the force reversed
    mm = m[:, :, ::-1]
    assert oracle.Oracle(mm, (-1, 0, 0)).solve(oracle.SIMPLE, **TIGHT)["k_hat"] == pytest.approx(k0, rel=1e-9)
    # mirror in y with the force unchanged
    my = m[:, ::-1, :]
    assert oracle.Oracle(my, (1, 0, 0)).solve(oracle.UZAWA, **TIGHT)["k_hat"] == pytest.approx(k0, rel=1e-9)
    # x <-> y swap (array axes 2 <-> 1) with the force moved to y
    ms = np.ascontiguousarray(np.swapaxes(m, 1, 2))
    assert oracle.Oracle(ms, (0, 1, 0)).solve(oracle.SIMPLE, **TIGHT)["k_hat"] == pytest.approx(k0, rel=1e-9)
    # x <-> z swap with the force moved to z
    mz = np.ascontiguousarray(np.swapaxes(m, 0, 2))
    assert oracle.Oracle(mz, (0, 0, 1)).solve(oracle.UZAWA, **TIGHT)["k_hat"] == pytest.approx(k0, rel=1e-9)
    # linearity in the force magnitude
    k2 = oracle.Oracle(m, (2.5, 0, 0)).solve(oracle.SIMPLE, **TIGHT)["k_hat"]
    assert k2 == pytest.approx(k0, rel=1e-9)


# --------------------------------------------------------------------------
# P15: geometry descriptors and component labels by brute force
# --------------------------------------------------------------------------
def periodic_components(m):
    N = m.shape[0]
    idx = np.arange(N ** 3).reshape(N, N, N)
    rows, cols = [], []
    for ax in range(3):
        nb = np.roll(idx, -1, axis=ax)
        both = (m == 1) & (np.roll(m, -1, axis=ax) == 1)
        rows.append(idx[both])
        cols.append(nb[both])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    G = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(N ** 3, N ** 3))
    n, lab = csg.connected_components(G, directed=False)
    fluid_labels = np.unique(lab[m.ravel() == 1])
    return len(fluid_labels)


@pytest.mark.parametrize("N,seed,phi", [(4, 0, 0.5), (6, 1, 0.35), (7, 2, 0.3), (8, 3, 0.6)])
def test_geometry_descriptors_brute_force(oracle_mod, N, seed, phi):
    m = random_mask(N, seed, phi)
    o = oracle.Oracle(m, (1, 0, 0))
    assert o.nfluid_in == int(m.sum())
    # surface voxels: solid with a fluid face neighbour (periodic)
    nb = np.zeros_like(m, dtype=bool)
    for ax in range(3):
        for s in (-1, 1):
            nb |= np.roll(m, s, axis=ax) == 1
    assert o.nsurf == int(((m == 0) & nb).sum())
    assert o.ncomp_all == periodic_components(m)


def test_slit_stv_ratio(oracle_mod):
    for W in (4, 6, 8):
        N = W + 2
        o = oracle.Oracle(slits(4 * N, W), (1, 0, 0))
        assert o.stv_ratio == pytest.approx(2.0 / W, rel=1e-14)


def test_winding_detection_tiled_box(oracle_mod):
    """A component conducts along x exactly when, in the box doubled along x, it
    does not split into two copies (brute force with a library labeller).  This
    holds for windings of odd x-multiplicity, which random masks realise."""
    for seed in range(6):
        N = 5
        m = random_mask(N, 100 + seed, 0.45)
        o = oracle.Oracle(m, (1, 0, 0))
        n_single = periodic_components(m)
        m2 = np.concatenate([m, m], axis=2)            # doubled along x (array axis 2)
        # periodic labeller on a non-cubic box
        idx = np.arange(m2.size).reshape(m2.shape)
        rows, cols = [], []
        for ax in range(3):
            both = (m2 == 1) & (np.roll(m2, -1, axis=ax) == 1)
            rows.append(idx[both])
            cols.append(np.roll(idx, -1, axis=ax)[both])
        G = sp.csr_matrix((np.ones(sum(len(r) for r in rows)),
                           (np.concatenate(rows), np.concatenate(cols))), shape=(m2.size, m2.size))
        _, lab = csg.connected_components(G, directed=False)
        n_double = len(np.unique(lab[m2.ravel() == 1]))
        # each wrapping component stays one piece, each other component doubles
        assert n_double - n_single == n_single - o.ncomp_kept


# --------------------------------------------------------------------------
# The paper's qualitative claim (Sec. 4.1.2, 4.2.2): SIMPLE needs far fewer outer
# iterations than Uzawa when the surface-to-volume ratio is high, and Uzawa
# catches up when it is low.
# --------------------------------------------------------------------------
def test_simple_beats_uzawa_when_tight(oracle_mod):
    m = spheres(16, 1.5, 0.3, 5)
    o = oracle.Oracle(m, (1, 0, 0))
    assert o.stv_ratio > 0.6
    ru = o.solve(oracle.UZAWA, tol=1e-8)
    rs = o.solve(oracle.SIMPLE, tol=1e-8)
    assert rs["outer_iters"] * 2 < ru["outer_iters"]
    assert rs["k_hat"] == pytest.approx(ru["k_hat"], rel=1e-6)
    # open geometry: Uzawa is not worse than SIMPLE
    m2 = spheres(16, 3.0, 0.8, 5)
    o2 = oracle.Oracle(m2, (1, 0, 0))
    assert o2.stv_ratio < 0.2
    ru2 = o2.solve(oracle.UZAWA, tol=1e-8)
    rs2 = o2.solve(oracle.SIMPLE, tol=1e-8)
    assert ru2["outer_iters"] <= rs2["outer_iters"]


# --------------------------------------------------------------------------
# Sampled residual rows (used at sizes too large to assemble): the row-by-row
# evaluation must equal the assembled operators at every unknown, vanish on
# the exact discrete solution, and mark non-unknowns.
# --------------------------------------------------------------------------
def test_sampled_residuals_match_assembled_operators(oracle_mod):
    from synth import grf
    rng = np.random.default_rng(3)
    for m, force in [(spheres(12, 2.0, 0.5, 1), (1.0, 0.0, 0.0)), (grf(10, 2.0, 0.45, 2), (0.3, -1.0, 0.5))]:
        N = m.shape[0]
        o = oracle.Oracle(m, force)
        light = oracle.Oracle(m, force, assemble=False)
        u = rng.standard_normal(3 * N ** 3)
        p = rng.standard_normal(N ** 3)
        # dense reference from the assembled operators; inactive u entries are ignored by both
        dA = o.apply(oracle.OP_DIAG_A, None).reshape(-1)
        f = np.concatenate([np.full(N ** 3, force[c]) for c in range(3)]) * (dA > 0)
        mom = o.apply(oracle.OP_A, u.reshape(3, N, N, N)).reshape(-1) + \
            o.apply(oracle.OP_BT, p.reshape(N, N, N)).reshape(-1) - f
        cont = o.apply(oracle.OP_B, u.reshape(3, N, N, N)).reshape(-1)
        fpos = np.arange(3 * N ** 3)
        cpos = np.arange(N ** 3)
        for orc in (o, light):
            rf, rc = oracle.sample_residuals(orc, u, p, fpos, cpos)
            act = dA > 0
            fl = o.masks()[0].reshape(-1) == 1
            assert np.all(np.isnan(rf[~act])) and np.all(np.isnan(rc[~fl]))
            assert np.allclose(rf[act], mom[act], rtol=0, atol=1e-12)
            assert np.allclose(rc[fl], cont[fl], rtol=0, atol=1e-12)
        # on the (tightly) solved system both residuals vanish
        r = o.solve(oracle.SIMPLE, tol=1e-12)
        rf, rc = oracle.sample_residuals(light, r["u"], r["p"], fpos, cpos)
        assert np.nanmax(np.abs(rf)) < 1e-8 and np.nanmax(np.abs(rc)) < 1e-8


# --------------------------------------------------------------------------
# Given right-hand sides g = B xi (consistent: in the range of B), the outer
# loop started from p = 0, u = 0: the random-consistent-RHS runs of the slit
# stacks (outer counts against the surface-to-volume ratio)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,seed,phi", [(6, 1, 0.7), (7, 2, 0.6), (8, 3, 0.65)])
def test_given_rhs_solves_schur_system(oracle_mod, N, seed, phi):
    """p from the outer PCG with g = B xi equals a dense least-squares solve of
    S p = g with S = B A^-1 B^T formed from the assembled matrices, per-component
    means removed; the residual B A^-1 B^T p - g vanishes."""
    rng = np.random.default_rng(seed)
    m = (rng.random((N, N, N)) < phi).astype(np.uint8)
    o = oracle.Oracle(m, (1.0, 0.0, 0.0), strip=False)
    xi = rng.standard_normal((3, N, N, N))
    g = o.apply(oracle.OP_B, xi)
    A = o.csr("A").toarray()
    B = o.csr("B").toarray()
    _, cpos = o.unknowns()
    S = B @ np.linalg.solve(A, B.T)
    gv = g.reshape(-1)[cpos]
    pv, *_ = np.linalg.lstsq(S, gv, rcond=None)
    comp = o.masks()[1].reshape(-1)[cpos]
    for c in np.unique(comp):
        pv[comp == c] -= pv[comp == c].mean()
    for pc in (oracle.UZAWA, oracle.SIMPLE):
        r = o.solve(pc, tol=1e-12, eps_A=1e-14, eps_S=1e-14, g=g)
        assert r["status"] == 0 and r["outer_iters"] > 0
        p = r["p"].reshape(-1)[cpos]
        assert np.abs(p - pv).max() <= 1e-8 * np.abs(pv).max()
        assert np.abs(S @ p - gv).max() <= 1e-9 * np.abs(gv).max()


def test_given_rhs_equal_to_force_rhs(oracle_mod):
    """With g = B A^-1 f the given-RHS loop reaches the pressure of the ordinary solve."""
    m = spheres(12, 2.0, 0.6, 4)
    o = oracle.Oracle(m, (1.0, 0.0, 0.0))
    a = o.solve(oracle.SIMPLE, **TIGHT)
    f = np.zeros((3, 12, 12, 12))
    f[0] = o.apply(oracle.OP_DIAG_A, None)[0] > 0
    u0, _ = o.inner_solve(0, f, eps=1e-14)
    g = o.apply(oracle.OP_B, u0)
    b = o.solve(oracle.SIMPLE, g=g, **TIGHT)
    assert np.abs(a["p"] - b["p"]).max() <= 1e-8 * np.abs(a["p"]).max()
    assert abs(a["outer_iters"] - b["outer_iters"]) <= 1
