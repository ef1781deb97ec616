"""CPU-side checks of the C ABI: the library loads, exports every declared
entry point, validates its arguments, and its host-only geometry step agrees
with the oracle.  No compute call reaches the GPU here."""

import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from synth import grf, slits, spheres

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("stokes.h", "stokes_server.h")]


@pytest.fixture(scope="module")
def P():
    import paper_2307_05266_amd as P
    P.load()
    return P


def declared_functions():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stokes_[a-z_]+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("stokes_setup", "stokes_solve", "stokes_permeability", "stokes_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(P):
    from paper_2307_05266_amd.stokes import LIB_PATH, EXPORTED
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["stokes.h", "stokes_server.h"]
    out = subprocess.run(["nm", "-D", "--defined-only", LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (stokes_[a-z_]+)\b", out))
    for name in declared_functions():
        assert name in exported, name
    from paper_2307_05266_amd.stokes import EXPORTED_SERVER
    assert set(EXPORTED) | set(EXPORTED_SERVER) == set(declared_functions())


def test_status_strings(P):
    from paper_2307_05266_amd.stokes import status_str
    assert status_str(0) == "ok"
    assert status_str(-1) == "invalid argument"
    assert status_str(-5) == "invalid state"


def test_argument_validation_without_device(P):
    from paper_2307_05266_amd.stokes import StokesError, stokes_preprocess, stokes_setup
    m = np.ones((4, 4, 4), np.uint8)
    with pytest.raises(StokesError) as e:
        stokes_preprocess(m, 4, (0.0, 0.0, 0.0))
    assert e.value.status == -1
    with pytest.raises(StokesError):
        stokes_preprocess(m, 4, (np.nan, 0.0, 0.0))
    bad = m.copy()
    bad[0, 0, 0] = 2
    with pytest.raises(StokesError):
        stokes_preprocess(bad, 4, (1.0, 0.0, 0.0))
    with pytest.raises(StokesError):
        stokes_preprocess(np.ones(1, np.uint8), 1, (1.0, 0.0, 0.0))
    # setup validates before touching the device
    with pytest.raises(StokesError) as e:
        stokes_setup(m, 4, (0.0, 0.0, 0.0))
    assert e.value.status == -1


@pytest.mark.parametrize("case", ["spheres", "slits_oblique", "grf", "random", "keep_all"])
def test_preprocess_matches_oracle(P, case):
    from paper_2307_05266_amd.stokes import STOKES_KEEP_ALL_COMPONENTS, stokes_preprocess
    force, flags, strip = (1.0, 0.0, 0.0), 0, True
    if case == "spheres":
        m = spheres(24, 3.0, 0.45, 3)
    elif case == "slits_oblique":
        m = slits(24, [3, 5], axis=1)
        force = (1.0, 0.5, 0.0)
    elif case == "grf":
        m = grf(32, 4.0, 0.2, 1)
        force = (0.0, 0.0, 1.0)
    elif case == "random":
        m = (np.random.default_rng(5).random((9, 9, 9)) < 0.4).astype(np.uint8)
        force = (0.0, 1.0, 0.0)
    else:
        m = spheres(16, 2.0, 0.35, 2)
        flags, strip = STOKES_KEEP_ALL_COMPONENTS, False
    N = m.shape[0]
    g = stokes_preprocess(m, N, force, flags)
    o = oracle.Oracle(m, force, strip=strip)
    fl, comp = o.masks()
    assert (g["nfluid_in"], g["nfluid"], g["nsurf"], g["ncomp_all"], g["ncomp_kept"]) == \
        (o.nfluid_in, o.nfluid, o.nsurf, o.ncomp_all, o.ncomp_kept)
    assert np.array_equal(g["fluid"], fl)
    assert np.array_equal(g["label"], comp)


def test_preprocess_slit_normal_force_removes_everything(P):
    from paper_2307_05266_amd.stokes import stokes_preprocess
    g = stokes_preprocess(slits(16, 4, axis=2), 16, (0.0, 0.0, 1.0))
    assert g["nfluid"] == 0 and g["ncomp_kept"] == 0 and g["ncomp_all"] > 0


def test_estimate_bytes_host_only(P):
    """The admission bound is host arithmetic: it grows with N, the mixed path's
    FP32 vectors add to it, and bad arguments are rejected."""
    from paper_2307_05266_amd.stokes import StokesError
    est = [P.stokes_estimate_bytes(N) for N in (8, 16, 32, 64, 128)]
    assert all(a < b for a, b in zip(est, est[1:]))
    for N in (16, 32, 128, 256):
        e64, e32 = P.stokes_estimate_bytes(N, 0), P.stokes_estimate_bytes(N, 1)
        assert e32 > e64
        # dominant terms: 5 face and 9 cell FP64 vectors, 4 face and 5 cell FP32 vectors
        n3 = N ** 3
        assert e64 >= (5 * 3 + 9) * 8 * n3
        assert e32 - e64 >= (4 * 3 + 5) * 4 * n3
    for bad in [(1, 0, 0), (801, 0, 0), (32, 2, 0), (32, 0, 2)]:
        with pytest.raises(StokesError):
            P.stokes_estimate_bytes(bad[0], precision=bad[2], flags=bad[1])


def test_binding_constants_match_the_header(P):
    """Every enumerator of include/stokes.h (status codes, preconditioners,
    operators) has the same value in the Python binding."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADERS[0]).read(), flags=re.S)
    found = {}
    for body in re.findall(r"typedef\s+enum\s*\{(.*?)\}", src, flags=re.S):
        for name, val in re.findall(r"\b(STOKES_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            found[name] = int(val)
    assert {"STOKES_OP_MG_SHAT", "STOKES_OP_MG_A", "STOKES_SIMPLE", "STOKES_E_LIMIT"} <= set(found)
    from paper_2307_05266_amd import stokes as B
    for name, val in found.items():
        assert getattr(B, name) == val, name
