"""CPU FP64 oracle for the Stokes pressure Schur-complement solve.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the product package never imports it and shares no
code with it.  The arithmetic lives in stokes_oracle.c (plain C, explicit
sparse matrices over the active unknowns); this module loads it with ctypes
and adds the Lanczos condition estimate of Sec. 4.1.2 (Ritz values of the CG
tridiagonal, computed with numpy).

Parity pins: see tests/test_oracle_pins.py.  The paper's own permeabilities,
iteration counts and condition numbers are "parity unpinned": their inputs
(CT images, the seeds of the 2D packings) are not available.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stokes_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

UZAWA, SIMPLE = 0, 1
OP_A, OP_B, OP_BT, OP_SHAT, OP_DIAG_A, OP_DIAG_SHAT, OP_PROJECT = range(7)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-D_POSIX_C_SOURCE=199309L", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, dp, lp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), \
        ctypes.POINTER(ctypes.c_long), ctypes.c_int
    lib.oracle_create.restype = vp
    lib.oracle_create.argtypes = [ip, ctypes.c_void_p, dp, ip]
    lib.oracle_create_ex.restype = vp
    lib.oracle_create_ex.argtypes = [ip, ctypes.c_void_p, dp, ip, ip]
    lib.oracle_sample_residuals.argtypes = [vp, dp, dp, ctypes.c_long, ctypes.c_void_p, dp, ctypes.c_long,
                                            ctypes.c_void_p, dp]
    lib.oracle_destroy.argtypes = [vp]
    lib.oracle_info.argtypes = [vp, lp]
    lib.oracle_masks.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_csr.argtypes = [vp, ip, lp, lp, dp]
    lib.oracle_unknowns.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_apply.argtypes = [vp, ip, dp, dp]
    lib.oracle_apply.restype = ip
    lib.oracle_solve.argtypes = [vp, ip, dp, ctypes.c_void_p, ctypes.c_void_p, dp,
                                 ctypes.c_void_p, ip]
    lib.oracle_solve.restype = ip
    lib.oracle_solve_g.argtypes = [vp, ip, dp, dp, ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_void_p, ip]
    lib.oracle_solve_g.restype = ip
    lib.oracle_inner_solve.argtypes = [vp, ip, dp, dp, ctypes.c_double, ip]
    lib.oracle_inner_solve.restype = ip
    lib.oracle_threads.restype = ip
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def threads() -> int:
    return int(_load().oracle_threads())


def lanczos_ritz(alphas, betas):
    """Ritz values of the CG tridiagonal T_k built from the CG coefficients
    (Saad, Sec. 6.7.3): diag_0 = 1/alpha_0, diag_j = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    offdiag_j = sqrt(beta_{j-1})/alpha_{j-1}."""
    a = np.asarray(alphas, dtype=np.float64)
    b = np.asarray(betas, dtype=np.float64)
    k = len(a)
    if k == 0:
        return np.zeros(0)
    diag = 1.0 / a
    diag[1:] += b[:k - 1] / a[:k - 1]
    off = np.sqrt(b[:k - 1]) / a[:k - 1]
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    return np.linalg.eigvalsh(T)


class Oracle:
    """One geometry, assembled.  mask: uint8 (N, N, N) [k][j][i], 1 = fluid."""

    def __init__(self, mask, force=(1.0, 0.0, 0.0), strip=True, assemble=True):
        lib = _load()
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert mask.ndim == 3 and mask.shape[0] == mask.shape[1] == mask.shape[2]
        self.N = mask.shape[0]
        self.force = np.array(force, dtype=np.float64)
        self.assembled = bool(assemble)
        self._h = lib.oracle_create_ex(self.N, mask.ctypes.data, _dptr(self.force), int(bool(strip)),
                                       int(self.assembled))
        if not self._h:
            raise ValueError("oracle_create rejected the input")
        info = np.zeros(10, dtype=np.int64)
        lib.oracle_info(self._h, info.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
        (_, self.nfluid_in, self.nfluid, self.nsurf, self.ncomp_all, self.ncomp_kept,
         self.nf, self.nc, self.nnzA, self.nnzB) = (int(v) for v in info)

    def close(self):
        if self._h:
            _load().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- geometry -----------------------------------------------------------
    @property
    def porosity(self):
        return self.nfluid_in / self.N ** 3

    @property
    def stv_ratio(self):
        """Surface-to-volume ratio (eq. s-t-v-ration), as a fraction."""
        return self.nsurf / self.nfluid_in if self.nfluid_in else 0.0

    def masks(self):
        N = self.N
        fl = np.zeros(N ** 3, dtype=np.uint8)
        comp = np.zeros(N ** 3, dtype=np.int32)
        _load().oracle_masks(self._h, fl.ctypes.data, comp.ctypes.data)
        return fl.reshape(N, N, N), comp.reshape(N, N, N)

    # ---- matrices -----------------------------------------------------------
    def csr(self, which):
        """which: 'A', 'B' or 'BT'.  Returns scipy.sparse.csr_matrix over the
        active unknowns (faces for A and B^T rows, fluid cells for B rows)."""
        import scipy.sparse as sp
        w = {"A": 0, "B": 1, "BT": 2}[which]
        nrow = {"A": self.nf, "B": self.nc, "BT": self.nf}[which]
        ncol = {"A": self.nf, "B": self.nf, "BT": self.nc}[which]
        nnz = {"A": self.nnzA, "B": self.nnzB, "BT": 2 * self.nf}[which]
        ptr = np.zeros(nrow + 1, dtype=np.int64)
        col = np.zeros(max(nnz, 1), dtype=np.int64)
        val = np.zeros(max(nnz, 1), dtype=np.float64)
        lp = ctypes.POINTER(ctypes.c_long)
        _load().oracle_csr(self._h, w, ptr.ctypes.data_as(lp), col.ctypes.data_as(lp), _dptr(val))
        return sp.csr_matrix((val[:nnz], col[:nnz], ptr), shape=(nrow, ncol))

    def unknowns(self):
        """Dense positions of the unknowns: face_pos (c*N^3 + X), cell_pos (X)."""
        fp = np.zeros(max(self.nf, 1), dtype=np.int64)
        cp = np.zeros(max(self.nc, 1), dtype=np.int64)
        _load().oracle_unknowns(self._h, fp.ctypes.data, cp.ctypes.data)
        return fp[:self.nf], cp[:self.nc]

    # ---- operators on dense fields -----------------------------------------
    def apply(self, op, x):
        N = self.N
        face_in = op in (OP_A, OP_B)
        face_out = op in (OP_A, OP_BT, OP_DIAG_A)
        xin = np.ascontiguousarray(x, dtype=np.float64).ravel()
        if op not in (OP_DIAG_A, OP_DIAG_SHAT):
            assert xin.size == (3 if face_in else 1) * N ** 3
        else:
            xin = np.zeros(3 * N ** 3)
        out = np.zeros((3 if face_out else 1) * N ** 3)
        rc = _load().oracle_apply(self._h, op, _dptr(xin), _dptr(out))
        if rc != 0:
            raise ValueError("bad op")
        return out.reshape((3, N, N, N) if face_out else (N, N, N))

    def inner_solve(self, which, b, eps=1e-12, maxit=100000):
        N = self.N
        b = np.ascontiguousarray(b, dtype=np.float64).ravel()
        x = np.zeros_like(b)
        it = _load().oracle_inner_solve(self._h, which, _dptr(b), _dptr(x), eps, maxit)
        shape = (3, N, N, N) if which == 0 else (N, N, N)
        return x.reshape(shape), it

    # ---- the solve ------------------------------------------------------------
    def solve(self, precond=SIMPLE, tol=1e-8, eps_A=1e-12, eps_S=1e-12, max_outer=2000,
              max_inner=200000, stop_prec=False, true_u=False, hist_cap=4000, zero_rhs_factor=1000.0,
              g=None):
        """g: optional right-hand side of S p = g (N^3 cell field) in place of
        g = B A^-1 f; the loop then starts from u0 = 0."""
        N = self.N
        params = np.array([tol, eps_A, eps_S, max_outer, max_inner, int(stop_prec),
                           int(true_u), zero_rhs_factor], dtype=np.float64)
        p = np.zeros(N ** 3)
        u = np.zeros(3 * N ** 3)
        stats = np.zeros(24)
        hist = np.zeros((hist_cap, 8))
        if g is None:
            st = _load().oracle_solve(self._h, int(precond), _dptr(params), p.ctypes.data,
                                      u.ctypes.data, _dptr(stats), hist.ctypes.data, hist_cap)
        else:
            gd = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
            assert gd.size == N ** 3
            st = _load().oracle_solve_g(self._h, int(precond), _dptr(params), _dptr(gd), p.ctypes.data,
                                        u.ctypes.data, _dptr(stats), hist.ctypes.data, hist_cap)
        k = int(stats[2])
        h = hist[:min(k, hist_cap)]
        res = {
            "status": int(st),
            "k_hat": stats[0], "k_vox": stats[1], "outer_iters": k,
            "inner_A": int(stats[3]), "inner_S": int(stats[4]),
            "rel_res": stats[5], "rel_res_prec": stats[6], "div_norm": stats[7],
            "r0": stats[9], "z0": stats[10],
            "k_hat_true": stats[11], "div_true": stats[12],
            "mean_u": stats[13:16].copy(), "seconds": stats[16], "threads": int(stats[17]),
            "zero_rhs": bool(stats[18]), "f_dot_u0": stats[19],
            "hist": h.copy(),
            "p": p.reshape(N, N, N), "u": u.reshape(3, N, N, N),
        }
        # the loop's alpha/beta pairs; beta of the last step is absent when it stopped
        alphas = h[:, 5]
        betas = h[:, 6]
        if k > 0:
            res["ritz"] = lanczos_ritz(alphas, betas)
            res["cond_est"] = float(res["ritz"].max() / res["ritz"].min())
        else:
            res["ritz"] = np.zeros(0)
            res["cond_est"] = float("nan")
        return res


def sample_residuals(orc, u, p, face_pos, cell_pos):
    """Residual rows of the discrete Stokes system at sampled unknowns, evaluated
    one by one from the assembly rules (no matrix is formed):
    (A u + B^T p - f) at face positions c*N^3 + X, (B u) at cells X; NaN where
    the position is not an unknown.  `orc` may be created with assemble=False."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    p = np.ascontiguousarray(p, dtype=np.float64).reshape(-1)
    N = orc.N
    assert u.size == 3 * N ** 3 and p.size == N ** 3
    fpos = np.ascontiguousarray(face_pos, dtype=np.int64)
    cpos = np.ascontiguousarray(cell_pos, dtype=np.int64)
    rf = np.empty(fpos.size)
    rc = np.empty(cpos.size)
    _load().oracle_sample_residuals(orc._h, _dptr(u), _dptr(p), fpos.size, fpos.ctypes.data, _dptr(rf),
                                    cpos.size, cpos.ctypes.data, _dptr(rc))
    return rf, rc
