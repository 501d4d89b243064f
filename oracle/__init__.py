"""CPU oracle for the one-band Hubbard sector problem (two-spin basis).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the GPU library.  It shares no code
with the GPU path.  Parity status of each function (what pins it) is listed in
its docstring; the pins live in ``tests/test_oracle_*.py``.

Layers
------
* ``liboracle.so`` (``oracle.c``, plain C + OpenMP): Algorithm I enumeration
  (Appendix A), the sorted two-spin keys I = I_up + 2^M I_dn (Sec. II), the full
  sparse H built from Eq. (count1) with the esign rule of Sec. III A and binary
  search for the hopped key, SpMV, matrix-free row evaluation, and the parameter
  bilinear forms used for Hellmann-Feynman derivatives.
* Python (numpy / scipy): dense diagonalisation (LAPACK ``eigh``) and a Lanczos
  iteration (Sec. IV) whose tridiagonal eigenproblem is solved by LAPACK
  (``scipy.linalg.eigh_tridiagonal``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
        L.orc_enumerate.restype = i64
        L.orc_enumerate.argtypes = [ctypes.c_int, ctypes.c_int, P]
        L.orc_two_spin_keys.restype = ctypes.c_int
        L.orc_two_spin_keys.argtypes = [ctypes.c_int, P, i64, P, i64, P]
        L.orc_build_csr.restype = ctypes.c_int
        L.orc_build_csr.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, i64, P, i64, P, P, P]
        L.orc_spmv.restype = None
        L.orc_spmv.argtypes = [i64, P, P, P, P, P]
        L.orc_start_vector.restype = None
        L.orc_start_vector.argtypes = [u64, i64, i64, P]
        L.orc_apply_rows.restype = ctypes.c_int
        L.orc_apply_rows.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, i64, P, i64,
                                     P, u64, P, i64, P]
        L.orc_param_bilinear.restype = ctypes.c_int
        L.orc_param_bilinear.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, i64, P, i64, P, P, P, P, P]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
# Bases (Algorithm I) and two-spin keys (Sec. II)
# --------------------------------------------------------------------------

def enumerate_basis(M: int, N: int) -> np.ndarray:
    """Ascending one-spin basis by the Algorithm I scan (Appendix A).
    Pinned: Table I, binomial counts, itertools brute force, complement rule."""
    n = lib().orc_enumerate(M, N, None)
    if n < 0:
        raise ValueError("bad (M, N)")
    out = np.zeros(max(n, 1), dtype=np.uint64)
    lib().orc_enumerate(M, N, _p(out))
    return out[:n]


def two_spin_keys(M: int, up: np.ndarray, dn: np.ndarray) -> np.ndarray:
    """Sorted two-spin keys I = I_up + 2^M I_dn (Sec. II).  Pinned: Table I."""
    up = np.ascontiguousarray(up, dtype=np.uint64)
    dn = np.ascontiguousarray(dn, dtype=np.uint64)
    keys = np.zeros(len(up) * len(dn), dtype=np.uint64)
    if lib().orc_two_spin_keys(M, _p(up), len(up), _p(dn), len(dn), _p(keys)) != 0:
        raise ValueError("2M must be <= 64")
    return keys


@dataclass
class OracleModel:
    M: int
    bi: np.ndarray
    bj: np.ndarray
    t: np.ndarray
    U: np.ndarray
    eps: np.ndarray
    n_up: int
    n_dn: int

    @staticmethod
    def from_model(m) -> "OracleModel":
        bi = np.array([b[0] for b in m.bonds], dtype=np.int32)
        bj = np.array([b[1] for b in m.bonds], dtype=np.int32)
        return OracleModel(m.n_sites, bi, bj, np.array(m.t, dtype=np.float64),
                           np.array(m.U, dtype=np.float64), np.array(m.eps, dtype=np.float64),
                           m.n_up, m.n_dn)


class Sector:
    """Two-spin sector: one-spin lists by Algorithm I, sorted two-spin keys."""

    def __init__(self, model, explicit_keys: bool = True):
        self.m = model if isinstance(model, OracleModel) else OracleModel.from_model(model)
        M = self.m.M
        self.up = enumerate_basis(M, self.m.n_up)
        self.dn = enumerate_basis(M, self.m.n_dn)
        self.cu, self.cd = len(self.up), len(self.dn)
        self.dim = self.cu * self.cd
        self.keys = two_spin_keys(M, self.up, self.dn) if explicit_keys else None

    def _margs(self, with_values=True):
        m = self.m
        a = [m.M, len(m.bi), _p(m.bi), _p(m.bj)]
        if with_values:
            a += [_p(m.t), _p(m.U), _p(m.eps)]
        a += [_p(self.keys), _p(self.up), self.cu, _p(self.dn), self.cd]
        return a

    # ------------------------------------------------------------------
    def csr(self):
        """Full H (diagonal included) as CSR (row_ptr int64, col int32, val f64).
        Pinned: Jordan-Wigner construction, U=0 / t=0 closed forms, dimer,
        Hermiticity, nnz formula."""
        if self.dim >= 2 ** 31:
            raise ValueError("dim too large for int32 columns")
        rp = np.zeros(self.dim + 1, dtype=np.int64)
        rc = lib().orc_build_csr(*self._margs(), _p(rp), None, None)
        if rc != 0:
            raise RuntimeError(f"orc_build_csr count pass failed ({rc})")
        nnz = int(rp[-1])
        col = np.zeros(max(nnz, 1), dtype=np.int32)
        val = np.zeros(max(nnz, 1), dtype=np.float64)
        rc = lib().orc_build_csr(*self._margs(), _p(rp), _p(col), _p(val))
        if rc != 0:
            raise RuntimeError(f"orc_build_csr fill pass failed ({rc})")
        return rp, col[:nnz], val[:nnz]

    def dense(self) -> np.ndarray:
        rp, col, val = self.csr()
        H = np.zeros((self.dim, self.dim))
        rows = np.repeat(np.arange(self.dim), np.diff(rp))
        np.add.at(H, (rows, col), val)
        return H

    def apply_rows(self, rows: np.ndarray, x: Optional[np.ndarray] = None, seed: int = 0) -> np.ndarray:
        """y[rows] = (H x)[rows] without storing H; x=None means the unnormalised
        SplitMix64 start vector of `seed`."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        y = np.zeros(len(rows), dtype=np.float64)
        xx = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
        rc = lib().orc_apply_rows(*self._margs(), _p(xx), ctypes.c_uint64(seed), _p(rows), len(rows), _p(y))
        if rc != 0:
            raise RuntimeError(f"orc_apply_rows failed ({rc})")
        return y

    def param_bilinear(self, g: np.ndarray, x: np.ndarray):
        """(dbond, dU, deps): g^T (dH/dtheta) x for every bond t_b, site U_i and
        site energy eps_i.  Pinned: central finite differences of dense
        eigenvalues and the Euler identity E0 = sum theta dE0/dtheta."""
        m = self.m
        g = np.ascontiguousarray(g, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        db = np.zeros(len(m.bi))
        dU = np.zeros(m.M)
        de = np.zeros(m.M)
        rc = lib().orc_param_bilinear(*self._margs(with_values=False), _p(g), _p(x), _p(db), _p(dU), _p(de))
        if rc != 0:
            raise RuntimeError(f"orc_param_bilinear failed ({rc})")
        return db, dU, de


def start_vector(seed: int, n: int, k0: int = 0) -> np.ndarray:
    """Unnormalised start vector x_k = -1 + 2 u_k (SplitMix64 counter mode)."""
    out = np.zeros(n, dtype=np.float64)
    lib().orc_start_vector(ctypes.c_uint64(seed), k0, n, _p(out))
    return out


def spmv(csr, x: np.ndarray) -> np.ndarray:
    rp, col, val = csr
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    lib().orc_spmv(len(rp) - 1, _p(rp), _p(col), _p(val), _p(x), _p(y))
    return y


# --------------------------------------------------------------------------
# Eigensolvers (Sec. IV)
# --------------------------------------------------------------------------

def dense_ground_state(H: np.ndarray):
    """Lowest eigenpair by LAPACK (numpy.linalg.eigh)."""
    w, v = np.linalg.eigh(H)
    return float(w[0]), v[:, 0]


@dataclass
class LanczosResult:
    e0: float
    psi: Optional[np.ndarray]
    iters: int
    residual: float
    alphas: np.ndarray
    betas: np.ndarray


def _tri_lowest(alpha, beta):
    from scipy.linalg import eigh_tridiagonal
    w, v = eigh_tridiagonal(alpha, beta, select="i", select_range=(0, 0))
    return float(w[0]), v[:, 0]


def lanczos(matvec, n: int, v0: np.ndarray, *, max_iter: int = 400, tol: float = 1e-12,
            reorth: bool = False, want_vector: bool = True) -> LanczosResult:
    """Lanczos for the lowest eigenpair of a symmetric operator (Sec. IV).

    Recurrence: w = H v_k - beta_k v_{k-1}; alpha_k = <w, v_k>; w -= alpha_k v_k;
    (optionally full Gram-Schmidt against all previous v, done twice);
    beta_{k+1} = ||w||; v_{k+1} = w / beta_{k+1}.  Stops when the Ritz residual
    beta_{k+1} |y_k| <= tol |theta|, or on breakdown.  The eigenvector is formed
    from stored vectors (reorth=True) or by re-running the same recurrence."""
    v = v0 / np.linalg.norm(v0)
    alphas, betas = [], []
    Q = [v.copy()] if reorth else None
    v_prev = np.zeros(n)
    beta = 0.0
    theta, y = 0.0, np.ones(1)
    res = np.inf
    k = 0
    for k in range(1, max_iter + 1):
        w = matvec(v) - beta * v_prev
        a = float(np.dot(w, v))
        w -= a * v
        if reorth:
            for _ in range(2):
                for q in Q:
                    w -= np.dot(q, w) * q
        alphas.append(a)
        b = float(np.linalg.norm(w))
        theta, y = _tri_lowest(np.array(alphas), np.array(betas))
        res = b * abs(y[-1])
        if res <= tol * abs(theta) or b <= 1e-300 or k == n:
            break
        betas.append(b)
        v_prev, v = v, w / b
        beta = b
        if reorth:
            Q.append(v.copy())
    psi = None
    if want_vector:
        m = len(alphas)
        if reorth:
            psi = np.zeros(n)
            for j in range(m):
                psi += y[j] * Q[j]
        else:
            v = v0 / np.linalg.norm(v0)
            v_prev = np.zeros(n)
            psi = y[0] * v
            beta = 0.0
            for j in range(1, m):
                w = matvec(v) - beta * v_prev
                w -= alphas[j - 1] * v
                b = betas[j - 1]
                v_prev, v = v, w / b
                beta = b
                psi += y[j] * v
        psi /= np.linalg.norm(psi)
    return LanczosResult(theta, psi, k, res, np.array(alphas), np.array(betas))


def canonical_sign(psi: np.ndarray) -> np.ndarray:
    """Fix the sign of an eigenvector: largest-magnitude entry positive (lowest
    index wins ties)."""
    i = int(np.argmax(np.abs(psi)))
    return psi if psi[i] >= 0 else -psi


def ground_state(model, *, v0_seed: int = 7542, dense_max: int = 4096, tol: float = 1e-12,
                 reorth: Optional[bool] = None, want_vector: bool = True):
    """E0 (and psi) of a model sector: dense eigh up to `dense_max`, else Lanczos
    on the oracle CSR with the SplitMix64 start vector."""
    sec = Sector(model, explicit_keys=True)
    if sec.dim <= dense_max:
        e0, psi = dense_ground_state(sec.dense())
        return sec, e0, canonical_sign(psi)
    csr = sec.csr()
    v0 = start_vector(v0_seed, sec.dim)
    if reorth is None:
        reorth = sec.dim <= 200_000
    r = lanczos(lambda x: spmv(csr, x), sec.dim, v0, tol=tol, reorth=reorth, want_vector=want_vector)
    return sec, r.e0, (canonical_sign(r.psi) if r.psi is not None else None)
