"""Python binding of libhubbard (ctypes): argument marshalling only.

Every step of the computation runs in the HIP kernels behind the C ABI declared
in ``include/hubbard.h``; PyTorch only provides device memory and the stream.
Importing works without a GPU, but any call that needs the library raises if
``libhubbard.so`` has not been built (``python -m paper_1307_7542_amd._build``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhubbard.so")

HUB_OK = 0
HUB_ERR_NOT_CONVERGED = 5
F64, F32 = 0, 1
SPIN_UP, SPIN_DN = 0, 1

EXPORTED = [
    "hub_sector_create", "hub_sector_destroy", "hub_sector_dims", "hub_sector_bonds", "hub_basis",
    "hub_rank", "hub_hopping_nnz", "hub_hopping_csr", "hub_diagonal", "hub_start_vector",
    "hub_matvec", "hub_ground_state", "hub_param_bilinear", "hub_matvec_bytes", "hub_status_str",
    "hub_last_error", "hub_version", "hub_batch_create", "hub_batch_destroy", "hub_batch_offsets",
    "hub_batch_matvec", "hub_batch_ground_state", "hub_apply_fermion", "hub_lanczos_coefficients",
    "hub_continued_fraction", "hub_greens_function", "hub_sector_create_k0", "hub_k0_layout",
    "hub_set_schedule", "hub_get_schedule", "hub_start_vector_noalloc", "hub_gram",
]

SCHED_AUTO, SCHED_COLUMNS, SCHED_CHUNKED, SCHED_ROWS, SCHED_CSR = 0, 1, 2, 3, 4


class HubError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class _Model(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int32), ("n_bonds", ctypes.c_int32),
        ("bond_i", ctypes.c_void_p), ("bond_j", ctypes.c_void_p),
        ("t", ctypes.c_void_p), ("U", ctypes.c_void_p), ("eps", ctypes.c_void_p),
    ]


class Schedule(ctypes.Structure):
    """hub_schedule: product schedule (family and tile shape)."""
    _fields_ = [
        ("family", ctypes.c_int32), ("tile_cols", ctypes.c_int32), ("block", ctypes.c_int32),
        ("order", ctypes.c_int32), ("quads_per_lane", ctypes.c_int32), ("chunk_rows", ctypes.c_int32),
        ("no_fused_update", ctypes.c_int32), ("ms", ctypes.c_float),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LanczosOpts(ctypes.Structure):
    _fields_ = [
        ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("dev_start", ctypes.c_void_p), ("vec_dtype", ctypes.c_int32), ("reorth", ctypes.c_int32),
        ("want_vector", ctypes.c_int32), ("refine", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("time_kernels", ctypes.c_int32), ("e0_target", ctypes.c_double), ("e0_target_rel", ctypes.c_double),
        ("orth_check", ctypes.c_int32), ("batch_no_graph", ctypes.c_int32),
    ]


class LanczosInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("breakdown", ctypes.c_int32),
        ("matvec_count", ctypes.c_int32), ("e0_ritz", ctypes.c_double), ("e0_refined", ctypes.c_double),
        ("residual", ctypes.c_double), ("true_residual", ctypes.c_double), ("seconds", ctypes.c_double),
        ("seconds_to_e0", ctypes.c_double), ("matvec_ms", ctypes.c_double), ("matvec_bytes", ctypes.c_int64),
        ("iters_to_target", ctypes.c_int32), ("seconds_to_target", ctypes.c_double),
        ("matvec_timed", ctypes.c_int32), ("reorth_steps", ctypes.c_int32), ("orth_loss", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libhubbard.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        sig = {
            "hub_sector_create": (i32, [P, i32, i32, P]),
            "hub_sector_destroy": (None, [P]),
            "hub_sector_dims": (i32, [P, P, P, P]),
            "hub_sector_bonds": (i32, [P, P, P, P, P]),
            "hub_basis": (i32, [P, i32, P]),
            "hub_rank": (i32, [P, i32, P, i64, P]),
            "hub_hopping_nnz": (i32, [P, i32, P]),
            "hub_hopping_csr": (i32, [P, i32, P, P, P, P]),
            "hub_diagonal": (i32, [P, i32, P, P]),
            "hub_start_vector": (i32, [P, i32, u64, i32, P, P]),
            "hub_start_vector_noalloc": (i32, [P, i32, u64, i32, P, P]),
            "hub_gram": (i32, [i32, P, i32, i64, P, P]),
            "hub_matvec": (i32, [P, i32, P, P, P]),
            "hub_ground_state": (i32, [P, P, P, P, P, P]),
            "hub_param_bilinear": (i32, [P, P, P, P, P, P, P]),
            "hub_matvec_bytes": (i32, [P, i32, P]),
            "hub_batch_create": (i32, [P, i32, P]),
            "hub_batch_destroy": (None, [P]),
            "hub_batch_offsets": (i32, [P, P]),
            "hub_batch_matvec": (i32, [P, i32, P, P, P]),
            "hub_batch_ground_state": (i32, [P, P, P, P, P, P, P]),
            "hub_apply_fermion": (i32, [P, P, i32, i32, i32, P, P, P]),
            "hub_lanczos_coefficients": (i32, [P, P, i32, P, P, P, P, P]),
            "hub_continued_fraction": (i32, [P, P, i32, ctypes.c_double, i32, P, P, P, P]),
            "hub_greens_function": (i32, [P, ctypes.c_double, P, i32, i32, i32, i32, P, P, P, P, P, P, P]),
            "hub_sector_create_k0": (i32, [P, i32, i32, i32, P]),
            "hub_k0_layout": (i32, [P, P, P, P]),
            "hub_set_schedule": (i32, [P, i32, P]),
            "hub_get_schedule": (i32, [P, i32, i32, P]),
            "hub_status_str": (ctypes.c_char_p, [i32]),
            "hub_last_error": (ctypes.c_char_p, []),
            "hub_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int, where: str, allow=(HUB_OK,)):
    if status not in allow:
        L = lib()
        raise HubError(status, where, f"{L.hub_status_str(status).decode()}: {L.hub_last_error().decode()}")
    return status


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype_code: int, n: int, name: str):
    torch = _torch()
    want = torch.float64 if dtype_code == F64 else torch.float32
    if not t.is_cuda or t.dtype != want or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous CUDA {want} tensor with {n} elements")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class GroundState:
    e0: float
    psi: Optional[object]
    info: dict


class Sector:
    """One (N_up, N_dn) sector of a Hubbard / Anderson model on the GPU.

    `model` is any object with attributes n_sites, bonds [(i, j)], t, U (per
    site) and eps (per site), plus n_up / n_dn unless given here."""

    def __init__(self, model, n_up: Optional[int] = None, n_dn: Optional[int] = None, translation: int = 0):
        """translation = w > 0: the k = 0 block under the relabelling i -> i - w (mod M)."""
        L = lib()
        M = int(model.n_sites)
        self.n_up = int(model.n_up if n_up is None else n_up)
        self.n_dn = int(model.n_dn if n_dn is None else n_dn)
        self._bi = np.ascontiguousarray([b[0] for b in model.bonds], dtype=np.int32)
        self._bj = np.ascontiguousarray([b[1] for b in model.bonds], dtype=np.int32)
        self._t = np.ascontiguousarray(model.t, dtype=np.float64)
        self._U = np.ascontiguousarray(model.U, dtype=np.float64)
        self._eps = np.ascontiguousarray(model.eps, dtype=np.float64)
        m = _Model(M, len(self._bi), _ptr(self._bi) if len(self._bi) else None,
                   _ptr(self._bj) if len(self._bj) else None, _ptr(self._t) if len(self._t) else None,
                   _ptr(self._U), _ptr(self._eps))
        h = ctypes.c_void_p()
        if translation:
            _check(L.hub_sector_create_k0(ctypes.byref(m), self.n_up, self.n_dn, int(translation), ctypes.byref(h)),
                   "hub_sector_create_k0")
        else:
            _check(L.hub_sector_create(ctypes.byref(m), self.n_up, self.n_dn, ctypes.byref(h)), "hub_sector_create")
        self.translation = int(translation)
        self._h = h
        self.M = M
        cu, cd, dim = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(L.hub_sector_dims(h, ctypes.byref(cu), ctypes.byref(cd), ctypes.byref(dim)), "hub_sector_dims")
        self.count_up, self.count_dn, self.dim = cu.value, cd.value, dim.value

    def close(self):
        if getattr(self, "_h", None):
            lib().hub_sector_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ tables
    def bonds(self):
        n = ctypes.c_int32()
        _check(lib().hub_sector_bonds(self._h, ctypes.byref(n), None, None, None), "hub_sector_bonds")
        bi = np.zeros(n.value, dtype=np.int32)
        bj = np.zeros(n.value, dtype=np.int32)
        t = np.zeros(n.value, dtype=np.float64)
        _check(lib().hub_sector_bonds(self._h, ctypes.byref(n), _ptr(bi), _ptr(bj), _ptr(t)), "hub_sector_bonds")
        return bi, bj, t

    def count(self, spin: int) -> int:
        return self.count_up if spin == SPIN_UP else self.count_dn

    def basis(self, spin: int) -> np.ndarray:
        out = np.zeros(self.count(spin), dtype=np.uint64)
        _check(lib().hub_basis(self._h, spin, _ptr(out)), "hub_basis")
        return out

    def rank(self, spin: int, xs: Sequence[int]) -> np.ndarray:
        x = np.ascontiguousarray(xs, dtype=np.uint64)
        out = np.zeros(len(x), dtype=np.int64)
        if len(x):
            _check(lib().hub_rank(self._h, spin, _ptr(x), len(x), _ptr(out)), "hub_rank")
        return out

    def hopping_nnz(self, spin: int) -> int:
        n = ctypes.c_int64()
        _check(lib().hub_hopping_nnz(self._h, spin, ctypes.byref(n)), "hub_hopping_nnz")
        return n.value

    def hopping_csr(self, spin: int):
        nnz = self.hopping_nnz(spin)
        rp = np.zeros(self.count(spin) + 1, dtype=np.int64)
        col = np.zeros(max(nnz, 1), dtype=np.int32)
        val = np.zeros(max(nnz, 1), dtype=np.float64)
        bond = np.zeros(max(nnz, 1), dtype=np.int32)
        _check(lib().hub_hopping_csr(self._h, spin, _ptr(rp), _ptr(col), _ptr(val), _ptr(bond)), "hub_hopping_csr")
        return rp, col[:nnz], val[:nnz], bond[:nnz]

    def set_schedule(self, dtype: int, family: Optional[int] = None, *, tile_cols: int = 1, block: int = 1024,
                     order: int = 1, quads_per_lane: int = 4, chunk_rows: int = 0, no_fused_update: bool = False):
        """Force the product schedule of `dtype` (family None: back to the tuned one)."""
        if family is None:
            _check(lib().hub_set_schedule(self._h, dtype, None), "hub_set_schedule")
            return
        if family == SCHED_CHUNKED:
            order, block = 0, 1024
        sc = Schedule(family, tile_cols, block, order, quads_per_lane, chunk_rows, int(no_fused_update), 0.0)
        _check(lib().hub_set_schedule(self._h, dtype, ctypes.byref(sc)), "hub_set_schedule")

    def schedule(self, dtype: int = F64, fused: bool = False) -> dict:
        """The product schedule in use (family 0: not chosen yet)."""
        sc = Schedule()
        _check(lib().hub_get_schedule(self._h, dtype, int(fused), ctypes.byref(sc)), "hub_get_schedule")
        return sc.as_dict()

    def matvec_bytes(self, dtype: int = F64) -> int:
        b = ctypes.c_int64()
        _check(lib().hub_matvec_bytes(self._h, dtype, ctypes.byref(b)), "hub_matvec_bytes")
        return b.value

    # ------------------------------------------------------------ vectors
    def empty(self, dtype: int = F64, device="cuda"):
        torch = _torch()
        return torch.empty(self.dim, dtype=torch.float64 if dtype == F64 else torch.float32, device=device)

    def diagonal(self, dtype: int = F64, out=None, stream=None):
        out = self.empty(dtype) if out is None else out
        _check(lib().hub_diagonal(self._h, dtype, _dev_ptr(out, dtype, self.dim, "out"), _stream(stream)),
               "hub_diagonal")
        return out

    def start_vector(self, seed: int, dtype: int = F64, normalize: bool = True, out=None, stream=None,
                     noalloc: bool = False):
        """noalloc: hub_start_vector_noalloc (static scratch, no allocation, no synchronisation)."""
        out = self.empty(dtype) if out is None else out
        fn = lib().hub_start_vector_noalloc if noalloc else lib().hub_start_vector
        _check(fn(self._h, dtype, ctypes.c_uint64(seed), int(normalize), _dev_ptr(out, dtype, self.dim, "out"),
                  _stream(stream)), "hub_start_vector_noalloc" if noalloc else "hub_start_vector")
        return out

    def matvec(self, x, y=None, stream=None):
        torch = _torch()
        dtype = F64 if x.dtype == torch.float64 else F32
        y = self.empty(dtype, device=x.device) if y is None else y
        _check(lib().hub_matvec(self._h, dtype, _dev_ptr(x, dtype, self.dim, "x"),
                                _dev_ptr(y, dtype, self.dim, "y"), _stream(stream)), "hub_matvec")
        return y

    def ground_state(self, *, dtype: int = F64, reorth=False, want_vector: bool = True,
                     refine: bool = False, max_iter: int = 400, tol: float = 0.0, seed: int = 7542,
                     start=None, check_every: int = 1, time_kernels: int = 0, psi=None,
                     stream=None, allow_not_converged: bool = False, e0_target: Optional[float] = None,
                     e0_target_rel: float = 0.0, orth_check: bool = False) -> GroundState:
        """reorth: False / 0 plain recurrence, True / 1 / "full" full, 2 / "partial" partial
        reorthogonalisation (Simon's omega recurrence)."""
        ro = {"full": 1, "partial": 2}.get(reorth, reorth) if isinstance(reorth, str) else int(reorth)
        want = want_vector or refine
        if want and psi is None:
            psi = self.empty(F64)
        o = LanczosOpts(max_iter, tol, seed,
                        _dev_ptr(start, F64, self.dim, "start") if start is not None else None,
                        dtype, ro, int(want_vector), int(refine), check_every, int(time_kernels),
                        float(e0_target or 0.0), float(e0_target_rel if e0_target is not None else 0.0),
                        int(orth_check))
        info = LanczosInfo()
        e0 = ctypes.c_double()
        allow = (HUB_OK, HUB_ERR_NOT_CONVERGED) if allow_not_converged else (HUB_OK,)
        _check(lib().hub_ground_state(self._h, ctypes.byref(o), ctypes.byref(e0),
                                      _dev_ptr(psi, F64, self.dim, "psi") if want else None,
                                      _stream(stream), ctypes.byref(info)), "hub_ground_state", allow)
        return GroundState(e0.value, psi if want else None, info.as_dict())

    def k0_layout(self):
        """(reps, periods) of a translation sector: rows of its vectors."""
        n = ctypes.c_int64()
        _check(lib().hub_k0_layout(self._h, ctypes.byref(n), None, None), "hub_k0_layout")
        reps = np.zeros(n.value, dtype=np.uint64)
        per = np.zeros(n.value, dtype=np.int32)
        _check(lib().hub_k0_layout(self._h, ctypes.byref(n), _ptr(reps), _ptr(per)), "hub_k0_layout")
        return reps, per

    # ------------------------------------------------ Green's function
    def apply_fermion(self, dst: "Sector", site: int, spin: int, create: bool, x, y=None, stream=None):
        """y = c+_{site,spin} x (create) or c_{site,spin} x into sector `dst` (FP64)."""
        y = dst.empty(F64) if y is None else y
        _check(lib().hub_apply_fermion(self._h, dst._h, int(site), int(spin), int(bool(create)),
                                       _dev_ptr(x, F64, self.dim, "x"), _dev_ptr(y, F64, dst.dim, "y"),
                                       _stream(stream)), "hub_apply_fermion")
        return y

    def lanczos_coefficients(self, f, max_steps: int, stream=None):
        """(alpha, beta, norm2, steps) of <f|(w - H)^-1|f> by plain FP64 Lanczos."""
        a = np.zeros(max_steps + 1)
        b = np.zeros(max_steps + 1)
        n2 = ctypes.c_double()
        m = ctypes.c_int32()
        _check(lib().hub_lanczos_coefficients(self._h, _dev_ptr(f, F64, self.dim, "f"), int(max_steps), _ptr(a),
                                              _ptr(b), ctypes.byref(n2), ctypes.byref(m), _stream(stream)),
               "hub_lanczos_coefficients")
        return a, b, n2.value, m.value

    def greens_function(self, e0: float, psi, site: int, spin: int, z, max_steps: int = 200, stream=None):
        """Zero-temperature G_spin(site, z) at complex points z; returns
        (G, info, coefficients [alpha_p, beta_p, alpha_h, beta_h])."""
        z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
        zr = np.ascontiguousarray(z.real)
        zi = np.ascontiguousarray(z.imag)
        gr = np.zeros(len(z))
        gi = np.zeros(len(z))
        coef = np.zeros((4, max_steps + 1))
        info = GfInfo()
        _check(lib().hub_greens_function(self._h, float(e0), _dev_ptr(psi, F64, self.dim, "psi"), int(site),
                                         int(spin), int(max_steps), len(z), _ptr(zr), _ptr(zi), _ptr(gr), _ptr(gi),
                                         _ptr(coef), ctypes.byref(info), _stream(stream)), "hub_greens_function")
        return gr + 1j * gi, info.as_dict(), coef

    def param_bilinear(self, g, x, stream=None):
        """(dbond, dU, deps) = g^T (dH/dtheta) x for canonical bonds, U_i and eps_i."""
        nb = len(self.bonds()[0])
        db = np.zeros(max(nb, 1))
        dU = np.zeros(self.M)
        de = np.zeros(self.M)
        _check(lib().hub_param_bilinear(self._h, _dev_ptr(g, F64, self.dim, "g"), _dev_ptr(x, F64, self.dim, "x"),
                                        _ptr(db), _ptr(dU), _ptr(de), _stream(stream)), "hub_param_bilinear")
        return db[:nb], dU, de


class GfInfo(ctypes.Structure):
    _fields_ = [
        ("steps_particle", ctypes.c_int32), ("steps_hole", ctypes.c_int32), ("norm2_particle", ctypes.c_double),
        ("norm2_hole", ctypes.c_double), ("seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def continued_fraction(alpha, beta, steps: int, norm2: float, w) -> np.ndarray:
    """<f|(w - H)^-1|f> from Lanczos coefficients, at complex points w."""
    w = np.atleast_1d(np.asarray(w, dtype=np.complex128))
    wr = np.ascontiguousarray(w.real)
    wi = np.ascontiguousarray(w.imag)
    orr = np.zeros(len(w))
    oi = np.zeros(len(w))
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    _check(lib().hub_continued_fraction(_ptr(a), _ptr(b), int(steps), float(norm2), len(w), _ptr(wr), _ptr(wi),
                                        _ptr(orr), _ptr(oi)), "hub_continued_fraction")
    return orr + 1j * oi


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int32), ("graph_replays", ctypes.c_int32), ("rows_per_lane", ctypes.c_int32),
        ("block_size", ctypes.c_int32), ("cols_per_lane", ctypes.c_int32), ("seconds", ctypes.c_double), ("tune_seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Batch:
    """Independent sectors solved together (one product launch for all of
    them, lockstep Lanczos replayed from a captured HIP graph).  Batch vectors
    concatenate the sector vectors in order; `offsets` gives the slices."""

    def __init__(self, sectors: Sequence[Sector]):
        self.sectors = list(sectors)  # keep them alive
        arr = (ctypes.c_void_p * len(self.sectors))(*[s._h.value for s in self.sectors])
        h = ctypes.c_void_p()
        _check(lib().hub_batch_create(arr, len(self.sectors), ctypes.byref(h)), "hub_batch_create")
        self._h = h
        off = np.zeros(len(self.sectors) + 1, dtype=np.int64)
        _check(lib().hub_batch_offsets(h, _ptr(off)), "hub_batch_offsets")
        self.offsets = off
        self.total = int(off[-1])

    def close(self):
        if getattr(self, "_h", None):
            lib().hub_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self, dtype: int = F64):
        torch = _torch()
        return torch.empty(self.total, dtype=torch.float64 if dtype == F64 else torch.float32, device="cuda")

    def matvec(self, x, y=None, stream=None):
        torch = _torch()
        dtype = F64 if x.dtype == torch.float64 else F32
        y = self.empty(dtype) if y is None else y
        _check(lib().hub_batch_matvec(self._h, dtype, _dev_ptr(x, dtype, self.total, "x"),
                                      _dev_ptr(y, dtype, self.total, "y"), _stream(stream)), "hub_batch_matvec")
        return y

    def ground_state(self, *, dtype: int = F64, want_vector: bool = False, refine: bool = False,
                     max_iter: int = 400, tol: float = 0.0, seed: int = 7542, check_every: int = 5,
                     stream=None, allow_not_converged: bool = False, graph: bool = True):
        want = want_vector or refine
        psi = self.empty(F64) if want else None
        o = LanczosOpts(max_iter, tol, seed, None, dtype, 0, int(want_vector), int(refine), check_every, 0, 0.0, 0.0,
                        0, int(not graph))
        e0 = np.zeros(len(self.sectors))
        it = np.zeros(len(self.sectors), dtype=np.int32)
        info = BatchInfo()
        allow = (HUB_OK, HUB_ERR_NOT_CONVERGED) if allow_not_converged else (HUB_OK,)
        _check(lib().hub_batch_ground_state(self._h, ctypes.byref(o), _ptr(e0), _ptr(it),
                                            _dev_ptr(psi, F64, self.total, "psi") if want else None,
                                            _stream(stream), ctypes.byref(info)), "hub_batch_ground_state", allow)
        return e0, it, psi, info.as_dict()


def version() -> str:
    return lib().hub_version().decode()


def gram(vectors, stream=None) -> np.ndarray:
    """G = Q^T Q (FP64, on the FP64 matrix cores) of equal-length contiguous CUDA
    vectors of one dtype (hub_gram)."""
    torch = _torch()
    if not vectors:
        return np.zeros((0, 0))
    dt = F64 if vectors[0].dtype == torch.float64 else F32
    n = vectors[0].numel()
    ptrs = (ctypes.c_void_p * len(vectors))(*[_dev_ptr(v, dt, n, "vector").value for v in vectors])
    out = np.zeros((len(vectors), len(vectors)), dtype=np.float64)
    _check(lib().hub_gram(dt, ptrs, len(vectors), n, _ptr(out), _stream(stream)), "hub_gram")
    return out
