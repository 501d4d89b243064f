"""Oracle for the zero-temperature one-particle Green's function (Sec. VII A).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Everything here works
in the two-spin basis of Sec. II: the keys I = I_up + 2^M I_dn of a sector,
fermion modes m = site (up) and m = M + site (down).

* ``fermion_operator``: the matrix of c+_m or c_m between two sectors, built
  from its definition on occupation-number kets whose creation operators are
  ordered by increasing mode index (all up sites, then all down sites): c+_m on
  a key with mode m empty gives the key with m set, times (-1) to the number of
  occupied modes below m.  Pinned by the Jordan-Wigner Fock-space operators and
  the anticommutator in ``tests/test_oracle_greens.py``.
* ``lehmann``: G(z) from its spectral (Lehmann) form, summing over every
  eigenstate of the N+1 and N-1 sectors (dense LAPACK ``eigh``): the plain
  definition of the second equation labelled count8.  Pinned by the
  non-interacting resolvent [(z - h)^-1]_pp at U = 0, the Hubbard atom, the
  sum rule and particle-hole symmetry.
* ``lanczos_coefficients`` / ``continued_fraction``: the Lanczos continued
  fraction for <f|(w - H)^-1|f>, for sectors too large for ``lehmann``;
  checked against ``lehmann`` where both run.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import scipy.sparse as sp

from . import OracleModel, Sector, spmv


def shifted(model, spin: int, d: int) -> OracleModel:
    """The same lattice with N_spin changed by d."""
    m = model if isinstance(model, OracleModel) else OracleModel.from_model(model)
    if spin == 0:
        return replace(m, n_up=m.n_up + d)
    return replace(m, n_dn=m.n_dn + d)


def fermion_operator(src: Sector, dst: Sector, site: int, spin: int, create: bool) -> sp.csr_matrix:
    """dst.dim x src.dim matrix of c+_{site,spin} (create) or c_{site,spin}."""
    M = src.m.M
    mode = site + spin * M
    bit = np.uint64(1 << mode)
    keys = src.keys.astype(np.uint64)
    occupied = (keys & bit) != 0
    take = ~occupied if create else occupied
    cols = np.nonzero(take)[0]
    new = keys[cols] ^ bit
    below = np.bitwise_count(keys[cols] & (bit - np.uint64(1))).astype(np.int64)
    dkeys = dst.keys.astype(np.uint64)
    rows = np.searchsorted(dkeys, new)
    assert np.all(dkeys[rows] == new), "target key missing from the destination sector"
    vals = np.where(below % 2 == 1, -1.0, 1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dst.dim, src.dim))


def _eig(model):
    sec = Sector(model)
    w, v = np.linalg.eigh(sec.dense())
    return sec, w, v


def lehmann(model, site: int, spin: int, z, e0: float, psi: np.ndarray, src: Sector = None):
    """G_spin(site, z) = sum_n |<n|c+|psi>|^2 / (z + E0 - E_n)
                        + sum_n |<n|c|psi>|^2 / (z - E0 + E_n)
    over all eigenstates n of the N+1 and N-1 sectors (dense eigh)."""
    m = model if isinstance(model, OracleModel) else OracleModel.from_model(model)
    src = Sector(m) if src is None else src
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    g = np.zeros(len(z), dtype=np.complex128)
    N = m.n_up if spin == 0 else m.n_dn
    if N < m.M:
        sec, w, v = _eig(shifted(m, spin, +1))
        f = fermion_operator(src, sec, site, spin, True) @ psi
        wt = (v.T @ f) ** 2
        g += (wt[None, :] / (z[:, None] + e0 - w[None, :])).sum(axis=1)
    if N > 0:
        sec, w, v = _eig(shifted(m, spin, -1))
        f = fermion_operator(src, sec, site, spin, False) @ psi
        wt = (v.T @ f) ** 2
        g += (wt[None, :] / (z[:, None] - e0 + w[None, :])).sum(axis=1)
    return g


def lanczos_coefficients(matvec, f: np.ndarray, steps: int):
    """Plain Lanczos from v0 = f/|f| (Sec. IV): alpha_0..alpha_{m-1},
    beta_1..beta_{m-1} and |f|^2; stops early on an (exact) breakdown."""
    n2 = float(f @ f)
    if n2 == 0.0:
        return np.zeros(0), np.zeros(0), 0.0
    v = f / np.sqrt(n2)
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    alphas, betas = [], []
    for k in range(min(steps, len(f))):
        w = matvec(v) - b_prev * v_prev
        a = float(w @ v)
        w = w - a * v
        alphas.append(a)
        b = float(np.sqrt(w @ w))
        if k + 1 == min(steps, len(f)) or b <= 1e-13 * (abs(a) + b_prev + 1.0):
            break
        betas.append(b)
        v_prev, v, b_prev = v, w / b, b
    return np.array(alphas), np.array(betas[:len(alphas) - 1]), n2


def continued_fraction(alphas, betas, n2: float, w):
    """n2 / (w - a0 - b1^2 / (w - a1 - b2^2 / ( ... (w - a_{m-1}))))."""
    w = np.atleast_1d(np.asarray(w, dtype=np.complex128))
    if len(alphas) == 0:
        return np.zeros(len(w), dtype=np.complex128)
    d = w - alphas[-1]
    for j in range(len(alphas) - 2, -1, -1):
        d = w - alphas[j] - betas[j] ** 2 / d
    return n2 / d


def greens_lanczos(model, site: int, spin: int, z, e0: float, psi: np.ndarray, steps: int = 300):
    """G_spin(site, z) by the continued fractions of the particle and hole parts
    (oracle CSR products)."""
    m = model if isinstance(model, OracleModel) else OracleModel.from_model(model)
    src = Sector(m)
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    g = np.zeros(len(z), dtype=np.complex128)
    N = m.n_up if spin == 0 else m.n_dn
    for d, create in ((1, True), (-1, False)):
        if (create and N >= m.M) or (not create and N <= 0):
            continue
        sec = Sector(shifted(m, spin, d))
        f = fermion_operator(src, sec, site, spin, create) @ psi
        csr = sec.csr()
        a, b, n2 = lanczos_coefficients(lambda x: spmv(csr, x), f, steps)
        if create:
            g += continued_fraction(a, b, n2, z + e0)
        else:
            g -= continued_fraction(a, b, n2, e0 - z)
    return g
