"""Oracle for translation symmetry, k = 0 (Sec. VI).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Translation G acts on an M-bit occupation integer by lowering every bit
position by w (cyclically): G x = rotr(x, w).  With w = 1 this is the paper's
T; the direction is the one that reproduces Tables V and VI (representatives
are the smallest integer of their cycle, and 1001 is one translation of
0011).  Applied to a ket whose creation operators are in increasing site
order, G moves the k operators of the lowest w sites to the top, past the
other N - k, so G|x> = (-1)^(k (N - k)) |G x>.  On the two-spin kets of
Sec. II (all up operators, then all down ones) G acts on each block, and
the signs multiply.

* ``spin_orbits``: period, representative, translation and phase of every
  one-spin basis state (Table VI's per / rep / trans / esign_trans, and
  esignb).
* ``period_counts``: representatives per period by direct orbit counting;
  ``period_counts_formula``: Eq. (count6) with the number of states of exact
  period i subtracted for each proper period i.
* ``combined_reps``: Eq. (count7) enumeration (Table V).
* ``k0_basis``: the k = 0 subspace of a two-spin sector from its definition:
  every cycle of two-spin keys under G whose accumulated phase around the
  cycle is +1 gives the unit vector L^-1/2 sum_r G^r|c>; cycles with phase -1
  have no k = 0 component.  H_k0 = B^T H B with the oracle's full CSR H.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import OracleModel, Sector, enumerate_basis


def rotr(x: int, M: int, w: int) -> int:
    mask = (1 << M) - 1
    return ((x >> w) | (x << (M - w))) & mask


def gsign(x: int, N: int, w: int) -> int:
    k = bin(x & ((1 << w) - 1)).count("1")
    return -1 if (k * (N - k)) % 2 else 1


@dataclass
class SpinOrbitTables:
    basis: np.ndarray        # Algorithm I order
    rep: np.ndarray          # representative integer of each basis state
    trans: np.ndarray        # s with G^s rep = state
    esign: np.ndarray        # G^s |rep> = esign |state>
    period: np.ndarray       # period of the state's cycle
    esignb: np.ndarray       # G^period |rep> = esignb |rep>


def spin_orbits(M: int, N: int, w: int = 1) -> SpinOrbitTables:
    basis = enumerate_basis(M, N)
    n = len(basis)
    rep = np.zeros(n, dtype=np.int64)
    trans = np.zeros(n, dtype=np.int64)
    esign = np.zeros(n, dtype=np.int64)
    period = np.zeros(n, dtype=np.int64)
    esignb = np.zeros(n, dtype=np.int64)
    index = {int(x): k for k, x in enumerate(basis)}
    done = np.zeros(n, dtype=bool)
    for k0, x0 in enumerate(basis):
        if done[k0]:
            continue
        # walk the cycle from x0, recording the phase of G^r |x0>
        cyc, ph = [int(x0)], [1]
        y, s = int(x0), 1
        while True:
            s *= gsign(y, N, w)
            y = rotr(y, M, w)
            if y == int(x0):
                break
            cyc.append(y)
            ph.append(s)
        back = s  # G^P |x0> = back |x0>
        P = len(cyc)
        r = cyc.index(min(cyc))
        # re-express relative to the representative: G^j |rep> for j = 0..P-1
        for j in range(P):
            t = (r + j) % P
            phase = ph[t] * ph[r]          # G^t|x0> = ph[t]|..>, G^r|x0> = ph[r]|rep>
            if r + j >= P:
                phase *= back              # wrapped once around the cycle
            k = index[cyc[t]]
            rep[k], trans[k], esign[k], period[k], esignb[k] = cyc[r], j, phase, P, back
            done[k] = True
    return SpinOrbitTables(basis, rep, trans, esign, period, esignb)


def valid_periods(M: int, N: int, w: int = 1):
    """Periods z (in units of G) allowed by Eqs. (count4) and (count5)."""
    L = M // w
    return [z for z in range(L, 0, -1) if L % z == 0 and (N * z) % L == 0 and (N * z) // L <= z * w]


def period_counts(M: int, N: int, w: int = 1) -> dict:
    t = spin_orbits(M, N, w)
    out = {}
    for p in np.unique(t.period):
        out[int(p)] = int(np.sum((t.period == p) & (t.trans == 0)))
    return out


def period_counts_formula(M: int, N: int, w: int = 1) -> dict:
    """Eq. (count6) for w = 1: (C(z, y_z) - sum_i i nstate(i)) / z over the
    proper periods i of z, y_b = N b / M."""
    assert w == 1
    out = {}
    for z in sorted(valid_periods(M, N, 1)):
        y = N * z // M
        sub = sum(i * out[i] for i in out if z % i == 0 and i < z)
        out[z] = (math.comb(z, y) - sub) // z
    return out


def period_counts_printed(M: int, N: int) -> dict:
    """Eq. (count6) exactly as printed: C(i, y_i) subtracted for each proper period i."""
    out = {}
    for z in sorted(valid_periods(M, N, 1)):
        y = N * z // M
        sub = sum(math.comb(i, N * i // M) for i in valid_periods(M, N, 1) if i < z and z % i == 0)
        out[z] = (math.comb(z, y) - sub) / z
    return out


def paper_spin_table(M: int, N: int):
    """Table VI columns: per (1-based index of the period in decreasing order),
    rep (1-based index of the representative within its period, increasing
    integers), trans, esign_trans; one row per basis state."""
    t = spin_orbits(M, N, 1)
    periods = sorted(set(int(p) for p in t.period), reverse=True)
    reps_of = {p: sorted(set(int(r) for r, q in zip(t.rep, t.period) if q == p)) for p in periods}
    rows = []
    for k, x in enumerate(t.basis):
        p = int(t.period[k])
        rows.append((int(x), periods.index(p) + 1, reps_of[p].index(int(t.rep[k])) + 1, int(t.trans[k]),
                     int(t.esign[k])))
    return rows


def combined_reps(M: int, n_up: int, n_dn: int):
    """Eq. (count7): |r_up> T^n |r_dn>, n = 0 .. gcd(P_up, P_dn) - 1, up
    representatives outer (periods decreasing, integers increasing), then down."""
    tu, td = spin_orbits(M, n_up, 1), spin_orbits(M, n_dn, 1)

    def reps(t):
        out = []
        for p in sorted(set(int(q) for q in t.period), reverse=True):
            out += [(int(r), p) for r in sorted(set(int(r) for r, q in zip(t.rep, t.period) if q == p))]
        return out

    rows = []
    for ru, pu in reps(tu):
        for rd, pd in reps(td):
            y = rd
            for n in range(math.gcd(pu, pd)):
                rows.append((ru, rd, n, y))
                y = rotr(y, M, 1)
    return rows


def _key_rotate(keys: np.ndarray, M: int, w: int, n_up: int, n_dn: int):
    """G on two-spin keys (vectorised): new keys and phases."""
    mask = np.uint64((1 << M) - 1)
    low = np.uint64((1 << w) - 1)
    up = keys & mask
    dn = keys >> np.uint64(M)

    def rot(x):
        return ((x >> np.uint64(w)) | (x << np.uint64(M - w))) & mask

    def sgn(x, N):
        k = np.bitwise_count(x & low).astype(np.int64)
        return np.where((k * (N - k)) % 2 == 1, -1.0, 1.0)

    return rot(up) | (rot(dn) << np.uint64(M)), sgn(up, n_up) * sgn(dn, n_dn)


def translation_operator(sec: Sector, w: int = 1) -> sp.csr_matrix:
    """G on the sector as a signed permutation matrix (full two-spin basis)."""
    keys = sec.keys.astype(np.uint64)
    new, ph = _key_rotate(keys, sec.m.M, w, sec.m.n_up, sec.m.n_dn)
    rows = np.searchsorted(keys, new)
    assert np.all(keys[rows] == new)
    return sp.csr_matrix((ph, (rows, np.arange(len(keys)))), shape=(len(keys), len(keys)))


def k0_basis(sec: Sector, w: int = 1) -> sp.csr_matrix:
    """Columns: the orthonormal k = 0 states, one per cycle with phase +1,
    ordered by the smallest key of the cycle."""
    M = sec.m.M
    keys = sec.keys.astype(np.uint64)
    n = len(keys)
    G = translation_operator(sec, w)
    img = G.indices[np.argsort(G.indices)]  # not used; G is a permutation
    del img
    perm_to = np.zeros(n, dtype=np.int64)   # index of G c
    phase = np.zeros(n)
    Gc = G.tocoo()
    perm_to[Gc.col] = Gc.row
    phase[Gc.col] = Gc.data
    seen = np.zeros(n, dtype=bool)
    rows, cols, vals = [], [], []
    ncol = 0
    for c in range(n):          # keys ascending: c is the smallest key of its cycle when first seen
        if seen[c]:
            continue
        members, ph = [c], [1.0]
        s, y = 1.0, c
        while True:
            s *= phase[y]
            y = perm_to[y]
            if y == c:
                break
            members.append(y)
            ph.append(s)
        for m_ in members:
            seen[m_] = True
        if s < 0:               # G^L |c> = -|c>: no k = 0 state on this cycle
            continue
        L = len(members)
        rows += members
        cols += [ncol] * L
        vals += [p / math.sqrt(L) for p in ph]
        ncol += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, ncol))


def k0_hamiltonian(model, w: int = 1):
    m = model if isinstance(model, OracleModel) else OracleModel.from_model(model)
    sec = Sector(m)
    B = k0_basis(sec, w)
    rp, col, val = sec.csr()
    H = sp.csr_matrix((val, col, rp), shape=(sec.dim, sec.dim))
    return sec, B, (B.T @ H @ B).tocsr(), H


def k0_project(sec: Sector, x: np.ndarray, w: int = 1) -> np.ndarray:
    """(1/L) sum_r G^r x on the full two-spin space."""
    L = sec.m.M // w
    G = translation_operator(sec, w)
    acc = x.copy()
    y = x.copy()
    for _ in range(L - 1):
        y = G @ y
        acc += y
    return acc / L


def rep_layout(sec: Sector, w: int = 1):
    """Up representatives (ascending) with their periods, for the layout in
    which a k = 0 state is stored as phi[i, b] = sqrt(P_i) psi(R_i, b) over every
    down state b (b in Algorithm I order)."""
    t = spin_orbits(sec.m.M, sec.m.n_up, w)
    sel = t.trans == 0
    order = np.argsort(t.basis[sel])
    return t.basis[sel][order].astype(np.int64), t.period[sel][order].astype(np.int64)


def restrict(sec: Sector, psi: np.ndarray, reps: np.ndarray, periods: np.ndarray) -> np.ndarray:
    """phi[i + b R] = sqrt(P_i) psi(key(R_i, b)) (column-major, R rows)."""
    M = sec.m.M
    keys = sec.keys.astype(np.uint64)
    dn = np.array(sec.dn, dtype=np.uint64)
    R = len(reps)
    want = (np.array(reps, dtype=np.uint64)[:, None] | (dn[None, :] << np.uint64(M))).reshape(-1, order="F")
    idx = np.searchsorted(keys, want)
    assert np.all(keys[idx] == want)
    scale = np.sqrt(np.tile(np.asarray(periods, dtype=float), len(dn)))
    return scale * psi[idx]
