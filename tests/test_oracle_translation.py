"""Pins of the translation-symmetry oracle (Sec. VI): Tables V and VI, the
stated phase T^2|0101> = -|0101>, the representative counts of Eq. (count6),
and the k = 0 block against an independent construction (range of the group
projector (1/L) sum_r T^r, found by SVD), [H, T] = 0 and T^L = 1.  CPU only."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import oracle.translation as ot
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_table6_spin_table():
    ref = {int(r[0], 2): tuple(r[1:]) for r in _load("table6_m4_n2.json")["rows"]}
    got = {x: rest for x, *rest in ot.paper_spin_table(4, 2)}
    assert {k: tuple(v) for k, v in got.items()} == ref


def test_t_squared_on_0101():
    t = ot.spin_orbits(4, 2)
    k = list(t.basis).index(0b0101)
    assert t.period[k] == 2 and t.esignb[k] == -1


def test_table5_combined_representatives():
    ref = [(int(a, 2), int(b, 2), n, int(c, 2)) for a, b, n, c, _ in _load("table5_m4_n2_1.json")["rows"]]
    assert ot.combined_reps(4, 2, 1) == ref
    # and the k = 0 block of that sector has exactly these six states
    m = W.ring(4, U=3.0, n_up=2, n_dn=1)
    assert ot.k0_basis(oracle.Sector(m)).shape[1] == 6


@pytest.mark.parametrize("M,N", [(4, 2), (6, 2), (6, 3), (8, 4), (9, 3), (10, 4), (12, 6), (12, 4), (14, 7), (16, 8)])
def test_representative_counts(M, N):
    """Direct cycle counts against Eq. (count6) with the states of exact period i
    subtracted; the printed form (C(i, y_i) subtracted) agrees whenever z has at
    most one proper period below it."""
    direct = ot.period_counts(M, N)
    assert direct == ot.period_counts_formula(M, N)
    assert sum(z * n for z, n in direct.items()) == len(oracle.enumerate_basis(M, N))
    printed = ot.period_counts_printed(M, N)
    for z, n in direct.items():
        proper = [i for i in direct if i < z and z % i == 0]
        if len(proper) <= 1:
            assert printed[z] == n


def _models():
    return [
        (W.ring(6, U=4.0, n_up=3, n_dn=3), 1),
        (W.ring(6, U=4.0, n_up=2, n_dn=3), 1),
        (W.ring(6, U=2.5, n_up=2, n_dn=2), 1),
        (W.ring(8, U=2.0, n_up=4, n_dn=2), 1),
        (W.ring(4, U=3.0, n_up=2, n_dn=1), 1),
        (W.ring(8, U=2.0, n_up=4, n_dn=4), 2),
        (W.ladder(3, rung_lo=0.7, rung_hi=0.7).with_params(n_up=3, n_dn=2), 2),
    ]


@pytest.mark.parametrize("idx", range(7))
def test_k0_block_against_group_projector(idx):
    m, w = _models()[idx]
    sec, B, Hk, H = ot.k0_hamiltonian(m, w)
    Hd = H.toarray()
    G = ot.translation_operator(sec, w).toarray()
    L = m.n_sites // w
    assert np.array_equal(G @ Hd, Hd @ G)                                       # [H, T] = 0
    assert np.array_equal(np.linalg.matrix_power(G, L), np.eye(sec.dim))       # T^L = 1
    P = sum(np.linalg.matrix_power(G, r) for r in range(L)) / L
    assert B.shape[1] == round(np.trace(P))
    U_, s_, _ = np.linalg.svd(P)
    Q = U_[:, s_ > 0.5]
    wq = np.linalg.eigvalsh(Q.T @ Hd @ Q)
    wk = np.linalg.eigvalsh(Hk.toarray())
    np.testing.assert_allclose(np.sort(wk), np.sort(wq), rtol=0, atol=1e-12)
    w_full = np.linalg.eigvalsh(Hd)
    assert max(np.min(np.abs(w_full - x)) for x in wk) <= 1e-12
    # the layout (up representative, every down state) is an isometry on k = 0 vectors
    x0 = ot.k0_project(sec, oracle.start_vector(3, sec.dim), w)
    reps, per = ot.rep_layout(sec, w)
    phi = ot.restrict(sec, x0, reps, per)
    assert abs(np.linalg.norm(phi) - np.linalg.norm(x0)) <= 1e-14 * np.linalg.norm(x0)


def test_odd_filling_ring_ground_state_has_k0():
    """Half-filled ring with odd N per spin: the ground state lies in k = 0."""
    m = W.ring(6, U=4.0, n_up=3, n_dn=3)
    sec, B, Hk, H = ot.k0_hamiltonian(m)
    e_full = np.linalg.eigvalsh(H.toarray())[0]
    e_k0 = np.linalg.eigvalsh(Hk.toarray())[0]
    assert abs(e_full - e_k0) <= 1e-12
