"""Pins of the Green's-function oracle (Sec. VII A) against things it does not
compute itself: Jordan-Wigner Fock-space operators, canonical anticommutation,
the non-interacting resolvent, the Hubbard atom, the sum rule, the 1/z tail and
particle-hole symmetry.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import oracle.greens as og
import workloads as W


def _fock_c(M, m):
    """Annihilator of mode m on the 2^(2M) Fock space: a on mode m, Z on the
    modes below m (creation operators ordered by increasing mode)."""
    a = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))
    Z = sp.csr_matrix(np.diag([1.0, -1.0]))
    I2 = sp.identity(2, format="csr")
    op = sp.identity(1, format="csr")
    for k in range(2 * M - 1, -1, -1):  # first factor = most significant bit
        op = sp.kron(op, a if k == m else (Z if k < m else I2), format="csr")
    return op


def _matsubara(beta=10.0, n=12):
    return 1j * np.pi * (2 * np.arange(n) + 1) / beta


@pytest.mark.parametrize("seed,M", [(11, 3), (12, 4)])
def test_fermion_operator_matches_jordan_wigner(seed, M):
    base = W.random_graph(M, M + 1, seed=seed, site_U=True)
    for spin in (0, 1):
        for site in range(M):
            c = _fock_c(M, site + spin * M)
            cdag = c.T.tocsr()
            for n_up in range(M + 1):
                for n_dn in range(M + 1):
                    src = oracle.Sector(base.with_params(n_up=n_up, n_dn=n_dn))
                    for create, d in ((True, 1), (False, -1)):
                        nu = n_up + (d if spin == 0 else 0)
                        nd = n_dn + (d if spin == 1 else 0)
                        if not (0 <= nu <= M and 0 <= nd <= M):
                            continue
                        dst = oracle.Sector(base.with_params(n_up=nu, n_dn=nd))
                        got = og.fermion_operator(src, dst, site, spin, create).toarray()
                        ref = (cdag if create else c)[dst.keys.astype(np.int64)][:, src.keys.astype(np.int64)]
                        np.testing.assert_array_equal(got, ref.toarray())


def test_anticommutators_within_a_sector():
    """{c_m, c+_m'} = delta_mm' on the (2, 3) sector of a 5-site lattice."""
    m = W.random_graph(5, 6, seed=3).with_params(n_up=2, n_dn=3)
    src = oracle.Sector(m)
    M = 5

    def op(site, spin, create, frm):
        d = 1 if create else -1
        to = og.shifted(frm.m, spin, d)
        dst = oracle.Sector(to)
        return og.fermion_operator(frm, dst, site, spin, create), dst

    eye = np.eye(src.dim)
    for s1 in range(2):
        for p1 in range(M):
            for s2 in range(2):
                for p2 in range(M):
                    cd, mid = op(p2, s2, True, src)            # c+_{p2 s2}: N -> N+1
                    c_after, _ = op(p1, s1, False, mid)        # c_{p1 s1}: N+1 -> ...
                    c_first, mid2 = op(p1, s1, False, src)     # c_{p1 s1}: N -> N-1
                    cd_after, _ = op(p2, s2, True, mid2)       # c+_{p2 s2}
                    if s1 != s2:
                        # both products land in the (N_s1 - 1, N_s2 + 1) sector
                        acomm = (c_after @ cd + cd_after @ c_first).toarray()
                        assert np.max(np.abs(acomm)) == 0.0
                        continue
                    acomm = (c_after @ cd + cd_after @ c_first).toarray()
                    ref = eye if p1 == p2 else np.zeros_like(eye)
                    np.testing.assert_array_equal(acomm, ref)


@pytest.mark.parametrize("spin", [0, 1])
def test_u0_green_function_is_the_one_body_resolvent(spin):
    """U = 0, non-degenerate closed-shell ground state: G_s(p, z) = [(z - h)^-1]_pp
    with h the one-body matrix (-t on bonds, eps on the diagonal)."""
    m = W.random_graph(6, 9, seed=21, U=0.0).with_params(n_up=3, n_dn=3)
    h = np.diag(np.array(m.eps, dtype=float))
    for (i, j), t in zip(m.bonds, m.t):
        h[i, j] -= t
        h[j, i] -= t
    lev = np.linalg.eigvalsh(h)
    assert lev[3] - lev[2] > 1e-3  # closed shell
    sec, e0, psi = oracle.ground_state(m)
    z = np.concatenate([_matsubara(), np.array([0.3 + 0.2j, -1.1 + 0.05j])])
    for p in range(6):
        g = og.lehmann(m, p, spin, z, e0, psi, src=sec)
        ref = np.array([np.linalg.inv(zz * np.eye(6) - h)[p, p] for zz in z])
        np.testing.assert_allclose(g, ref, rtol=0, atol=1e-11)


def test_hubbard_atom():
    """One site, U and eps: the poles sit at eps (remove from a singly occupied
    site / add to an empty one) and eps + U (the second electron)."""
    U, eps = 3.0, -0.7
    z = _matsubara()
    atom = W.Model("atom", 1, [], [], [U], [eps], 1, 0)
    for (nu, nd), (g_up, g_dn) in {
        (1, 0): (1 / (z - eps), 1 / (z - eps - U)),
        (1, 1): (1 / (z - eps - U), 1 / (z - eps - U)),
        (0, 0): (1 / (z - eps), 1 / (z - eps)),
    }.items():
        m = atom.with_params(n_up=nu, n_dn=nd)
        sec, e0, psi = oracle.ground_state(m)
        np.testing.assert_allclose(og.lehmann(m, 0, 0, z, e0, psi, src=sec), g_up, rtol=0, atol=1e-14)
        np.testing.assert_allclose(og.lehmann(m, 0, 1, z, e0, psi, src=sec), g_dn, rtol=0, atol=1e-14)


def test_sum_rule_tail_and_particle_hole_symmetry():
    """Half-filled even ring with eps = -U/2 (particle-hole symmetric on a
    bipartite lattice): Re G(i w_n) = 0; z G(z) -> <c c+ + c+ c> = 1; G_up = G_dn."""
    U = 4.0
    m = W.ring(6, U=U, n_up=3, n_dn=3).with_params(eps=[-U / 2] * 6)
    sec, e0, psi = oracle.ground_state(m)
    z = _matsubara()
    for p in (0, 2):
        gu = og.lehmann(m, p, 0, z, e0, psi, src=sec)
        gd = og.lehmann(m, p, 1, z, e0, psi, src=sec)
        assert np.max(np.abs(gu.real)) <= 1e-12
        np.testing.assert_allclose(gu, gd, rtol=0, atol=1e-12)
        big = np.array([1e7j, 1e7 + 1e7j])
        np.testing.assert_allclose(big * og.lehmann(m, p, 0, big, e0, psi, src=sec), 1.0, rtol=0, atol=1e-6)
    # translation invariance of the ring: every site has the same G
    g0 = og.lehmann(m, 0, 0, z, e0, psi, src=sec)
    g4 = og.lehmann(m, 4, 0, z, e0, psi, src=sec)
    np.testing.assert_allclose(g0, g4, rtol=0, atol=1e-12)


def test_continued_fraction_matches_lehmann():
    """Plain Lanczos continued fraction on the oracle CSR against the Lehmann sum
    (different arithmetic: a recurrence versus a full eigendecomposition)."""
    m = W.random_graph(7, 11, seed=601, site_U=True).with_params(n_up=3, n_dn=4)
    sec, e0, psi = oracle.ground_state(m)
    z = np.concatenate([_matsubara(), np.array([0.5 + 0.1j, -2.0 + 0.1j])])
    for spin in (0, 1):
        for p in (0, 3, 6):
            g1 = og.lehmann(m, p, spin, z, e0, psi, src=sec)
            g2 = og.greens_lanczos(m, p, spin, z, e0, psi, steps=400)
            np.testing.assert_allclose(g2, g1, rtol=0, atol=1e-10)


def test_continued_fraction_closed_forms():
    """Two-pole and one-pole fractions written out by hand."""
    w = np.array([0.3 + 1j, -2 + 0.5j])
    np.testing.assert_allclose(og.continued_fraction(np.array([1.5]), np.zeros(0), 2.0, w), 2.0 / (w - 1.5))
    a0, a1, b1 = 0.2, -0.7, 0.9
    ref = 1.0 / (w - a0 - b1 ** 2 / (w - a1))
    np.testing.assert_allclose(og.continued_fraction(np.array([a0, a1]), np.array([b1]), 1.0, w), ref)
    # same two poles from the 2x2 tridiagonal matrix
    lam, vec = np.linalg.eigh(np.array([[a0, b1], [b1, a1]]))
    spec = sum(vec[0, k] ** 2 / (w - lam[k]) for k in range(2))
    np.testing.assert_allclose(ref, spec, rtol=1e-14)
