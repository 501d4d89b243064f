"""GPU tests of the zero-temperature Green's function path (Sec. VII A): the
c+ / c gather kernel (bit-exact against the oracle's two-spin operator), the
continued-fraction Lanczos coefficients, and G(z) against the oracle's Lehmann
sum; full-size properties on the M=14 ring."""
import numpy as np
import pytest

import oracle
import oracle.greens as og
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hub():
    import torch
    import paper_1307_7542_amd as hub
    hub.lib()
    torch.cuda.set_device(0)
    return hub


def _z():
    return np.concatenate([1j * np.pi * (2 * np.arange(20) + 1) / 10.0, [0.5 + 0.1j, -1.0 + 0.1j, 2.0 + 0.1j]])


def _models():
    return [
        W.config("ring8"),
        W.random_graph(7, 11, seed=601, site_U=True).with_params(n_up=3, n_dn=4),
        W.aim_batch(5)[2],
        W.ring(6, U=3.0, n_up=6, n_dn=3),   # up band full: no particle part for spin up
        W.ring(6, U=3.0, n_up=0, n_dn=3),   # no up electrons: no hole part for spin up
    ]


@pytest.mark.parametrize("idx", range(5))
def test_apply_fermion_bit_exact(hub, idx):
    import torch
    m = _models()[idx]
    src = hub.Sector(m)
    osrc = oracle.Sector(m)
    x_np = oracle.start_vector(77, src.dim)
    x = torch.from_numpy(x_np).cuda()
    for spin in (0, 1):
        for create in (True, False):
            d = 1 if create else -1
            nu = m.n_up + (d if spin == 0 else 0)
            nd = m.n_dn + (d if spin == 1 else 0)
            if not (0 <= nu <= m.n_sites and 0 <= nd <= m.n_sites):
                continue
            mm = m.with_params(n_up=nu, n_dn=nd)
            dst = hub.Sector(mm)
            odst = oracle.Sector(mm)
            for site in sorted({0, m.n_sites // 2, m.n_sites - 1}):
                y = src.apply_fermion(dst, site, spin, create, x).cpu().numpy()
                ref = og.fermion_operator(osrc, odst, site, spin, create) @ x_np
                assert np.array_equal(y, ref), (m.name, spin, create, site)
            dst.close()
    src.close()


def test_apply_fermion_rejects_mismatched_sectors(hub):
    import torch
    m = W.config("ring8")
    src = hub.Sector(m)
    wrong = hub.Sector(m.with_params(n_up=5, n_dn=5))
    x = torch.zeros(src.dim, dtype=torch.float64, device="cuda")
    with pytest.raises(hub.HubError):
        src.apply_fermion(wrong, 0, 0, True, x)
    right = hub.Sector(m.with_params(n_up=5))
    with pytest.raises(hub.HubError):
        src.apply_fermion(right, 8, 0, True, x)   # site out of range
    with pytest.raises(hub.HubError):
        src.apply_fermion(right, 0, 1, True, x)   # wrong spin for this pair
    for s in (src, wrong, right):
        s.close()


@pytest.mark.parametrize("which", ["graph7", "ring8_n5"])
def test_lanczos_coefficients_match_oracle(hub, which):
    """The continued-fraction coefficients against the oracle's recurrence; on a
    sector of 35 up states (product and first update separate) and of 56 (the
    product with the update fused in)."""
    import torch
    if which == "graph7":
        m = W.random_graph(7, 11, seed=601, site_U=True).with_params(n_up=3, n_dn=4)
    else:
        m = W.ring(8, U=3.0, n_up=5, n_dn=4).with_params(eps=[0.05 * i for i in range(8)])
    s = hub.Sector(m)
    assert (s.count_up % 4 == 0) == (which == "ring8_n5")
    osec = oracle.Sector(m)
    f_np = oracle.start_vector(5, s.dim) * 0.37
    a, b, n2, steps = s.lanczos_coefficients(torch.from_numpy(f_np).cuda(), 40)
    ra, rb, rn2 = og.lanczos_coefficients(lambda v: oracle.spmv(osec.csr(), v), f_np, 40)
    assert steps == 40 and len(ra) == 40
    assert abs(n2 - rn2) <= 1e-14 * rn2
    np.testing.assert_allclose(a[:25], ra[:25], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(b[1:25], rb[:24], rtol=1e-10, atol=1e-12)
    if which != "graph7":
        s.close()
        return
    # an invariant subspace ends the recurrence: a single basis vector of a
    # one-state sector breaks down after one step
    one = hub.Sector(W.ring(6, U=2.0, n_up=6, n_dn=6))
    a1, b1, n21, st1 = one.lanczos_coefficients(torch.ones(1, dtype=torch.float64, device="cuda") * 2.0, 10)
    assert st1 == 1 and n21 == 4.0 and a1[0] == 12.0
    s.close()
    one.close()


@pytest.mark.parametrize("idx", range(5))
def test_greens_function_matches_lehmann(hub, idx):
    m = _models()[idx]
    s = hub.Sector(m)
    gs = s.ground_state(dtype=hub.F64, tol=1e-13, want_vector=True)
    osec, e0, psi = oracle.ground_state(m, dense_max=5000)
    assert abs(gs.e0 - e0) <= 1e-10 * max(1.0, abs(e0))
    z = _z()
    for spin in (0, 1):
        for p in sorted({0, m.n_sites - 1}):
            g, info, coef = s.greens_function(gs.e0, gs.psi, p, spin, z, max_steps=200)
            ref = og.lehmann(m, p, spin, z, e0, psi, src=osec)
            np.testing.assert_allclose(g, ref, rtol=0, atol=1e-9 * max(1.0, np.max(np.abs(ref))))
            assert abs(info["norm2_particle"] + info["norm2_hole"] - 1.0) <= 1e-12
            N = m.n_up if spin == 0 else m.n_dn
            if N == m.n_sites:
                assert info["steps_particle"] == 0 and info["norm2_particle"] == 0.0
            if N == 0:
                assert info["steps_hole"] == 0 and info["norm2_hole"] == 0.0
    s.close()


def test_greens_function_ring14_full_size(hub):
    """M = 14 ring, U = 4, N = 7/7 (dim 11,778,624; N+1 sector 10,306,296):
    half filling on a bipartite lattice makes Re G(U/2 + i w_n) vanish; the
    ring's translation invariance makes every site equal; spin symmetry of the
    singlet makes G_up = G_dn (different gather paths); sum rule and 1/z tail."""
    m = W.config("ring14_u4")
    s = hub.Sector(m)
    gs = s.ground_state(dtype=hub.F64, tol=1e-13, want_vector=True, max_iter=600)
    wn = np.pi * (2 * np.arange(12) + 1) / 10.0
    z = 2.0 + 1j * wn
    g0, info0, _ = s.greens_function(gs.e0, gs.psi, 0, 0, z, max_steps=150)
    g5, _, _ = s.greens_function(gs.e0, gs.psi, 5, 0, z, max_steps=150)
    g0d, _, _ = s.greens_function(gs.e0, gs.psi, 0, 1, z, max_steps=150)
    scale = np.max(np.abs(g0))
    assert np.max(np.abs(g0.real)) <= 1e-8 * scale
    np.testing.assert_allclose(g5, g0, rtol=0, atol=1e-8 * scale)
    np.testing.assert_allclose(g0d, g0, rtol=0, atol=1e-8 * scale)
    assert abs(info0["norm2_particle"] - 0.5) <= 1e-10 and abs(info0["norm2_hole"] - 0.5) <= 1e-10
    big = np.array([1e7j])
    gb, _, _ = s.greens_function(gs.e0, gs.psi, 0, 0, big, max_steps=20)
    assert abs(big[0] * gb[0] - 1.0) <= 1e-5
    s.close()
