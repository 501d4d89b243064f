"""GPU tests of the translation-symmetric (k = 0) sector path (Sec. VI): layout,
product and ground energies against the oracle's k = 0 block, and Table IV's
M = 14 energy from the k = 0 sector (dim 844,272 instead of 11,778,624)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import oracle.translation as ot
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hub():
    import torch
    import paper_1307_7542_amd as hub
    hub.lib()
    torch.cuda.set_device(0)
    return hub


def _models():
    return [
        (W.ring(6, U=4.0, n_up=3, n_dn=3), 1),
        (W.ring(6, U=4.0, n_up=2, n_dn=3), 1),
        (W.ring(6, U=2.5, n_up=2, n_dn=2), 1),
        (W.ring(8, U=2.0, n_up=4, n_dn=2), 1),
        (W.ring(4, U=3.0, n_up=2, n_dn=1), 1),
        (W.ring(8, U=2.0, n_up=4, n_dn=4), 2),
        (W.ladder(3, rung_lo=0.7, rung_hi=0.7).with_params(n_up=3, n_dn=2), 2),
        (W.ring(10, U=4.0, n_up=5, n_dn=4).with_params(eps=[0.3] * 10), 1),
        (W.ring(12, U=3.0, n_up=6, n_dn=6), 1),
        (W.ring(8, U=5.0, n_up=8, n_dn=3), 1),
    ]


@pytest.mark.parametrize("idx", range(10))
def test_k0_layout_and_product(hub, idx):
    import torch
    m, w = _models()[idx]
    s = hub.Sector(m, translation=w)
    osec = oracle.Sector(m)
    reps, per = ot.rep_layout(osec, w)
    greps, gper = s.k0_layout()
    assert np.array_equal(greps.astype(np.int64), reps) and np.array_equal(gper.astype(np.int64), per)
    assert s.dim == len(reps) * s.count_dn
    rp, col, val = osec.csr()
    H = sp.csr_matrix((val, col, rp), shape=(osec.dim, osec.dim))
    x0 = ot.k0_project(osec, oracle.start_vector(3, osec.dim), w)
    phi = ot.restrict(osec, x0, reps, per)
    ref = ot.restrict(osec, H @ x0, reps, per)
    scale = np.max(np.abs(ref)) + 1.0
    for dt, tol in ((hub.F64, 1e-13), (hub.F32, 2e-6)):
        x = torch.from_numpy(phi).cuda()
        if dt == hub.F32:
            x = x.float()
        y = s.matvec(x).double().cpu().numpy()
        assert np.max(np.abs(y - ref)) <= tol * scale, (m.name, dt)
    s.close()


@pytest.mark.parametrize("idx", range(10))
def test_k0_ground_energy(hub, idx):
    m, w = _models()[idx]
    s = hub.Sector(m, translation=w)
    _, _, Hk, _ = ot.k0_hamiltonian(m, w)
    e_ref = float(np.linalg.eigvalsh(Hk.toarray())[0]) if Hk.shape[0] <= 3000 else None
    g64 = s.ground_state(dtype=hub.F64, tol=1e-13, want_vector=True, max_iter=800)
    if e_ref is None:
        vals = sp.linalg.eigsh(Hk, k=1, which="SA", tol=1e-14)[0]
        e_ref = float(vals[0])
    assert abs(g64.e0 - e_ref) <= 1e-10 * max(1.0, abs(e_ref)), (m.name, g64.e0, e_ref)
    import torch
    assert abs(float(torch.linalg.norm(g64.psi)) - 1.0) <= 1e-12
    g32 = s.ground_state(dtype=hub.F32, reorth=True, refine=True, tol=1e-7, max_iter=800)
    assert abs(g32.e0 - e_ref) <= 1e-9 * max(1.0, abs(e_ref))
    s.close()


def test_k0_table4_ring14(hub):
    """Sec. V, Table IV, M = 14, U = 4: the ground state has k = 0 (odd N per
    spin), so the k = 0 sector of 246 x 3432 states reproduces E_min."""
    m = W.config("ring14_u4")
    s = hub.Sector(m, translation=1)
    reps, per = s.k0_layout()
    assert len(reps) == 246 and s.dim == 246 * 3432
    assert sorted(set(per.tolist())) == [2, 14]
    g = s.ground_state(dtype=hub.F64, tol=1e-12, max_iter=600, want_vector=False)
    with open(os.path.join(os.path.dirname(__file__), "golden", "table4_emin.json")) as f:
        t4 = json.load(f)
    printed = [r for r in t4["rows"] if r["M"] == 14][0]["E_min"]
    assert abs(g.e0 - printed) <= 1e-9
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")) as f:
        full = json.load(f)["entries"]["ring14_u4"]["e0"]
    assert abs(g.e0 - full) <= 1e-10 * abs(full)
    s.close()


def test_k0_ring16_even_filling(hub):
    """M = 16, U = 4, N = 8/8: the lowest energy of the k = 0 block is bounded
    below by the full sector's E0 (the oracle's matrix-free Lanczos value)."""
    m = W.ring(16, U=4.0, n_up=8, n_dn=8)
    s = hub.Sector(m, translation=1)
    g = s.ground_state(dtype=hub.F64, tol=1e-12, max_iter=800, want_vector=False)
    with open(os.path.join(os.path.dirname(__file__), "golden", "ring16_u4_oracle.json")) as f:
        e_full = json.load(f)["e0"]
    print("ring16 k=0 E0", g.e0, "full sector (oracle)", e_full)
    assert g.e0 >= e_full - 1e-10 * abs(e_full)
    s.close()


def test_k0_rejects_non_invariant_models(hub):
    m = W.ring(6, U=4.0, n_up=3, n_dn=3)
    t = list(m.t)
    t[2] = 1.1
    with pytest.raises(hub.HubError):
        hub.Sector(m.with_params(t=t), translation=1)
    with pytest.raises(hub.HubError):
        hub.Sector(m.with_params(eps=[0.0] * 5 + [0.2]), translation=1)
    with pytest.raises(hub.HubError):
        hub.Sector(m, translation=4)   # does not divide M
    s = hub.Sector(m, translation=1)
    with pytest.raises(hub.HubError):
        s.diagonal()
    plain = hub.Sector(m)
    with pytest.raises(hub.HubError):
        plain.k0_layout()
    s.close()
    plain.close()
