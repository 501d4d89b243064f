"""Full-size ground states of the two largest workloads -- the 4x4 torus N=7/7
(dim 130,873,600) and the 2x9 ladder N=9/9 (dim 2,363,904,400) -- against what
the mathematics fixes at the same size, and mixed-precision gradients.

* U = 0: H is the Kronecker sum of two free one-spin sectors (Sec. IV A with
  D = 0), so E0 is the sum of the lowest N_up and the lowest N_dn eigenvalues
  of the one-body matrix h (h_ij = -t_ij on every bond).
* t = 0: H = D (Eq. count1 without hopping); with uniform U the fewest doubly
  occupied sites is max(0, N_up + N_dn - M), so E0 = U max(0, N_up + N_dn - M).
* Mixed-precision gradients: dE0/dt for every bond and dE0/dU from the FP32
  solve with FP64 refinement, against the FP64 solve's values and central
  finite differences.

FP64 plain Lanczos (the paper's recurrence) must agree to 1e-10 relative;
FP32 vectors with FP64 scalars and the FP64 refinement to 1e-6 relative.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hub():
    import torch
    import paper_1307_7542_amd as hub
    hub.lib()
    torch.cuda.set_device(0)
    return hub


def _free_energy(m):
    h = np.zeros((m.n_sites, m.n_sites))
    for (i, j), t in zip(m.bonds, m.t):
        h[i, j] -= t
        h[j, i] -= t
    w = np.linalg.eigvalsh(h)
    return float(w[:m.n_up].sum() + w[:m.n_dn].sum())


def _solve_both(hub, m, max_iter):
    """(FP64 plain E0, FP32-mixed refined E0) of the model's sector."""
    import torch
    s = hub.Sector(m)
    g64 = s.ground_state(dtype=hub.F64, want_vector=False, tol=1e-12, max_iter=max_iter, check_every=4)
    torch.cuda.empty_cache()
    g32 = s.ground_state(dtype=hub.F32, refine=True, tol=1e-7, max_iter=max_iter, check_every=4)
    out = (g64.e0, g32.e0, g64.info, g32.info, s.dim)
    del g32
    s.close()
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("name", ["square4x4", "ladder2x9"])
def test_u0_closed_form_full_size(hub, name):
    """U = 0 on the full 4x4 torus (random t) and 2x9 ladder (random rungs)."""
    m = W.config(name)
    m = m.with_params(U=[0.0] * m.n_sites)
    e_cf = _free_energy(m)
    e64, e32, i64, i32, dim = _solve_both(hub, m, max_iter=1500)
    assert dim == (130_873_600 if name == "square4x4" else 2_363_904_400)
    assert abs(e64 - e_cf) <= 1e-10 * abs(e_cf), (name, e64, e_cf, i64["iters"])
    assert abs(e32 - e_cf) <= 1e-6 * abs(e_cf), (name, e32, e_cf, i32["iters"])


@pytest.mark.parametrize("name,n,expect", [("square4x4", 7, 0.0), ("square4x4", 9, 8.0), ("ladder2x9", 9, 0.0)])
def test_t0_closed_form_full_size(hub, name, n, expect):
    """t = 0: H = D; N = 9/9 on the 16-site torus forces two doubly occupied
    sites (E0 = 2 U = 8) with the same 11440 x 11440 dimension as N = 7/7."""
    m = W.config(name)
    U = m.U[0]
    m = m.with_params(t=[0.0] * len(m.t), n_up=n, n_dn=n)
    assert expect == U * max(0, 2 * n - m.n_sites)
    e64, e32, i64, i32, _ = _solve_both(hub, m, max_iter=100)
    assert i64["breakdown"] == 1 and i32["breakdown"] == 1
    assert abs(e64 - expect) <= 1e-12 * max(1.0, abs(expect)), (name, n, e64)
    assert abs(e32 - expect) <= 1e-6 * max(1.0, abs(expect)), (name, n, e32)


def test_square4x4_mixed_energy_against_fp64(hub):
    """U = 4 (the workload itself): the mixed solve's refined energy is within
    1e-6 relative of the FP64 plain solve, and so is its FP32 Ritz value."""
    m = W.config("square4x4")
    e64, e32, i64, i32, _ = _solve_both(hub, m, max_iter=2000)
    assert abs(e32 - e64) <= 1e-6 * abs(e64), (e32, e64)
    assert abs(i32["e0_ritz"] - e64) <= 1e-6 * abs(e64), (i32["e0_ritz"], e64)


def test_square4x4_mixed_gradients(hub):
    """dE0/dt for all 32 bonds and dE0/dU_i from the FP32-mixed, refined psi
    against the FP64 psi's (1e-5 relative, each component), and central
    differences of FP64 energies for four bonds and the uniform U (1e-5
    relative).  The Hellmann-Feynman value of an approximate eigenvector is
    off by a term linear in its error, so this bounds the mixed psi as well."""
    import torch
    from paper_1307_7542_amd.autograd import ground_energy
    m = W.config("square4x4")

    def grads(**kw):
        t = torch.tensor(m.t, dtype=torch.float64, requires_grad=True)
        U = torch.tensor(m.U, dtype=torch.float64, requires_grad=True)
        eps = torch.tensor(m.eps, dtype=torch.float64, requires_grad=True)
        E = ground_energy(t, U, eps, n_sites=m.n_sites, bonds=m.bonds, n_up=m.n_up, n_dn=m.n_dn,
                          max_iter=2000, check_every=4, **kw)
        E.backward()
        torch.cuda.empty_cache()
        return E.item(), t.grad.numpy().copy(), U.grad.numpy().copy()

    e64, dt64, dU64 = grads(dtype=hub.F64, tol=1e-12)
    e32, dt32, dU32 = grads(dtype=hub.F32, tol=1e-7, refine=True)
    assert abs(e32 - e64) <= 1e-6 * abs(e64)
    assert np.all(np.abs(dt32 - dt64) <= 1e-5 * np.abs(dt64)), np.max(np.abs(dt32 - dt64) / np.abs(dt64))
    assert np.all(np.abs(dU32 - dU64) <= 1e-5 * np.abs(dU64)), np.max(np.abs(dU32 - dU64) / np.abs(dU64))

    def energy(mm):
        s = hub.Sector(mm)
        e = s.ground_state(dtype=hub.F64, want_vector=False, tol=1e-12, max_iter=2000, check_every=4).e0
        s.close()
        return e
    h = 1e-3
    for b in (0, 9, 18, 31):
        tp = list(m.t); tp[b] += h
        tm = list(m.t); tm[b] -= h
        fd = (energy(m.with_params(t=tp)) - energy(m.with_params(t=tm))) / (2 * h)
        assert abs(fd - dt32[b]) <= 1e-5 * abs(fd), (b, fd, dt32[b])
    fdU = (energy(m.with_params(U=[4.0 + h] * 16)) - energy(m.with_params(U=[4.0 - h] * 16))) / (2 * h)
    assert abs(fdU - dU32.sum()) <= 1e-5 * abs(fdU), (fdU, dU32.sum())


def test_workspace_beyond_device_memory_is_refused(hub):
    """Full reorthogonalisation with max_iter = 400 on the 2x9 ladder would store
    up to 401 FP32 vectors of 9.46 GB: hub_ground_state returns HUB_ERR_OOM
    before allocating anything (free device memory unchanged), and the sector
    still serves products and small solves afterwards."""
    import torch
    m = W.config("ladder2x9")
    s = hub.Sector(m)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for dt in (hub.F32, hub.F64):
        with pytest.raises(hub.HubError) as ei:
            s.ground_state(dtype=dt, reorth=True, max_iter=400, want_vector=False)
        assert ei.value.status == 3, ei.value  # HUB_ERR_OOM
        assert "exceeds" in str(ei.value)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert abs(free1 - free0) < (64 << 20), (free0, free1)
    g = s.ground_state(dtype=hub.F32, max_iter=3, want_vector=False, allow_not_converged=True)
    assert g.info["iters"] == 3
    s.close()
