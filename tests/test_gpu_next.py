"""GPU tests of the widened rows: differentiable E0 through the adjoint kernel
(Hellmann-Feynman), and full-size product parity on the 2x9 ladder."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hub():
    import torch
    import paper_1307_7542_amd as hub
    hub.lib()
    torch.cuda.set_device(0)
    return hub


def _energy(m):
    import paper_1307_7542_amd as hub
    s = hub.Sector(m)
    e = s.ground_state(dtype=hub.F64, want_vector=False, tol=1e-13).e0
    s.close()
    return e


@pytest.mark.parametrize("which", ["square3x3", "rand7", "aim"])
def test_autograd_matches_finite_differences_and_oracle(hub, which):
    import torch
    from paper_1307_7542_amd.autograd import ground_energy
    if which == "square3x3":
        m = W.square_periodic(3, 3, n_up=4, n_dn=4)
    elif which == "rand7":
        m = W.random_graph(7, 11, seed=601, site_U=True).with_params(n_up=3, n_dn=4)
    else:
        m = W.aim_batch(5)[4]
    t = torch.tensor(m.t, dtype=torch.float64, requires_grad=True)
    U = torch.tensor(m.U, dtype=torch.float64, requires_grad=True)
    eps = torch.tensor(m.eps, dtype=torch.float64, requires_grad=True)
    E = ground_energy(t, U, eps, n_sites=m.n_sites, bonds=m.bonds, n_up=m.n_up, n_dn=m.n_dn)
    E.backward()
    # oracle Hellmann-Feynman values (dense ground state)
    osec, e_ref, psi = oracle.ground_state(m, dense_max=5000)
    db, dU, de = osec.param_bilinear(psi, psi)
    assert abs(E.item() - e_ref) <= 1e-10 * abs(e_ref)
    np.testing.assert_allclose(t.grad.numpy(), db, rtol=0, atol=1e-8)
    np.testing.assert_allclose(U.grad.numpy(), dU, rtol=0, atol=1e-8)
    np.testing.assert_allclose(eps.grad.numpy(), de, rtol=0, atol=1e-8)
    # central finite differences on the GPU solver, a few parameters
    h = 1e-4
    for b in range(min(3, len(m.t))):
        tp = list(m.t); tp[b] += h
        tm = list(m.t); tm[b] -= h
        fd = (_energy(m.with_params(t=tp)) - _energy(m.with_params(t=tm))) / (2 * h)
        assert abs(fd - t.grad[b].item()) <= 1e-5 * max(1.0, abs(fd))
    i = 0
    up = list(m.U); up[i] += h
    um = list(m.U); um[i] -= h
    fd = (_energy(m.with_params(U=up)) - _energy(m.with_params(U=um))) / (2 * h)
    assert abs(fd - U.grad[i].item()) <= 1e-5 * max(1.0, abs(fd))
    # Euler identity: H is linear in all parameters
    euler = (t.detach() * t.grad).sum() + (U.detach() * U.grad).sum() + (eps.detach() * eps.grad).sum()
    assert abs(euler.item() - E.item()) <= 1e-9 * abs(E.item())


def test_aim_hybridisation_gradient_sign(hub):
    """t_0k = -V_k, so dE0/dV_k = -dE0/dt_0k; E0 is even in each V_k."""
    import torch
    from paper_1307_7542_amd.autograd import ground_energy
    m = W.aim_batch(3)[1]
    V = -np.array(m.t)
    t = torch.tensor(m.t, dtype=torch.float64, requires_grad=True)
    U = torch.tensor(m.U, dtype=torch.float64)
    eps = torch.tensor(m.eps, dtype=torch.float64)
    E = ground_energy(t, U, eps, n_sites=m.n_sites, bonds=m.bonds, n_up=m.n_up, n_dn=m.n_dn)
    E.backward()
    dV = -t.grad.numpy()
    flipped = list(m.t)
    flipped[0] = -flipped[0]
    assert abs(_energy(m.with_params(t=flipped)) - E.item()) <= 1e-10 * abs(E.item())
    h = 1e-4
    tp = list(m.t); tp[0] = -(V[0] + h)
    tm = list(m.t); tm[0] = -(V[0] - h)
    fd = (_energy(m.with_params(t=tp)) - _energy(m.with_params(t=tm))) / (2 * h)
    assert abs(fd - dV[0]) <= 1e-5 * max(1.0, abs(fd))


def test_square4x4_gradients_full_size(hub):
    """4x4 torus N=7/7 (dim 1.3e8): dE0/dt for all 32 bonds and dE0/dU from the
    adjoint kernel, checked by the Euler identity and finite differences on one
    bond and on U."""
    import torch
    from paper_1307_7542_amd.autograd import ground_energy
    m = W.config("square4x4")
    t = torch.tensor(m.t, dtype=torch.float64, requires_grad=True)
    U = torch.tensor(m.U, dtype=torch.float64, requires_grad=True)
    eps = torch.tensor(m.eps, dtype=torch.float64, requires_grad=True)
    kw = dict(max_iter=2000, tol=1e-11, check_every=10)
    E = ground_energy(t, U, eps, n_sites=m.n_sites, bonds=m.bonds, n_up=m.n_up, n_dn=m.n_dn, **kw)
    E.backward()
    euler = (t.detach() * t.grad).sum() + (U.detach() * U.grad).sum()
    assert abs(euler.item() - E.item()) <= 1e-8 * abs(E.item())
    assert float(U.grad.sum()) > 0  # repulsion raises the energy

    def energy(mm):
        import paper_1307_7542_amd as h
        s = h.Sector(mm)
        e = s.ground_state(dtype=h.F64, want_vector=False, **kw).e0
        s.close()
        return e
    h = 1e-3
    tp = list(m.t); tp[5] += h
    tm = list(m.t); tm[5] -= h
    fd = (energy(m.with_params(t=tp)) - energy(m.with_params(t=tm))) / (2 * h)
    assert abs(fd - t.grad[5].item()) <= 1e-5 * max(1.0, abs(fd))
    dUs = float(U.grad.sum())
    fdU = (energy(m.with_params(U=[4.0 + h] * 16)) - energy(m.with_params(U=[4.0 - h] * 16))) / (2 * h)
    assert abs(fdU - dUs) <= 1e-5 * max(1.0, abs(fdU))


def test_ladder2x9_sampled_product(hub):
    """2x9 ladder N=9/9 (dim 2.36e9; one FP32 column is 194 KB, beyond the LDS):
    sampled rows of one FP32 and one FP64 product against the oracle's
    matrix-free two-spin rows on the same SplitMix64 vector."""
    import torch
    m = W.config("ladder2x9")
    s = hub.Sector(m)
    assert s.dim == math.comb(18, 9) ** 2
    osec = oracle.Sector(m, explicit_keys=False)
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([[0, s.dim - 1], rng.integers(0, s.dim, size=1500)]))
    yr = osec.apply_rows(rows, None, seed=99)
    idx = torch.from_numpy(rows).cuda()
    for dt, tol in ((hub.F32, 2e-5), (hub.F64, 1e-12)):
        x = s.start_vector(seed=99, dtype=dt, normalize=False)
        y = s.matvec(x)
        yg = y[idx].double().cpu().numpy()
        assert np.max(np.abs(yg - yr)) <= tol * (np.max(np.abs(yr)) + 1)
        del x, y
        torch.cuda.empty_cache()
    s.close()
