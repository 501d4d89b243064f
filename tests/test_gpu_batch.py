"""GPU tests of the batched sector solver: one product launch over many
independent sectors and lockstep Lanczos replayed from a captured HIP graph,
checked against the oracle (stored E0 of the 64 synthetic impurity models,
two-spin CSR products, dense ground states) and against the single-sector path."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")


@pytest.fixture(scope="module")
def hub():
    import torch
    import paper_1307_7542_amd as hub
    hub.lib()
    torch.cuda.set_device(0)
    return hub


@pytest.fixture(scope="module")
def aim64(hub):
    models = W.aim_batch(64)
    secs = [hub.Sector(m) for m in models]
    batch = hub.Batch(secs)
    yield models, secs, batch
    batch.close()
    for s in secs:
        s.close()


def _stored():
    with open(GOLDEN) as f:
        return json.load(f)["entries"]


def _mixed_models():
    """Sectors of different lattices, sizes and parameter kinds in one batch,
    including a one-state sector and a dimer."""
    return [
        W.config("ring8"),
        W.ring(6).with_params(n_up=0, n_dn=0),          # dimension 1
        W.dimer(t=1.0, U=3.0),
        W.aim_batch(4)[2],
        W.random_graph(7, 11, seed=601, site_U=True).with_params(n_up=3, n_dn=2),
        W.square_periodic(3, 3, n_up=4, n_dn=4),
        W.ring(10).with_params(n_up=3, n_dn=6),
    ]


def test_batch_offsets(hub, aim64):
    models, secs, batch = aim64
    off = batch.offsets
    assert off[0] == 0 and len(off) == 65
    assert list(np.diff(off)) == [s.dim for s in secs]
    st = _stored()
    assert [st[f"aim{p}"]["dim"] for p in range(64)] == [s.dim for s in secs]


@pytest.mark.parametrize("which", ["mixed", "aim12"])
def test_batch_product_matches_oracle_and_single(hub, which):
    """y = H x for every sector of the batch in one launch, FP64 and FP32,
    against the oracle's two-spin CSR product, and bit for bit against the
    single-sector product (both form each element in the same order)."""
    import torch
    models = _mixed_models() if which == "mixed" else W.aim_batch(12)
    secs = [hub.Sector(m) for m in models]
    batch = hub.Batch(secs)
    off = batch.offsets
    xs = [oracle.start_vector(100 + p, s.dim) for p, s in enumerate(secs)]
    x64 = torch.from_numpy(np.concatenate(xs)).cuda()
    for dt, tol in ((hub.F64, 1e-13), (hub.F32, 3e-6)):
        x = x64 if dt == hub.F64 else x64.float()
        y = batch.matvec(x).double().cpu().numpy()
        for p, (m, s) in enumerate(zip(models, secs)):
            osec = oracle.Sector(m)
            ref = oracle.spmv(osec.csr(), xs[p])
            yp = y[off[p]:off[p + 1]]
            scale = np.max(np.abs(ref)) + 1.0
            assert np.max(np.abs(yp - ref)) <= tol * scale, (p, m.name)
            single = s.matvec(x[off[p]:off[p + 1]].contiguous()).double().cpu().numpy()
            assert np.array_equal(yp, single), (p, m.name, np.max(np.abs(yp - single)))
    batch.close()
    for s in secs:
        s.close()


def test_batch_ground_state_fp64_64_impurity_models(hub, aim64):
    models, secs, batch = aim64
    e0, iters, psi, info = batch.ground_state(dtype=hub.F64, tol=1e-12, max_iter=400)
    st = _stored()
    ref = np.array([st[f"aim{p}"]["e0"] for p in range(64)])
    np.testing.assert_allclose(e0, ref, rtol=1e-10, atol=0)
    assert info["graph_replays"] > 0
    assert info["rows_per_lane"] in (1, 2, 4) and info["block_size"] in (256, 512)
    assert info["cols_per_lane"] in (1, 2, 4)
    assert np.all(iters >= 1) and np.all(iters <= info["steps"])
    # small sectors stop at (or before) their dimension
    dims = np.diff(batch.offsets)
    assert np.all(iters <= dims)


def test_batch_graph_replay_equals_eager(hub, aim64):
    """The captured step reads its vector roles and slots from the device step
    counter (advanced by the last block of the step's last kernel); replays must
    reproduce the eager steps bit for bit."""
    models, secs, batch = aim64
    e_g, it_g, _, info_g = batch.ground_state(dtype=hub.F64, tol=1e-12, max_iter=400)
    e_e, it_e, _, info_e = batch.ground_state(dtype=hub.F64, tol=1e-12, max_iter=400, graph=False)
    assert info_g["graph_replays"] > 0 and info_e["graph_replays"] == 0
    assert np.array_equal(it_g, it_e)
    assert np.array_equal(e_g, e_e)
    # and a second graph run is also identical (fresh capture, replays after the first)
    e_2, it_2, _, _ = batch.ground_state(dtype=hub.F64, tol=1e-12, max_iter=400)
    assert np.array_equal(e_g, e_2) and np.array_equal(it_g, it_2)


def test_batch_mixed_precision_with_refinement(hub, aim64):
    models, secs, batch = aim64
    st = _stored()
    ref = np.array([st[f"aim{p}"]["e0"] for p in range(64)])
    e_r, _, _, _ = batch.ground_state(dtype=hub.F32, tol=1e-7, max_iter=400)
    assert np.max(np.abs(e_r - ref) / np.abs(ref)) <= 2e-6
    e_f, _, psi, _ = batch.ground_state(dtype=hub.F32, tol=1e-7, max_iter=400, refine=True)
    # Rayleigh quotient of an FP32-built vector: error quadratic in the residual
    assert np.max(np.abs(e_f - ref) / np.abs(ref)) <= 1e-9
    assert np.all(e_f >= ref - 1e-12 * np.abs(ref))  # variational bound


def test_batch_vectors_and_gradients(hub):
    """psi of each sector (normalised, canonical sign) against the oracle's dense
    ground state; Hellmann-Feynman gradients from the sector slices."""
    import torch
    models = W.aim_batch(10)
    keep = [m for m in models if m.n_sites <= 9]
    secs = [hub.Sector(m) for m in keep]
    batch = hub.Batch(secs)
    e0, iters, psi, info = batch.ground_state(dtype=hub.F64, tol=1e-13, want_vector=True, max_iter=600)
    off = batch.offsets
    for p, (m, s) in enumerate(zip(keep, secs)):
        osec, e_ref, v_ref = oracle.ground_state(m, dense_max=5000)
        v_ref = oracle.canonical_sign(v_ref)
        assert abs(e0[p] - e_ref) <= 1e-10 * abs(e_ref)
        vp = psi[off[p]:off[p + 1]].contiguous()
        v = vp.cpu().numpy()
        assert abs(np.linalg.norm(v) - 1.0) <= 1e-12
        assert np.max(np.abs(v - v_ref)) <= 1e-7, (p, m.name)
        db, dU, de = s.param_bilinear(vp, vp)
        rb, rU, re = osec.param_bilinear(v_ref, v_ref)
        np.testing.assert_allclose(db, rb, atol=1e-8, rtol=0)
        np.testing.assert_allclose(dU, rU, atol=1e-8, rtol=0)
        np.testing.assert_allclose(de, re, atol=1e-8, rtol=0)
    batch.close()
    for s in secs:
        s.close()
    torch.cuda.synchronize()


def test_batch_mixed_sectors_and_edges(hub):
    """A dimension-1 sector breaks down at once; sectors of different lattices
    and parameter kinds converge to the oracle's dense energies; max_iter=1
    reports non-convergence with one step done."""
    models = _mixed_models()
    secs = [hub.Sector(m) for m in models]
    batch = hub.Batch(secs)
    e0, iters, _, info = batch.ground_state(dtype=hub.F64, tol=1e-12, max_iter=400)
    for p, m in enumerate(models):
        _, e_ref, _ = oracle.ground_state(m, dense_max=5000)
        assert abs(e0[p] - e_ref) <= 1e-10 * max(1.0, abs(e_ref)), (p, m.name)
    assert iters[1] == 1
    with pytest.raises(hub.HubError):
        batch.ground_state(dtype=hub.F64, max_iter=1)
    e1, it1, _, info1 = batch.ground_state(dtype=hub.F64, max_iter=1, allow_not_converged=True)
    assert np.all(it1 == 1) and info1["steps"] == 1 and info1["graph_replays"] == 0
    # alpha_0 = <v0, H v0> bounds E0 from above
    assert np.all(e1 >= e0 - 1e-12 * np.abs(e0))
    batch.close()
    for s in secs:
        s.close()


def test_batch_rejects_bad_options(hub):
    m = W.config("ring8")
    s = hub.Sector(m)
    batch = hub.Batch([s, s])
    import ctypes
    o = hub.LanczosOpts(50, 0.0, 1, None, hub.F64, 1, 0, 0, 5, 0)  # reorth requested
    st = hub.lib().hub_batch_ground_state(batch._h, ctypes.byref(o), None, None, None, None, None)
    assert st == 6  # unsupported
    o = hub.LanczosOpts(50, 0.0, 1, None, hub.F64, 0, 0, 1, 5, 0)  # refine without psi
    st = hub.lib().hub_batch_ground_state(batch._h, ctypes.byref(o), None, None, None, None, None)
    assert st == 1
    e0, _, _, _ = batch.ground_state(dtype=hub.F64)
    assert e0[0] == e0[1]
    batch.close()
    s.close()


def test_batch_mixed_gradients_vs_oracle(hub):
    """Hellmann-Feynman gradients (dE0/dt per bond, dE0/dU_i, dE0/deps_i) of the
    impurity models from the FP32-mixed batch solve with FP64 refinement of psi,
    against the oracle's values from its own FP64 ground states (dense, or
    Lanczos on the two-spin CSR for the 9-site models).  The gradient of an
    approximate eigenvector is off by about 2 |dpsi| |dH/dtheta| whatever the
    component's size, so each group (bonds, U, eps) is held to 1e-5 of its
    largest component: relative to the group's scale, no absolute floor."""
    models = [m for m in W.aim_batch(64) if m.n_sites <= 9]
    secs = [hub.Sector(m) for m in models]
    batch = hub.Batch(secs)
    e0, _, psi, _ = batch.ground_state(dtype=hub.F32, tol=1e-7, max_iter=400, refine=True)
    off = batch.offsets
    worst = 0.0
    for p, (m, s) in enumerate(zip(models, secs)):
        osec, e_ref, v_ref = oracle.ground_state(m, dense_max=5000)
        assert abs(e0[p] - e_ref) <= 1e-9 * abs(e_ref), (p, m.name)
        vp = psi[off[p]:off[p + 1]].contiguous()
        for got, ref in zip(s.param_bilinear(vp, vp), osec.param_bilinear(v_ref, v_ref)):
            rel = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
            worst = max(worst, rel)
            assert rel <= 1e-5, (p, m.name, rel)
    print("largest group-relative gradient error", worst)
    batch.close()
    for s in secs:
        s.close()
