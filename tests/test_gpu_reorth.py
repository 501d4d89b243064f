"""Reorthogonalised Lanczos and its orthogonality check.

* hub_gram (G = Q^T Q on the FP64 matrix cores) against numpy's FP64 product of
  the same vectors, for sizes that leave partial 16 x 16 tiles, a ragged last
  block of rows, several tile passes, and both storage precisions.
* Full (reorth = 1) and partial (reorth = 2, Simon's omega recurrence)
  reorthogonalisation: the energy matches the oracle's as on the plain path;
  the stored basis is orthogonal to rounding (full) or semi-orthogonal
  (partial: max |Q^T Q - I| within a small multiple of sqrt(eps) of the stored
  precision), and the partial variant runs its Gram-Schmidt passes on only a
  fraction of the steps.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def hub():
    import torch
    import paper_1307_7542_amd as hub
    hub.lib()
    torch.cuda.set_device(0)
    return hub


@pytest.mark.parametrize("m", [1, 3, 16, 17, 40, 90, 200])
@pytest.mark.parametrize("n", [1000, 70001])
def test_gram_matches_numpy(hub, m, n):
    import torch
    g = torch.Generator(device="cpu").manual_seed(1000 * m + n)
    base = torch.randn(m, n, generator=g, dtype=torch.float64)
    for tdt in (torch.float64, torch.float32):
        vecs = [base[i].to(tdt).cuda().contiguous() for i in range(m)]
        G = hub.gram(vecs)
        Q = np.stack([v.double().cpu().numpy() for v in vecs])
        ref = Q @ Q.T
        nrm = np.sqrt(np.diag(ref))
        bound = 1e-13 * np.outer(nrm, nrm) * max(1.0, np.sqrt(n) / 100)
        assert G.shape == (m, m)
        assert np.all(np.abs(G - ref) <= bound), (m, n, tdt, np.max(np.abs(G - ref) / np.outer(nrm, nrm)))
        assert np.array_equal(G, G.T)


def test_gram_rejects_too_many_vectors(hub):
    import torch
    vecs = [torch.zeros(64, dtype=torch.float64, device="cuda") for _ in range(305)]
    with pytest.raises(hub.HubError) as ei:
        hub.gram(vecs)
    assert ei.value.status == 6  # UNSUPPORTED


@pytest.mark.parametrize("name", ["ring12_u3", "square3x4_n5"])
def test_full_and_partial_reorthogonalisation(hub, name):
    if name == "ring12_u3":
        m = W.ring(12, U=3.0, n_up=6, n_dn=6)
        _, e_ref, _ = oracle.ground_state(m, want_vector=False)
    else:
        with open(os.path.join(GOLD, "oracle_values.json")) as f:
            e_ref = json.load(f)["entries"]["square3x4_n5"]["e0"]
        m = W.square_periodic(3, 4, n_up=5, n_dn=5)
    s = hub.Sector(m)
    for dt, tol, rel, eps in ((hub.F64, 1e-12, 1e-10, 2.0 ** -53), (hub.F32, 1e-7, 1e-6, 2.0 ** -24)):
        plain = s.ground_state(dtype=dt, tol=tol, want_vector=False, orth_check=True)
        assert plain.info["orth_loss"] == -1.0 and plain.info["reorth_steps"] == 0
        full = s.ground_state(dtype=dt, tol=tol, reorth=True, refine=True, orth_check=True)
        part = s.ground_state(dtype=dt, tol=tol, reorth="partial", refine=True, orth_check=True)
        for g in (plain, full, part):
            assert abs(g.e0 - e_ref) <= rel * abs(e_ref), (name, dt, g.e0, e_ref)
        fi, pi = full.info, part.info
        assert fi["reorth_steps"] == fi["iters"]
        assert 0 <= pi["reorth_steps"] < pi["iters"], pi
        # full: orthogonal to the rounding of the stored precision; partial: semi-orthogonal
        assert 0.0 <= fi["orth_loss"] <= 64 * eps * np.sqrt(fi["iters"]), (dt, fi["orth_loss"])
        assert 0.0 <= pi["orth_loss"] <= 8 * np.sqrt(eps), (dt, pi["orth_loss"])
        # the eigenvectors agree
        import torch
        assert abs(float(torch.dot(full.psi, part.psi))) >= 1.0 - (1e-9 if dt == hub.F64 else 1e-5)
    s.close()
