"""The allocation-free entry point hub_start_vector_noalloc (static device
scratch for the norm's partial sums) against hub_start_vector, bit for bit,
through the C ABI: two calls in a row on the same device, the second on a
smaller sector, in both precisions, plus a translation (k = 0) sector whose
start vector is projected before it is normalised."""
import ctypes

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


def _noalloc(hub, sec, dtype, seed, normalize, out):
    import torch
    st = torch.cuda.current_stream()
    rc = hub.lib().hub_start_vector_noalloc(sec._h, dtype, ctypes.c_uint64(seed), int(normalize),
                                            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream))
    assert rc == 0, hub.lib().hub_last_error().decode()
    return out


def test_noalloc_start_vector_matches_allocating_one(hub):
    import torch
    big = hub.Sector(W.config("square4x4").with_params(n_up=5, n_dn=5))   # 4368 x 4368
    small = hub.Sector(W.ring(10, U=2.0, n_up=4, n_dn=3))                  # 210 x 120
    assert small.dim < big.dim
    for dt in (hub.F64, hub.F32):
        for sec, seed in ((big, 7542), (small, 11)):
            for normalize in (True, False):
                ref = sec.start_vector(seed=seed, dtype=dt, normalize=normalize)
                got = _noalloc(hub, sec, dt, seed, normalize, sec.empty(dt))
                torch.cuda.synchronize()
                assert torch.equal(got, ref), (dt, sec.dim, normalize)
                if normalize:
                    assert abs(float(torch.linalg.vector_norm(got.double())) - 1.0) < 1e-6
    big.close()
    small.close()


def test_noalloc_start_vector_k0_sector(hub):
    import torch
    m = W.ring(12, U=3.0, n_up=6, n_dn=6)
    sec = hub.Sector(m, translation=1)
    for dt in (hub.F64, hub.F32):
        ref = sec.start_vector(seed=5, dtype=dt)
        got = sec.start_vector(seed=5, dtype=dt, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), dt
    sec.close()
