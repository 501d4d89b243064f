"""CPU checks of the C ABI boundary: the library loads, exports every function
declared in include/hubbard.h, and rejects bad arguments with status codes
before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hubbard.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hub_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_1307_7542_amd as hub
    return hub.lib()


def test_header_declares_expected_api():
    names = declared_functions()
    for n in ["hub_sector_create", "hub_matvec", "hub_ground_state", "hub_basis", "hub_hopping_csr",
              "hub_rank", "hub_param_bilinear"]:
        assert n in names


def test_library_exports_every_declared_function(L):
    import paper_1307_7542_amd as hub
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(hub.EXPORTED) == declared_functions()


_C_TYPES = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "uint64_t": ctypes.c_uint64,
            "uint32_t": ctypes.c_uint32, "double": ctypes.c_double, "float": ctypes.c_float}


def header_structs():
    """{struct name: [(field, C type), ...]} of the typedef'd structs of the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for name, body in re.findall(r"typedef struct (hub_[a-z0-9_]+) \{(.*?)\} \1;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = " ".join(decl.split())
            if not decl:
                continue
            m = re.match(r"(const )?([A-Za-z0-9_]+)\s+(.*)$", decl)
            assert m, decl
            for d in m.group(3).split(","):
                d = d.strip()
                fields.append((d.lstrip("* "), "ptr" if d.startswith("*") else m.group(2)))
        out[name] = fields
    return out


def test_binding_structs_match_header():
    """Every ctypes structure of the binding has the fields of its C struct, in
    order and of the same types (pointers as pointers)."""
    import paper_1307_7542_amd as hub
    pairs = {"hub_model": hub._Model, "hub_schedule": hub.Schedule, "hub_lanczos_opts": hub.LanczosOpts,
             "hub_lanczos_info": hub.LanczosInfo, "hub_batch_info": hub.BatchInfo, "hub_gf_info": hub.GfInfo}
    hs = header_structs()
    assert set(pairs) == set(hs)
    for cname, py in pairs.items():
        want = hs[cname]
        got = py._fields_
        assert [f for f, _ in want] == [f for f, _ in got], cname
        for (f, ct), (_, pt) in zip(want, got):
            if ct == "ptr":
                assert pt in (ctypes.c_void_p,) or issubclass(pt, ctypes._Pointer), (cname, f, pt)
            else:
                assert pt is _C_TYPES[ct], (cname, f, ct, pt)


def test_status_strings(L):
    assert L.hub_status_str(0) == b"HUB_OK"
    assert L.hub_status_str(2) == b"HUB_ERR_RANGE"
    assert L.hub_status_str(99) == b"HUB_ERR_UNKNOWN"
    assert b"gfx950" in L.hub_version()


def _model(M, bonds, t, U=None):
    import paper_1307_7542_amd as hub
    bi = (ctypes.c_int32 * max(1, len(bonds)))(*[b[0] for b in bonds])
    bj = (ctypes.c_int32 * max(1, len(bonds)))(*[b[1] for b in bonds])
    tt = (ctypes.c_double * max(1, len(t)))(*t)
    UU = (ctypes.c_double * max(1, M))(*(U if U is not None else [0.0] * max(1, M)))
    m = hub._Model(M, len(bonds), ctypes.cast(bi, ctypes.c_void_p), ctypes.cast(bj, ctypes.c_void_p),
                   ctypes.cast(tt, ctypes.c_void_p), ctypes.cast(UU, ctypes.c_void_p), None)
    return m, (bi, bj, tt, UU)


@pytest.mark.parametrize("M,n_up,n_dn,bonds,t,code", [
    (0, 0, 0, [], [], 2),            # M out of range
    (33, 1, 1, [], [], 2),
    (4, 5, 1, [(0, 1)], [1.0], 2),   # N > M
    (4, -1, 1, [(0, 1)], [1.0], 2),
    (4, 2, 2, [(0, 4)], [1.0], 1),   # bond endpoint out of range
    (4, 2, 2, [(2, 2)], [1.0], 1),   # i == j
    (4, 2, 2, [(0, 1)], [float("nan")], 1),
    (4, 2, 2, [(0, 1)], [float("inf")], 1),
])
def test_create_rejects_bad_input(L, M, n_up, n_dn, bonds, t, code):
    m, keep = _model(M, bonds, t)
    h = ctypes.c_void_p()
    st = L.hub_sector_create(ctypes.byref(m), n_up, n_dn, ctypes.byref(h))
    assert st == code
    assert h.value is None
    assert len(L.hub_last_error()) > 0


def test_null_arguments(L):
    h = ctypes.c_void_p()
    assert L.hub_sector_create(None, 1, 1, ctypes.byref(h)) == 1
    m, keep = _model(4, [(0, 1)], [1.0])
    assert L.hub_sector_create(ctypes.byref(m), 1, 1, None) == 1
    assert L.hub_matvec(None, 0, None, None, None) == 1
    assert L.hub_sector_dims(None, None, None, None) == 1
    L.hub_sector_destroy(None)


def test_nonfinite_U_rejected(L):
    m, keep = _model(3, [(0, 1)], [1.0], U=[1.0, float("nan"), 0.0])
    h = ctypes.c_void_p()
    assert L.hub_sector_create(ctypes.byref(m), 1, 1, ctypes.byref(h)) == 1


def test_continued_fraction_host_entry_point():
    """hub_continued_fraction runs on the host: compare with the oracle's own
    continued fraction on random coefficients, and check the empty fraction."""
    import numpy as np
    import oracle.greens as og
    import paper_1307_7542_amd as hub
    rng = np.random.default_rng(5)
    a = rng.normal(size=40)
    b = np.concatenate([[0.0], rng.uniform(0.2, 1.5, size=39)])
    w = rng.normal(size=16) + 1j * rng.uniform(0.05, 2.0, size=16)
    got = hub.continued_fraction(a, b, 40, 0.8, w)
    ref = og.continued_fraction(a, b[1:], 0.8, w)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)
    assert np.all(hub.continued_fraction(a, b, 0, 0.8, w) == 0)


def test_binding_fails_loudly_without_library(monkeypatch):
    """With the shared library absent the binding raises: there is no CPU path
    behind it."""
    import paper_1307_7542_amd as hub
    monkeypatch.setattr(hub, "LIB_PATH", os.path.join(ROOT, "does_not_exist", "libhubbard.so"))
    monkeypatch.setattr(hub, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        hub.lib()


def test_bench_refuses_several_gpus():
    """bench.py runs on one GPU; asked for more it prints one JSON line naming
    the error and exits with status 2 before touching a device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
