"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bit-exact: bases, ranks, hopping-matrix columns, values (exact negations of t)
and bond ids, start vectors.  Floating point: the product within
1e-13 * sum_J |H_IJ x_J| (FP64) and 1e-5 * sum_J |H_IJ x_J| (FP32 with FP32
accumulation, about 17 rounded terms per row); ground energies within 1e-10
relative (FP64) and 1e-6 relative (mixed).
"""
import itertools
import json
import math
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


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _nonuniform_models():
    ms = [W.random_graph(7, 10, seed=s, site_U=True) for s in (101, 102)]
    ms.append(W.aim_batch(4)[1])
    return ms


# ------------------------------------------------------------ bases ----

@pytest.mark.parametrize("M", [1, 2, 3, 5, 8, 13, 16, 20])
def test_basis_bit_exact(hub, M):
    for N in sorted({0, 1, M // 3, M // 2, M - 1, M}):
        if N < 0 or N > M:
            continue
        m = W.Model("chain", M, [], [], [1.0] * M, [0.0] * M, N, max(0, min(M, M - N)))
        s = hub.Sector(m)
        ref = oracle.enumerate_basis(M, N)
        assert np.array_equal(s.basis(0), ref)
        assert s.count_up == math.comb(M, N)
        s.close()


def test_basis_m32_edges(hub):
    for N in (0, 1, 2, 31, 32):
        m = W.Model("m32", 32, [], [], [0.0] * 32, [0.0] * 32, N, N)
        s = hub.Sector(m)
        ref = sorted(sum(1 << p for p in c) for c in itertools.combinations(range(32), N))
        assert s.basis(0).tolist() == ref
        s.close()


def test_rank_bit_exact_and_invalid(hub):
    M, N = 12, 5
    m = W.Model("r", M, [], [], [0.0] * M, [0.0] * M, N, N)
    s = hub.Sector(m)
    basis = oracle.enumerate_basis(M, N)
    rng = np.random.default_rng(3)
    xs = np.concatenate([basis, rng.integers(0, 1 << 14, size=3000).astype(np.uint64),
                         np.array([0, (1 << 12) - 1, 1 << 40, (1 << 64) - 1], dtype=np.uint64)])
    got = s.rank(0, xs)
    pos = {int(v): i for i, v in enumerate(basis)}
    exp = np.array([pos.get(int(v), -1) for v in xs], dtype=np.int64)
    assert np.array_equal(got, exp)
    s.close()


# ------------------------------------------------------ hopping CSR ----

def _project_sigma(osec, spin):
    """H_sigma read off the oracle's full H: entries whose other-spin part is
    unchanged, taken at the first other-spin state."""
    rp, col, val = osec.csr()
    M = osec.m.M
    cu, cd = osec.cu, osec.cd
    rows = {}
    if spin == 0:
        for a in range(cu):
            r = a  # b = 0
            ent = []
            for k in range(rp[r], rp[r + 1]):
                c = int(col[k])
                if c != r and c // cu == 0:
                    ent.append((c % cu, val[k]))
            rows[a] = ent
        n = cu
    else:
        for b in range(cd):
            r = b * cu  # a = 0
            ent = []
            for k in range(rp[r], rp[r + 1]):
                c = int(col[k])
                if c != r and c % cu == 0:
                    ent.append((c // cu, val[k]))
            rows[b] = ent
        n = cd
    del M
    return [rows[i] for i in range(n)]


@pytest.mark.parametrize("which", ["ring8", "rand7a", "rand7b", "aim", "square3x3", "ring6_32"])
def test_hopping_csr_bit_exact(hub, which):
    if which == "ring8":
        m = W.config("ring8")
    elif which == "rand7a":
        m = W.random_graph(7, 12, seed=201).with_params(n_up=3, n_dn=4)
    elif which == "rand7b":
        m = W.random_graph(7, 21, seed=202).with_params(n_up=2, n_dn=5)
    elif which == "aim":
        m = W.aim_batch(3)[0]
    elif which == "square3x3":
        m = W.square_periodic(3, 3, n_up=4, n_dn=3)
    else:
        m = W.ring(6, n_up=3, n_dn=2)
    s = hub.Sector(m)
    osec = oracle.Sector(m)
    bi, bj, tt = s.bonds()
    for spin in (0, 1):
        rp, col, val, bond = s.hopping_csr(spin)
        ref = _project_sigma(osec, spin)
        basis = s.basis(spin)
        assert rp[0] == 0 and rp[-1] == len(col)
        for p, ent in enumerate(ref):
            got_c = col[rp[p]:rp[p + 1]].tolist()
            got_v = val[rp[p]:rp[p + 1]].tolist()
            assert got_c == [c for c, _ in ent], (spin, p)
            assert got_v == [v for _, v in ent], (spin, p)
            for k in range(rp[p], rp[p + 1]):
                mask = int(basis[p]) ^ int(basis[col[k]])
                e = bond[k]
                assert mask == (1 << int(bi[e])) | (1 << int(bj[e]))
        N = m.n_up if spin == 0 else m.n_dn
        if m.n_sites > 2 and 0 < N < m.n_sites:
            assert len(col) == 2 * len(bi) * math.comb(m.n_sites - 2, N - 1)
    s.close()


def test_shared_tables_when_sz0(hub):
    m = W.config("ring8")
    s = hub.Sector(m)
    a = s.hopping_csr(0)
    b = s.hopping_csr(1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    s.close()


def test_duplicate_bonds_merged(hub):
    m = W.ring(5, n_up=2, n_dn=2)
    m2 = m.with_params()
    m2.bonds = list(m.bonds) + [(1, 0), (3, 2)]
    m2.t = list(m.t) + [0.25, -0.5]
    s = hub.Sector(m2)
    bi, bj, tt = s.bonds()
    assert len(bi) == 5
    assert tt[0] == 1.25 and tt[2] == 0.5
    osec = oracle.Sector(m2)
    rp, col, val, _ = s.hopping_csr(0)
    ref = _project_sigma(osec, 0)
    for p, ent in enumerate(ref):
        assert col[rp[p]:rp[p + 1]].tolist() == [c for c, _ in ent]
        np.testing.assert_allclose(val[rp[p]:rp[p + 1]], [v for _, v in ent], rtol=0, atol=1e-15)
    s.close()


# ---------------------------------------------------------- product ----

def _row_abs(osec, x):
    rp, col, val = osec.csr()
    import scipy.sparse as sp
    A = sp.csr_matrix((np.abs(val), col, rp), shape=(osec.dim, osec.dim))
    return A @ np.abs(x)


@pytest.mark.parametrize("which", ["ring8", "rand8", "aim", "square3x4", "ladder2x5", "ring10_odd", "dimn0"])
def test_matvec_parity(hub, which):
    import torch
    if which == "ring8":
        m = W.config("ring8")
    elif which == "rand8":
        m = W.random_graph(8, 14, seed=301, site_U=True).with_params(n_up=4, n_dn=3)
    elif which == "aim":
        m = W.aim_batch(8)[5]
    elif which == "square3x4":
        m = W.square_periodic(3, 4, n_up=4, n_dn=5)
    elif which == "ladder2x5":
        m = W.ladder(5, n_up=5, n_dn=4)
    elif which == "ring10_odd":
        m = W.ring(10, U=3.0, n_up=3, n_dn=6)
    else:
        m = W.ring(6, n_up=0, n_dn=3)
    s = hub.Sector(m)
    osec = oracle.Sector(m)
    assert s.dim == osec.dim
    x64 = s.start_vector(seed=77, normalize=False)
    xr = oracle.start_vector(77, osec.dim)
    assert np.array_equal(x64.cpu().numpy(), xr)
    yr = oracle.spmv(osec.csr(), xr)
    bound = _row_abs(osec, xr)
    y64 = s.matvec(x64).cpu().numpy()
    assert np.all(np.abs(y64 - yr) <= 1e-13 * bound + 1e-300)
    x32 = x64.to(torch.float32)
    y32 = s.matvec(x32).cpu().numpy().astype(np.float64)
    yr32 = oracle.spmv(osec.csr(), x32.cpu().numpy().astype(np.float64))
    assert np.all(np.abs(y32 - yr32) <= 1e-5 * bound + 1e-30)
    # the diagonal alone
    d = s.diagonal().cpu().numpy()
    rp, col, val = osec.csr()
    dr = np.array([val[rp[r]:rp[r + 1]][col[rp[r]:rp[r + 1]] == r].sum() for r in range(osec.dim)])
    scale = np.sum(np.abs(m.U)) + 2 * np.sum(np.abs(m.eps)) + 1e-300
    assert np.all(np.abs(d - dr) <= 1e-14 * scale)
    s.close()


def test_matvec_repeatable_bitwise(hub):
    m = W.square_periodic(3, 4, n_up=5, n_dn=5)
    s = hub.Sector(m)
    x = s.start_vector(seed=5)
    y1 = s.matvec(x).cpu().numpy()
    y2 = s.matvec(x).cpu().numpy()
    assert np.array_equal(y1, y2)
    s.close()


def test_matvec_rejects_overlap(hub):
    import ctypes
    import torch
    s = hub.Sector(W.config("ring8"))
    x = s.start_vector(seed=1)
    with pytest.raises(hub.HubError):
        s.matvec(x, x)
    buf = torch.zeros(2 * s.dim + 4, dtype=torch.float64, device="cuda")
    with pytest.raises(hub.HubError):          # partial overlap
        s.matvec(buf[:s.dim], buf[5:5 + s.dim])
    # a pointer that is not aligned to its element is refused before any launch
    st = hub.lib().hub_matvec(s._h, hub.F64, ctypes.c_void_p(buf.data_ptr() + 4),
                              ctypes.c_void_p(buf.data_ptr() + 8 * (s.dim + 2)), None)
    assert st == 1  # HUB_ERR_INVALID_ARG
    s.close()


@pytest.mark.parametrize("name", ["ring14_u4", "square4x4"])
def test_matvec_sampled_full_size(hub, name):
    """Full-size workloads: rows sampled across the whole vector (first, last,
    random) checked against the oracle's matrix-free rows on the same
    SplitMix64 vector."""
    m = W.config(name)
    s = hub.Sector(m)
    osec = oracle.Sector(m, explicit_keys=False)
    x = s.start_vector(seed=4242, normalize=False)
    rng = np.random.default_rng(9)
    rows = np.unique(np.concatenate([[0, 1, s.dim - 1, s.dim - 2], rng.integers(0, s.dim, size=4000)]))
    y = s.matvec(x)
    yg = y[rows].cpu().numpy() if False else y.cpu().numpy()[rows]
    yr = osec.apply_rows(rows, None, seed=4242)
    assert np.max(np.abs(yg - yr)) <= 1e-12 * (np.max(np.abs(yr)) + 1)
    import torch
    y32 = s.matvec(x.to(torch.float32)).cpu().numpy()[rows].astype(np.float64)
    assert np.max(np.abs(y32 - yr)) <= 2e-5 * (np.max(np.abs(yr)) + 1)
    s.close()


# ---------------------------------------------------------- Lanczos ----

@pytest.mark.parametrize("which", ["ring8", "rand8", "aim0", "aim3", "dimer", "square3x3"])
def test_ground_state_fp64_vs_dense(hub, which):
    import torch
    if which == "ring8":
        m = W.config("ring8")
    elif which == "rand8":
        m = W.random_graph(8, 13, seed=401, site_U=True).with_params(n_up=4, n_dn=3)
    elif which == "aim0":
        m = W.aim_batch(1)[0]
    elif which == "aim3":
        m = W.aim_batch(4)[3]
    elif which == "dimer":
        m = W.dimer(U=4.0)
    else:
        m = W.square_periodic(3, 3, n_up=4, n_dn=4)
    osec = oracle.Sector(m)
    if osec.dim <= 5000:
        w, v = np.linalg.eigh(osec.dense())
        e_ref, psi_ref, gap = w[0], v[:, 0], w[1] - w[0] if len(w) > 1 else 1.0
    else:
        _, e_ref, psi_ref = oracle.ground_state(m, dense_max=0, tol=1e-13)
        gap = 1.0
    s = hub.Sector(m)
    for reorth in (False, True):
        gs = s.ground_state(dtype=0, reorth=reorth, refine=True, tol=1e-13)
        assert abs(gs.e0 - e_ref) <= 1e-10 * abs(e_ref), (reorth, gs.e0, e_ref)
        assert abs(gs.info["e0_ritz"] - e_ref) <= 1e-10 * abs(e_ref)
        psi = gs.psi.cpu().numpy()
        assert abs(np.linalg.norm(psi) - 1) < 1e-12
        if gap > 1e-6:
            assert abs(np.dot(psi, psi_ref)) >= 1 - 1e-10
            assert np.allclose(psi, oracle.canonical_sign(psi_ref), atol=1e-6)
    s.close()
    del torch


@pytest.mark.parametrize("which", ["ring8", "aim2", "rand9"])
def test_ground_state_mixed(hub, which):
    if which == "ring8":
        m = W.config("ring8")
    elif which == "aim2":
        m = W.aim_batch(3)[2]
    else:
        m = W.random_graph(9, 15, seed=402).with_params(n_up=4, n_dn=4)
    osec = oracle.Sector(m)
    if osec.dim <= 5000:
        e_ref = np.linalg.eigvalsh(osec.dense())[0]
    else:
        _, e_ref, _ = oracle.ground_state(m, dense_max=0, tol=1e-13, want_vector=False)
    s = hub.Sector(m)
    for reorth in (True, False):
        gs = s.ground_state(dtype=1, reorth=reorth, refine=True)
        assert abs(gs.info["e0_ritz"] - e_ref) <= 1e-6 * abs(e_ref)
        assert abs(gs.e0 - e_ref) <= 1e-6 * abs(e_ref)
    s.close()


def test_degenerate_one_state_sectors(hub):
    """dim = 1 (N = 0 or N = M for both spins): E0 = D exactly, breakdown at step 1."""
    for n_up, n_dn, expect in [(0, 0, 0.0), (6, 6, 6 * 2.5), (6, 0, 0.0)]:
        m = W.ring(6, U=2.5, n_up=n_up, n_dn=n_dn)
        s = hub.Sector(m)
        assert s.dim == 1
        gs = s.ground_state(dtype=0)
        assert gs.e0 == expect
        assert gs.info["breakdown"] == 1
        s.close()


def test_t0_and_u0_closed_forms(hub):
    m = W.ring(10, t=0.0, U=3.0, n_up=6, n_dn=7)
    s = hub.Sector(m)
    gs = s.ground_state(dtype=0, want_vector=False)
    assert abs(gs.e0 - 3.0 * 3) < 1e-12
    s.close()
    m = W.ring(14, U=0.0, n_up=7, n_dn=7)
    s = hub.Sector(m)
    gs = s.ground_state(dtype=0, want_vector=False)
    h = np.zeros((14, 14))
    for (i, j), t in zip(m.bonds, m.t):
        h[i, j] -= t
        h[j, i] -= t
    w = np.linalg.eigvalsh(h)
    assert abs(gs.e0 - 2 * w[:7].sum()) <= 1e-10 * abs(gs.e0)
    s.close()


def test_table4_m14_m16(hub):
    """Sec. V, Table IV, U=4: FP64 Lanczos on the GPU against the oracle's
    energies (M=14 from the stored oracle values, M=16 from the oracle's
    matrix-free Lanczos, tests/golden/ring16_u4_oracle.json) at 1e-10, and
    against the printed E_min (values read as truncated at 10 decimals)."""
    g = _gold("table4_emin.json")
    ov = _gold("oracle_values.json")["entries"]
    e16 = _gold("ring16_u4_oracle.json")["e0"]
    for row in g["rows"]:
        m = W.ring(row["M"], U=4.0, n_up=row["n_up"], n_dn=row["n_dn"])
        s = hub.Sector(m)
        assert s.dim == row["dim"]
        gs = s.ground_state(dtype=0, want_vector=False, tol=1e-12)
        if row["M"] == 14:
            # agrees with the printed digits (truncated) and with the oracle
            assert row["E_min"] - 1e-10 < gs.e0 <= row["E_min"] + 1e-12, (row["M"], gs.e0)
            e_or = ov["ring14_u4"]["e0"]
            assert abs(gs.e0 - e_or) <= 1e-10 * abs(e_or)
        else:
            assert abs(gs.e0 - e16) <= 1e-10 * abs(e16), (gs.e0, e16)
            # the oracle's E0 is 3.8e-10 below the printed value, outside its print
            # precision: read as the paper's plain Lanczos stopping before full convergence
            assert 0.0 < row["E_min"] - e16 < 5e-10, (row["E_min"], e16)
            assert abs(gs.e0 - row["E_min"]) < 5e-10, (row["M"], gs.e0)
            # the other boundary reading (no fermion sign on the wrap-around hop,
            # i.e. antiperiodic one-body levels) is far from the printed value
            t_ap = list(m.t)
            t_ap[-1] = -t_ap[-1]
            s2 = hub.Sector(m.with_params(t=t_ap))
            ga = s2.ground_state(dtype=0, want_vector=False, tol=1e-10)
            assert abs(ga.e0 - row["E_min"]) > 1e-3, ga.e0
            s2.close()
        s.close()


@pytest.mark.parametrize("name", ["ring14_u2", "ring14_u8", "square3x4_n5", "ladder2x6", "aim7", "aim40"])
def test_ground_state_vs_stored_oracle(hub, name):
    ov = _gold("oracle_values.json")["entries"][name]
    if name.startswith("ring14"):
        m = W.config(name)
    elif name == "square3x4_n5":
        m = W.square_periodic(3, 4, n_up=5, n_dn=5)
    elif name == "ladder2x6":
        m = W.ladder(6)
    else:
        m = W.aim_batch(64)[int(name[3:])]
    s = hub.Sector(m)
    assert s.dim == ov["dim"]
    gs = s.ground_state(dtype=0, want_vector=False, tol=1e-12)
    assert abs(gs.e0 - ov["e0"]) <= 1e-10 * abs(ov["e0"])
    gm = s.ground_state(dtype=1, reorth=False, refine=True)
    assert abs(gm.e0 - ov["e0"]) <= 1e-6 * abs(ov["e0"])
    s.close()


# ---------------------------------------------------------- adjoint ----

@pytest.mark.parametrize("which", ["rand7", "aim5", "square3x3"])
def test_param_bilinear_vs_oracle(hub, which):
    import torch
    if which == "rand7":
        m = W.random_graph(7, 11, seed=501, site_U=True).with_params(n_up=3, n_dn=4)
    elif which == "aim5":
        m = W.aim_batch(6)[5]
    else:
        m = W.square_periodic(3, 3, n_up=4, n_dn=4)
    s = hub.Sector(m)
    osec = oracle.Sector(m)
    g = s.start_vector(seed=1)
    x = s.start_vector(seed=2)
    db, dU, de = s.param_bilinear(g, x)
    rdb, rdU, rde = osec.param_bilinear(oracle.start_vector(1, s.dim) / np.linalg.norm(oracle.start_vector(1, s.dim)),
                                        oracle.start_vector(2, s.dim) / np.linalg.norm(oracle.start_vector(2, s.dim)))
    np.testing.assert_allclose(db, rdb, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(dU, rdU, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(de, rde, rtol=1e-10, atol=1e-12)
    # Hellmann-Feynman at the ground state and the Euler identity
    gs = s.ground_state(dtype=0, tol=1e-13)
    db, dU, de = s.param_bilinear(gs.psi, gs.psi)
    euler = np.dot(m.t, db) + np.dot(m.U, dU) + np.dot(m.eps, de)
    assert abs(euler - gs.e0) <= 1e-9 * abs(gs.e0)
    s.close()
    del torch


# shapes of the row-chunked product (columns per work item, lane-quads per lane)
_CHUNKED_VARIANTS = {
    "tb1_q4": dict(tile_cols=1, quads_per_lane=4),
    "tb2_q4": dict(tile_cols=2, quads_per_lane=4),
    "tb1_q8": dict(tile_cols=1, quads_per_lane=8),
}


@pytest.mark.parametrize("chunk", [64, 200, 1000])
@pytest.mark.parametrize("variant", sorted(_CHUNKED_VARIANTS))
def test_matvec_row_chunked_parity(hub, chunk, variant):
    """The row-chunked product (used when a column exceeds the LDS) forced on
    small sectors with several chunks and a ragged last chunk, in each shape;
    products against the oracle, and a solve through the same schedule."""
    import torch
    kw = dict(_CHUNKED_VARIANTS[variant])
    for m in (W.square_periodic(3, 4, n_up=5, n_dn=4), W.random_graph(10, 17, seed=303, site_U=True, n_up=3)):
        s = hub.Sector(m)
        assert s.count_up % 4 == 0
        for dt in (hub.F64, hub.F32):
            s.set_schedule(dt, hub.SCHED_CHUNKED, chunk_rows=chunk, **kw)
        osec = oracle.Sector(m)
        xr = oracle.start_vector(5, osec.dim)
        yr = oracle.spmv(osec.csr(), xr)
        bound = _row_abs(osec, xr)
        x64 = s.start_vector(seed=5, normalize=False)
        y64 = s.matvec(x64).cpu().numpy()
        assert np.all(np.abs(y64 - yr) <= 1e-13 * bound + 1e-300)
        x32 = x64.to(torch.float32)
        y32 = s.matvec(x32).cpu().numpy().astype(np.float64)
        yr32 = oracle.spmv(osec.csr(), x32.cpu().numpy().astype(np.float64))
        assert np.all(np.abs(y32 - yr32) <= 1e-5 * bound + 1e-30)
        gs = s.ground_state(dtype=hub.F64, want_vector=False, tol=1e-12)
        e_ref = np.linalg.eigvalsh(osec.dense())[0] if osec.dim <= 4000 else None
        if e_ref is not None:
            assert abs(gs.e0 - e_ref) <= 1e-10 * abs(e_ref)
        s.close()


def _all_schedules(hub, s, dt):
    """Every schedule family and shape the sector can run in dtype dt."""
    out = []
    for tb in (1, 2, 3):
        for bs in (512, 1024):
            for xc in (0, 1):
                out.append(dict(family=hub.SCHED_COLUMNS, tile_cols=tb, block=bs, order=xc))
    shapes = [(1, 4), (2, 4), (1, 8)] + ([(2, 8), (4, 4)] if dt == hub.F32 else [])
    for tb, qpl in shapes:
        for chunk in (128, 200, 0):
            out.append(dict(family=hub.SCHED_CHUNKED, tile_cols=tb, quads_per_lane=qpl, chunk_rows=chunk))
    out.append(dict(family=hub.SCHED_ROWS))
    out.append(dict(family=hub.SCHED_CSR))
    return out


@pytest.mark.parametrize("which", ["ring10", "square3x4_n5", "ring12_u3"])
def test_product_schedules_bitwise(hub, which):
    """Every schedule the tuner may pick or a caller may force (whole columns in
    LDS with 1-3 columns per workgroup, row-chunked columns in every shape and
    chunk size, one row per lane, CSR rows) computes each element with the same
    operations in the same order: the products are bit-identical to the tuned
    one and match the oracle."""
    import torch
    if which == "ring10":
        m = W.ring(10, U=3.0, n_up=5, n_dn=4).with_params(eps=[0.1 * i for i in range(10)])
    elif which == "square3x4_n5":
        m = W.square_periodic(3, 4, n_up=5, n_dn=5)
    else:
        m = W.ring(12, U=3.0, n_up=6, n_dn=6)
    s = hub.Sector(m)
    assert s.count_up % 4 == 0
    osec = oracle.Sector(m)
    xr = oracle.start_vector(31, osec.dim)
    yr = oracle.spmv(osec.csr(), xr)
    bound = _row_abs(osec, xr)
    for dt, tol in ((hub.F64, 1e-13), (hub.F32, 1e-5)):
        x = torch.from_numpy(xr).cuda()
        if dt == hub.F32:
            x = x.float()
            ref = oracle.spmv(osec.csr(), x.cpu().numpy().astype(np.float64))
        else:
            ref = yr
        y0 = s.matvec(x).cpu().numpy()
        assert s.schedule(dt)["family"] in (hub.SCHED_COLUMNS, hub.SCHED_CHUNKED)
        assert np.all(np.abs(y0.astype(np.float64) - ref) <= tol * bound + 1e-30)
        for sc in _all_schedules(hub, s, dt):
            s.set_schedule(dt, **sc)
            y = s.matvec(x).cpu().numpy()
            assert np.array_equal(y, y0), (which, dt, sc)
        s.set_schedule(dt, None)
    s.close()


def test_time_to_target_energy(hub):
    """The solver records the first step whose lowest Ritz value is within the
    requested relative distance of a reference energy (the time-to-E0 measure)."""
    m = W.config("ring8")
    s = hub.Sector(m)
    _, e_ref, _ = oracle.ground_state(m)
    g = s.ground_state(dtype=hub.F64, tol=1e-12, want_vector=False, e0_target=e_ref, e0_target_rel=1e-6)
    it, sec = g.info["iters_to_target"], g.info["seconds_to_target"]
    assert 1 <= it <= g.info["iters"] and 0.0 < sec <= g.info["seconds"]
    g2 = s.ground_state(dtype=hub.F64, tol=1e-12, want_vector=False, e0_target=e_ref, e0_target_rel=1e-10)
    assert it <= g2.info["iters_to_target"] <= g2.info["iters"]
    g3 = s.ground_state(dtype=hub.F64, tol=1e-12, want_vector=False)
    assert g3.info["iters_to_target"] == -1 and g3.info["seconds_to_target"] == -1.0
    # a target never met (an energy below the ground state)
    g4 = s.ground_state(dtype=hub.F64, tol=1e-12, want_vector=False, e0_target=e_ref - 1.0, e0_target_rel=1e-6)
    assert g4.info["iters_to_target"] == -1
    s.close()


@pytest.mark.parametrize("which", ["ring12_u3", "square3x4_n5"])
def test_sampled_kernel_timing_leaves_results_unchanged(hub, which):
    """Timing every N-th product with HIP events changes no arithmetic: the
    energies and the eigenvector are bitwise those of an untimed solve, and the
    number of timed launches is ceil(products / N)."""
    import torch
    if which == "ring12_u3":
        m = W.ring(12, U=3.0, n_up=6, n_dn=6)
    else:
        m = W.square_periodic(3, 4, n_up=5, n_dn=5)
    s = hub.Sector(m)
    for dt in (hub.F64, hub.F32):
        kw = dict(dtype=dt, tol=1e-12 if dt == hub.F64 else 1e-7, want_vector=True, refine=True)
        g0 = s.ground_state(**kw)
        for every in (1, 3):
            g = s.ground_state(time_kernels=every, **kw)
            assert g.e0 == g0.e0 and g.info["e0_ritz"] == g0.info["e0_ritz"]
            assert torch.equal(g.psi, g0.psi)
            cnt = g.info["matvec_count"]
            assert g.info["matvec_timed"] == (cnt + every - 1) // every
            assert g.info["matvec_ms"] > 0.0
        assert g0.info["matvec_timed"] == 0 and g0.info["matvec_ms"] == 0.0
    s.close()


def test_unnormalised_recurrence_matches_normalised(hub):
    """The plain fused path keeps beta_k v_k instead of v_k; the energies and the
    eigenvector agree with the normalised, unfused recurrence (a schedule forced
    with no_fused_update)."""
    import torch
    m = W.ring(12, U=3.0, n_up=6, n_dn=6).with_params(eps=[0.05 * ((7 * i) % 12) for i in range(12)])
    s = hub.Sector(m)
    assert s.count_up % 4 == 0
    for dt, tol_e, tol_v in ((hub.F64, 1e-12, 1e-9), (hub.F32, 1e-9, 1e-5)):
        kw = dict(dtype=dt, tol=1e-12 if dt == hub.F64 else 1e-7, want_vector=True, refine=True)
        g_un = s.ground_state(**kw)
        s.set_schedule(dt, hub.SCHED_COLUMNS, tile_cols=1, block=512, order=1, no_fused_update=True)
        g_no = s.ground_state(**kw)
        s.set_schedule(dt, None)
        assert abs(g_un.e0 - g_no.e0) <= tol_e * abs(g_no.e0), (dt, g_un.e0, g_no.e0)
        ov = float(torch.dot(g_un.psi, g_no.psi))
        assert abs(ov) >= 1.0 - tol_v, (dt, ov)
        assert g_un.info["true_residual"] <= (1e-9 if dt == hub.F64 else 1e-5) * abs(g_un.e0)
        # convergence tested every 4th step (waits on a later published step)
        g4 = s.ground_state(check_every=4, **kw)
        assert abs(g4.e0 - g_no.e0) <= tol_e * abs(g_no.e0) and g4.info["iters"] % 4 == 0
    s.close()


def test_unnormalised_recurrence_breakdown(hub):
    """t = 0 on a sector the fused product handles: H = D has seven distinct
    values, so the recurrence breaks down early; E0 = 0 (a state without double
    occupancy exists at half filling) on both precisions, with and without full
    reorthogonalisation (whose norms come from the Gram update's partials; at the
    breakdown step w is rounding noise, where the gated second pass matters)."""
    m = W.ring(12, t=0.0, U=2.0, n_up=6, n_dn=6)
    s = hub.Sector(m)
    assert s.count_up % 4 == 0
    for dt in (hub.F64, hub.F32):
        for reorth in (False, True):
            g = s.ground_state(dtype=dt, reorth=reorth, want_vector=True, refine=True)
            assert g.info["breakdown"] == 1 and g.info["iters"] <= 10, (dt, reorth, g.info)
            assert abs(g.e0) <= 1e-12, (dt, reorth, g.e0)
            assert g.info["true_residual"] <= 1e-6, (dt, reorth, g.info)
    s.close()


@pytest.mark.gpu
def test_fused_solve_same_for_every_tile_shape(hub):
    """The fused product's tile shape (columns per workgroup, workgroup size,
    tile order; or the row-chunked schedule and its shape) is tuned in each
    process, so a solve must not depend on it.  On a sector whose 91 down-spin
    columns leave a partial tile of two and of three columns, and whose 3432
    rows leave a partial group of 64 lane-quads, every forced shape gives the
    same energy and step count bit for bit, on both precisions, and that energy
    is the oracle's."""
    m = W.ring(14, U=4.0, n_up=7, n_dn=2)
    s = hub.Sector(m)
    assert s.count_up % 4 == 0 and s.count_dn % 2 == 1 and s.count_dn % 3 != 0
    assert (s.count_up // 4) % 64 != 0
    _, e_ref, _ = oracle.ground_state(m, want_vector=False)
    shapes = [(hub.SCHED_COLUMNS, dict(tile_cols=tb, block=bs, order=xc))
              for tb in (1, 2, 3) for bs in (512, 1024) for xc in (0, 1)]
    # the row-chunked product with its fused update forms the same per-column partials
    shapes += [(hub.SCHED_CHUNKED, dict(tile_cols=tb, quads_per_lane=qpl, chunk_rows=rows))
               for tb, qpl, rows in ((1, 4, 1000), (2, 4, 1500), (1, 8, 3432))]
    for dt, tol, rel in ((hub.F64, 1e-12, 1e-10), (hub.F32, 1e-7, 1e-5)):
        got = []
        for fam, kw in shapes:
            s.set_schedule(dt, fam, **kw)
            g = s.ground_state(dtype=dt, tol=tol, want_vector=False)
            got.append((g.e0, g.info["iters"]))
        assert all(r == got[0] for r in got), (dt, list(zip(shapes, got)))
        assert abs(got[0][0] - e_ref) <= rel * abs(e_ref), (dt, got[0], e_ref)
        s.set_schedule(dt, None)
    s.close()


@pytest.mark.gpu
def test_concurrent_products_on_one_sector(hub):
    """A sector serves products from several host threads on their own streams:
    four threads start on a lattice whose tile shape is not tuned yet (so they
    tune at the same time) and every product is bit-identical to a
    single-thread one, in both precisions."""
    import threading
    import torch
    m = W.ring(10, U=2.5, n_up=5, n_dn=3).with_params(eps=[0.03 * i for i in range(10)])
    s = hub.Sector(m)
    assert s.count_up % 4 == 0
    xs = {dt: s.start_vector(seed=11, dtype=dt) for dt in (hub.F64, hub.F32)}
    out, errors = {}, []

    def work(tid):
        try:
            st = torch.cuda.Stream()
            res = []
            with torch.cuda.stream(st):
                for rep in range(3):
                    for dt in (hub.F32, hub.F64):
                        y = s.empty(dt)
                        s.matvec(xs[dt], y, stream=st)
                        res.append((dt, y))
            st.synchronize()
            out[tid] = [(dt, y.cpu()) for dt, y in res]
        except Exception as e:  # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    assert len(out) == 4
    ref = {dt: s.matvec(xs[dt]).cpu() for dt in (hub.F64, hub.F32)}
    for tid, res in out.items():
        for dt, y in res:
            assert torch.equal(y, ref[dt]), (tid, dt)
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["ring8_n44", "ring8_n54"])
def test_first_steps_match_the_oracle_recurrence(hub, which):
    """One and two steps from the seeded start vector: with max_iter = 1 the
    Ritz value is alpha_0 = <v0, H v0> of the normalised start vector, with 2 the
    lowest eigenvalue of the 2 x 2 tridiagonal matrix of the oracle's recurrence.
    The 70-state up spin takes the one-row product; the 56-state one the fused,
    unnormalised path, whose last step fetches beta instead of publishing it."""
    import numpy as np
    n_up = 4 if which == "ring8_n44" else 5
    m = W.ring(8, U=3.0, n_up=n_up, n_dn=4).with_params(eps=[0.02 * i for i in range(8)])
    s = hub.Sector(m)
    assert (s.count_up % 4 == 0) == (which == "ring8_n54")
    osec = oracle.Sector(m)
    csr = osec.csr()
    v0 = oracle.start_vector(7542, osec.dim)
    r = oracle.lanczos(lambda x: oracle.spmv(csr, x), osec.dim, v0, max_iter=2, tol=0.0, reorth=False,
                       want_vector=False)
    a, b = r.alphas, r.betas
    t2 = np.linalg.eigvalsh(np.array([[a[0], b[0]], [b[0], a[1]]]))[0]
    for dt, tol in ((hub.F64, 1e-13), (hub.F32, 1e-6)):
        g1 = s.ground_state(dtype=dt, max_iter=1, want_vector=False, allow_not_converged=True)
        assert g1.info["iters"] == 1
        assert abs(g1.e0 - a[0]) <= tol * abs(a[0]), (dt, g1.e0, a[0])
        g2 = s.ground_state(dtype=dt, max_iter=2, want_vector=False, allow_not_converged=True)
        assert g2.info["iters"] == 2
        assert abs(g2.e0 - t2) <= tol * abs(t2), (dt, g2.e0, t2)
    s.close()


@pytest.mark.gpu
def test_thirty_two_sites(hub):
    """The widest lattice the 32-bit patterns allow: a 32-site ring with two up
    and one down electron (496 x 32 states; the up count is a multiple of 4, so
    the four-rows-per-lane product and the fused solver run).  The wrap bond's
    sign spans all 30 sites between its ends, and per-site U and eps include
    site 31.  Products and E0 against the oracle."""
    import torch
    M = 32
    U = [2.0 + 0.25 * ((5 * i) % 7) for i in range(M)]
    eps = [0.1 * ((3 * i) % 5) - 0.2 for i in range(M)]
    m = W.ring(M, U=2.0, n_up=2, n_dn=1).with_params(U=U, eps=eps)
    s = hub.Sector(m)
    assert s.count_up == 496 and s.count_dn == 32 and s.count_up % 4 == 0
    osec = oracle.Sector(m)
    xr = oracle.start_vector(3, osec.dim)
    bound = _row_abs(osec, xr)
    yr = oracle.spmv(osec.csr(), xr)
    for dt, tol in ((hub.F64, 1e-13), (hub.F32, 1e-5)):
        x = torch.from_numpy(xr).cuda()
        ref = yr
        if dt == hub.F32:
            x = x.float()
            ref = oracle.spmv(osec.csr(), x.cpu().numpy().astype(np.float64))
        y = s.matvec(x).cpu().numpy().astype(np.float64)
        assert np.all(np.abs(y - ref) <= tol * bound + 1e-30), dt
    # E0 of the oracle's H by ARPACK (a gap ratio of 1.6e-4 makes the oracle's
    # own reorthogonalised Lanczos take minutes here); the solves get the steps
    # such a gap needs
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    rp, col, val = osec.csr()
    e_ref = float(np.min(sla.eigsh(sp.csr_matrix((val, col, rp), shape=(osec.dim, osec.dim)), k=1,
                                   which="SA", tol=1e-13)[0]))
    g64 = s.ground_state(dtype=hub.F64, want_vector=False, max_iter=3000)
    g32 = s.ground_state(dtype=hub.F32, refine=True, max_iter=3000)
    assert abs(g64.e0 - e_ref) <= 1e-10 * abs(e_ref), (g64.e0, e_ref)
    assert abs(g32.e0 - e_ref) <= 1e-9 * abs(e_ref), (g32.e0, e_ref)
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["ring8_n44", "ring8_n53"])
def test_algorithmic_bytes_formula(hub, which):
    """The bytes every GB/s figure divides by: read x and write y once (2 dim s)
    plus, per distinct spin table, row pointers 4 (c + 1), entries nnz (4 + s),
    basis integers 4 c and site sums s c; one table when N_up = N_dn.  The
    counts come from the oracle (C(M, N) and the entries of H_sigma projected
    out of its full H)."""
    from math import comb
    n_up, n_dn = (4, 4) if which == "ring8_n44" else (5, 3)
    m = W.ring(8, U=3.0, n_up=n_up, n_dn=n_dn)
    s = hub.Sector(m)
    osec = oracle.Sector(m)
    spins = [0] if n_up == n_dn else [0, 1]
    for dt, es in ((hub.F64, 8), (hub.F32, 4)):
        want = 2 * osec.dim * es
        for sp_ in spins:
            c = comb(8, n_up if sp_ == 0 else n_dn)
            rows = _project_sigma(osec, sp_)
            nnz = sum(len(v) for v in rows)
            want += 4 * (c + 1) + nnz * (4 + es) + 4 * c + es * c
        assert s.matvec_bytes(dt) == want, (which, dt, s.matvec_bytes(dt), want)
    s.close()


def _variant_model(which):
    if which == "ring10_eps":
        return W.ring(10, U=3.0, n_up=5, n_dn=4).with_params(eps=[0.1 * i for i in range(10)])
    if which == "ring9":
        return W.ring(9, U=2.0, n_up=4, n_dn=3)           # count_up = 126 (not a multiple of 4)
    return W.square_periodic(3, 4, n_up=5, n_dn=5)


@pytest.mark.parametrize("variant", ["csr", "rows", "columns", "chunked"])
@pytest.mark.parametrize("which", ["ring10_eps", "ring9", "square3x4_n5"])
def test_product_variants_match_oracle(hub, variant, which):
    """Every product schedule against the oracle, on a sector with count_up % 4
    != 0 too (ring9: only the one-row and CSR schedules apply; the others are
    refused with INVALID_ARG)."""
    import torch
    m = _variant_model(which)
    s = hub.Sector(m)
    osec = oracle.Sector(m)
    xr = oracle.start_vector(19, osec.dim)
    bound = _row_abs(osec, xr)
    yr = oracle.spmv(osec.csr(), xr)
    fam = {"csr": hub.SCHED_CSR, "rows": hub.SCHED_ROWS, "columns": hub.SCHED_COLUMNS,
           "chunked": hub.SCHED_CHUNKED}[variant]
    kw = dict(tile_cols=2, block=1024, order=1)
    if variant == "chunked":
        kw = dict(tile_cols=2, quads_per_lane=4, chunk_rows=96)
    for dt, tol in ((hub.F64, 1e-13), (hub.F32, 1e-5)):
        if s.count_up % 4 != 0 and fam in (hub.SCHED_COLUMNS, hub.SCHED_CHUNKED):
            with pytest.raises(hub.HubError) as ei:
                s.set_schedule(dt, fam, **kw)
            assert ei.value.status == 1
            continue
        s.set_schedule(dt, fam, **kw)
        x = torch.from_numpy(xr).cuda()
        if dt == hub.F32:
            x = x.float()
        y = s.matvec(x).double().cpu().numpy()
        ref = yr if dt == hub.F64 else oracle.spmv(osec.csr(), x.double().cpu().numpy())
        assert np.all(np.abs(y - ref) <= tol * bound + 1e-30), (variant, which, dt)
    s.close()


def test_many_bonds_use_packed_entries(hub):
    """More than 127 bonds do not fit the 8-bit entry code: the product falls back
    to packed entries (all 136 pairs of 17 sites, random t, eps; N = 2/1)."""
    import torch
    m = W.random_graph(17, 136, seed=917).with_params(n_up=2, n_dn=1)
    assert len(m.bonds) == 136
    s = hub.Sector(m)
    osec = oracle.Sector(m)
    xr = oracle.start_vector(23, osec.dim)
    bound = _row_abs(osec, xr)
    yr = oracle.spmv(osec.csr(), xr)
    y = s.matvec(torch.from_numpy(xr).cuda()).cpu().numpy()
    assert np.all(np.abs(y - yr) <= 1e-13 * bound + 1e-300)
    g = s.ground_state(dtype=hub.F64, want_vector=False)
    e_ref = float(np.linalg.eigvalsh(osec.dense())[0])
    assert abs(g.e0 - e_ref) <= 1e-10 * abs(e_ref)
    s.close()


@pytest.mark.parametrize("variant", ["tb1_q4", "tb2_q4", "tb1_q8"])
def test_matvec_row_chunked_several_row_parts(hub, variant):
    """count_up = 18564 (ring M=18, N_up=6) is more than one row part of the
    register-held output (4096 or 8192 rows per work item): parts, chunks of
    5000 rows, 1 or 2 columns per work item (18 columns: a ragged last tile) and
    the ragged ends all at once, against the oracle."""
    import torch
    kw = _CHUNKED_VARIANTS[variant]
    m = W.ring(18, U=3.0, n_up=6, n_dn=1).with_params(eps=[0.03 * i for i in range(18)])
    s = hub.Sector(m)
    assert s.count_up == 18564
    for dt in (hub.F64, hub.F32):
        s.set_schedule(dt, hub.SCHED_CHUNKED, chunk_rows=5000, **kw)
    osec = oracle.Sector(m)
    xr = oracle.start_vector(41, osec.dim)
    bound = _row_abs(osec, xr)
    yr = oracle.spmv(osec.csr(), xr)
    x64 = torch.from_numpy(xr).cuda()
    y64 = s.matvec(x64).cpu().numpy()
    assert np.all(np.abs(y64 - yr) <= 1e-13 * bound + 1e-300)
    x32 = x64.float()
    y32 = s.matvec(x32).double().cpu().numpy()
    yr32 = oracle.spmv(osec.csr(), x32.double().cpu().numpy())
    assert np.all(np.abs(y32 - yr32) <= 1e-5 * bound + 1e-30)
    s.close()


def test_chunked_solve_same_for_every_shape(hub):
    """The row-chunked product's shape (columns per work item, lane-quads per
    lane, chunk rows) is tuned in each process, so a solve through it must not
    depend on it: on count_up = 18564 (several row parts and chunks, 18 columns
    leaving ragged tiles of 2 and 4), every forced shape gives the same energy
    and step count bit for bit, in both precisions, and that energy is the
    oracle's."""
    m = W.ring(18, U=3.0, n_up=6, n_dn=1).with_params(eps=[0.03 * i for i in range(18)])
    s = hub.Sector(m)
    _, e_ref, _ = oracle.ground_state(m, want_vector=False)
    shapes = {hub.F64: [(1, 4, 5000), (2, 4, 5000), (1, 8, 5000), (1, 4, 12000)],
              hub.F32: [(1, 4, 5000), (2, 4, 5000), (1, 8, 5000), (2, 8, 5000), (4, 4, 5000)]}
    for dt, tol, rel in ((hub.F64, 1e-12, 1e-10), (hub.F32, 1e-7, 1e-5)):
        got = []
        for tb, qpl, rows in shapes[dt]:
            s.set_schedule(dt, hub.SCHED_CHUNKED, tile_cols=tb, quads_per_lane=qpl, chunk_rows=rows)
            g = s.ground_state(dtype=dt, tol=tol, want_vector=False)
            got.append((g.e0, g.info["iters"]))
        assert all(r == got[0] for r in got), (dt, list(zip(shapes[dt], got)))
        assert abs(got[0][0] - e_ref) <= rel * abs(e_ref), (dt, got[0], e_ref)
        s.set_schedule(dt, None)
    s.close()


@pytest.mark.parametrize("which", ["square3x4_n5", "ring10_eps"])
def test_matvec_unaligned_views(hub, which):
    """Vectors that start at an element but not a 16-byte boundary (views into a
    larger buffer) take the one-row-per-lane kernels and give the oracle's product;
    also with the row-chunked schedule forced."""
    import torch
    m = _variant_model(which)
    for chunk in (None, 200):
        s = hub.Sector(m)
        if chunk:
            for dt in (hub.F64, hub.F32):
                s.set_schedule(dt, hub.SCHED_CHUNKED, tile_cols=1, quads_per_lane=4, chunk_rows=chunk)
        osec = oracle.Sector(m)
        xr = oracle.start_vector(13, osec.dim)
        bound = _row_abs(osec, xr)
        for dt, tol in ((hub.F64, 1e-13), (hub.F32, 1e-5)):
            tdt = torch.float64 if dt == hub.F64 else torch.float32
            xb = torch.zeros(osec.dim + 1, dtype=tdt, device="cuda")
            yb = torch.zeros(osec.dim + 3, dtype=tdt, device="cuda")
            x = xb[1:]
            x.copy_(torch.from_numpy(xr).to(tdt))
            y = yb[3:]
            assert x.data_ptr() % 16 != 0 and y.data_ptr() % 16 != 0
            s.matvec(x, y)
            ref = oracle.spmv(osec.csr(), x.double().cpu().numpy())
            assert np.all(np.abs(y.double().cpu().numpy() - ref) <= tol * bound + 1e-30), (which, chunk, dt)
        s.close()