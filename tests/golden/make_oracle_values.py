"""Write oracle_values.json: ground energies computed by the CPU oracle only.

Run from the repository root:  python tests/golden/make_oracle_values.py
Each entry records the workload, the method (dense LAPACK eigh or FP64 Lanczos
on the oracle's two-spin CSR) and E0.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def solve(m):
    sec = oracle.Sector(m)
    if sec.dim <= 2500:
        e0 = float(np.linalg.eigvalsh(sec.dense())[0])
        return sec.dim, e0, "dense_eigh"
    csr = sec.csr()
    r = oracle.lanczos(lambda x: oracle.spmv(csr, x), sec.dim, oracle.start_vector(7542, sec.dim),
                       tol=1e-13, reorth=sec.dim <= 100_000, want_vector=False)
    return sec.dim, float(r.e0), "lanczos_fp64"


def main():
    out = {"note": "E0 computed by the CPU oracle (two-spin CSR); start seed 7542", "entries": {}}
    cases = [("ring8", W.config("ring8"))]
    for U in (2, 4, 8):
        cases.append((f"ring14_u{U}", W.config(f"ring14_u{U}")))
    cases.append(("square3x4_n5", W.square_periodic(3, 4, n_up=5, n_dn=5)))
    cases.append(("ladder2x5", W.ladder(5)))
    cases.append(("ladder2x6", W.ladder(6)))
    for p, m in enumerate(W.aim_batch(64)):
        cases.append((f"aim{p}", m))
    for name, m in cases:
        t = time.time()
        dim, e0, how = solve(m)
        out["entries"][name] = {"dim": dim, "e0": e0, "method": how, "n_up": m.n_up, "n_dn": m.n_dn,
                                "n_sites": m.n_sites}
        print(f"{name:14s} dim={dim:9d} e0={e0:.14f} {how} {time.time() - t:.1f}s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
