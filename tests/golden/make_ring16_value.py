"""Write ring16_u4_oracle.json: the ground energy of the periodic chain M=16,
t=1, U=4, N_up=N_dn=8 (dim 165,636,900; Table IV's second row), computed by
the CPU oracle only.

The two-spin CSR of this sector would not fit in host memory, so every product
is the oracle's matrix-free row evaluation (Eq. count1 row by row, hops by the
esign rule of Sec. III A, binary search over the implicit sorted two-spin keys
of Sec. II) inside the oracle's FP64 Lanczos without reorthogonalisation (the
recurrence of Sec. IV, as the paper runs it), from the SplitMix64 start vector
of seed 7542.  About an hour on 8 host cores.

Run from the repository root:  python tests/golden/make_ring16_value.py
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


def main():
    m = W.config("ring16")
    sec = oracle.Sector(m, explicit_keys=False)
    rows = np.arange(sec.dim, dtype=np.int64)
    calls = [0]
    t0 = time.time()

    def matvec(x):
        y = sec.apply_rows(rows, x)
        calls[0] += 1
        print(f"product {calls[0]} at {time.time() - t0:.0f} s", flush=True)
        return y

    r = oracle.lanczos(matvec, sec.dim, oracle.start_vector(7542, sec.dim), tol=1e-12, max_iter=400,
                       reorth=False, want_vector=False)
    out = {"workload": "ring16: periodic chain M=16, t=1, U=4, N_up=N_dn=8",
           "dim": int(sec.dim), "e0": float(r.e0), "iters": int(r.iters), "ritz_residual": float(r.residual),
           "method": "oracle matrix-free rows (two-spin keys, binary search) + FP64 Lanczos without "
                     "reorthogonalisation, Ritz residual <= 1e-12 |E0|, start seed 7542",
           "threads": oracle.num_threads(), "seconds": time.time() - t0,
           "table4_printed": -9.2144309716}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ring16_u4_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
