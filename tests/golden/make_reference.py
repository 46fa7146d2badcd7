"""Write the stored OLS references of the large workloads (calls only the oracle).

For each workload the script regenerates the seeded data, records its xxh64
fingerprint (so that a later run can check it regenerated bit for bit), and
stores from the oracle: beta_star (Householder-QR OLS of [X|Y] followed by
corrected-seminormal refinement with extended-precision residuals), the plain
QR solution's distance to it (the FP64 floor) and, for the backward workload,
lambda = (X^T X)^{-1} w.

    python tests/golden/make_reference.py [workload ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ols as O  # noqa: E402
from oracle import slse as OS  # noqa: E402
from scipy.linalg import solve_triangular  # noqa: E402
from slse_inputs import fingerprint, make_batched, make_problem  # noqa: E402
from slse_inputs.generators import loss_vector  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def batched():
    t0 = time.time()
    probs = make_batched()
    out = dict(workload="batched",
               provenance="written by tests/golden/make_reference.py from oracle.ols.ols_refined",
               problems=[])
    for p in probs:
        bstar, bqr, _ = O.ols_refined(p.X, p.Y)
        out["problems"].append(dict(N=int(p.n), d=int(p.d), fingerprint=fingerprint(p.X, p.Y),
                                    beta_star=[float(v) for v in bstar],
                                    fp64_floor=OS.rel_err(bqr, bstar)))
    out["seconds"] = time.time() - t0
    path = os.path.join(HERE, "ref_batched.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"batched: {len(probs)} problems, {out['seconds']:.0f}s -> {path}", flush=True)


def main(names):
    for name in names:
        if name == "batched":
            batched()
            continue
        t0 = time.time()
        p = make_problem(name)
        t1 = time.time()
        fp = fingerprint(p.X, p.Y)
        bstar, bqr, R = O.ols_refined(p.X, p.Y)
        out = dict(
            workload=name,
            provenance="written by tests/golden/make_reference.py from oracle.ols.ols_refined",
            N=int(p.n), d=int(p.d), dtype=p.X.dtype.name, fingerprint=fp,
            beta_star=[float(v) for v in bstar],
            fp64_floor=OS.rel_err(bqr, bstar),
            rel_err_vs_truth=OS.rel_err(bstar, p.beta_true),
            seconds_generate=t1 - t0, seconds_oracle=time.time() - t1,
        )
        if name == "backward":
            w = loss_vector(p.d)
            lam = solve_triangular(R, solve_triangular(R, w, trans="T"))
            out["w"] = [float(v) for v in w]
            out["lambda"] = [float(v) for v in lam]
        path = os.path.join(HERE, f"ref_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(f"{name}: floor {out['fp64_floor']:.2e}, generate {t1 - t0:.0f}s, oracle {out['seconds_oracle']:.0f}s -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["illcond", "backward", "mixed"])
