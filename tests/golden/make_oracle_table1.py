"""Write the oracle's tab:smooth results to ``table1_oracle.json``.

Calls only the CPU oracle (``oracle.etc_oracle``) and the closed-form problem
builder of ``tests/problems.py``: for each grid edge n, the smooth
orthotropic manufactured problem of tab:smooth (Section "Investigations on the
TPFA scheme") solved by alg:pcg at rtol 1e-9 with the midpoint reference
parameters and p0 = 0, and the L2 error of the solution against the exact
p at the cell centres (midpoint rule on the unit cube).

Usage:  python tests/golden/make_oracle_table1.py [n ...]   (default 128 256)
"""

from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for path in (ROOT, os.path.dirname(HERE)):
    if path not in sys.path:
        sys.path.insert(0, path)

from oracle import etc_oracle as O  # noqa: E402
from problems import smooth_problem  # noqa: E402

OUT = os.path.join(HERE, "table1_oracle.json")


def run(n: int) -> dict:
    t0 = time.time()
    comps, src, pin, pout, exact = smooth_problem(n)
    pb = O.make_problem(None, 2, pin, pout, L=(1.0, 1.0, 1.0), components=comps, source=src)
    res = O.pcg(pb, rtol=1e-9, max_iter=1000)
    p = O.decanonical(res.p, 2)
    err = math.sqrt(float(np.sum((p - exact) ** 2)) / n ** 3)
    rec = {"l2_error": err, "iters": res.iters, "relres": res.relres, "status": res.status,
           "seconds": time.time() - t0}
    print(f"n={n}: L2 error {err:.6e}, {res.iters} passes ({rec['seconds']:.0f} s)", flush=True)
    return rec


def main(argv):
    ns = [int(a) for a in argv] or [128, 256]
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["_about"] = ("oracle/etc_oracle.py alg:pcg at rtol 1e-9 (midpoint reference parameters, p0 = 0) on the "
                      "tab:smooth problem of tests/problems.py; L2 error against the exact solution at cell centres")
    for n in ns:
        data[str(n)] = run(n)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:])
