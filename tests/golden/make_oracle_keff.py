"""Write oracle K_eff values of the named workloads to ``oracle_keff.json``.

Calls only the CPU oracle (``oracle.etc_oracle``) and the seeded input
generators (``rvegen``).  For every workload it records two solves of the
same problem:

* ``traj``: the PCG of alg:pcg exactly as the GPU library runs it (midpoint
  reference parameters, p0 = 0, exit test eq:exit on the recursive residual)
  stopped at rtol 1e-6 -- K_out, K_in, K_energy, passes, last relres and the
  reference parameters;
* ``truth``: the same PCG continued from the trajectory's end point (warm
  start) down to ||b - A p|| / ||b|| <= 1e-10 -- K_out, K_in, K_energy of
  the solution of A p = b to that residual.

Each record also stores the input's shape, dtype, generator parameters and a
SHA-256 of the conductivity bytes, so that a test can check that it
regenerated the same array.  For the workloads in GRAD_SAMPLES it also stores
the oracle's gradient dK_out/dkappa (energy form at the truth solution) at 64
seeded voxels (user layout).

Usage:  python tests/golden/make_oracle_keff.py [name ...]
        (no names: every workload; existing records of other names are kept)
"""

from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import rvegen  # noqa: E402
from oracle import etc_oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_keff.json")
RTOL_TRAJ = 1e-6
RTOL_TRUTH = 1e-10
ENSEMBLE_EDGES = (48, 64, 96, 128, 160)
GRAD_SAMPLES = {"grf256": 33}   # workload -> seed of the sampled voxels


def kappa_sha256(kap: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(kap).tobytes()).hexdigest()


def ensemble_pick(edge: int) -> dict:
    """The first RVE of the 64-RVE log-normal ensemble (meta-seed 5) whose edge is ``edge``."""
    for s in rvegen.grf_ensemble_specs():
        if s["n"] == edge:
            return s
    raise KeyError(edge)


def workloads() -> dict:
    """name -> (builder returning (kappa, info), load axis)."""
    w = {}

    def cfg(name):
        return lambda: rvegen.make_config(name)

    w["spheres32"] = (cfg("spheres32"), 0)
    for axis, lab in enumerate("xyz"):
        w[f"spheroids128_{lab}"] = (cfg("spheroids128"), axis)
    w["grf256"] = (cfg("grf256"), 0)
    for e in ENSEMBLE_EDGES:
        def ens(e=e):
            s = ensemble_pick(e)
            kap = rvegen.grf_lognormal(s["n"], s["sigma2"], s["ell"], s["seed"], 1e3, np.float32)
            return kap, dict(s)
        w[f"ensemble{e}"] = (ens, 0)
    w["spheres512"] = (cfg("spheres512"), 0)
    w["spheres512_2000"] = (cfg("spheres512_2000"), 0)
    return w


def keff_record(pb, res, t0):
    k = O.keff(pb, res.p)
    return {"keff": k["out"], "k_in": k["in"], "k_energy": k["energy"], "iters": res.iters,
            "relres": res.relres, "status": res.status, "seconds": time.time() - t0}


def run(name: str, build, axis: int) -> dict:
    t0 = time.time()
    kap, info = build()
    rec = {"shape": list(kap.shape), "dtype": str(kap.dtype), "axis": axis, "info": info,
           "sha256": kappa_sha256(kap), "generate_seconds": time.time() - t0,
           "blas_threads": os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", "default"))}
    pb = O.make_problem(np.asarray(kap, dtype=np.float64), axis)
    kref = O.kref_mid(pb)
    rec["kref"] = [kref[f] for f in O.FAMILIES]
    t1 = time.time()
    traj = O.pcg(pb, rtol=RTOL_TRAJ, max_iter=5000, kref=kref)
    rec["traj"] = keff_record(pb, traj, t1)
    rec["traj"]["rtol"] = RTOL_TRAJ
    rec["traj"]["history"] = traj.history[:13]
    print(f"{name}: traj K={rec['traj']['keff']:.12g} iters={traj.iters} "
          f"({rec['traj']['seconds']:.1f} s)", flush=True)
    t2 = time.time()
    truth = O.pcg(pb, rtol=RTOL_TRUTH, max_iter=5000, kref=kref, p0=traj.p)
    # the residual of the warm start is recomputed as b - A p, so relres is the true one
    rec["truth"] = keff_record(pb, truth, t2)
    rec["truth"]["rtol"] = RTOL_TRUTH
    rec["truth"]["iters_after_traj"] = truth.iters
    print(f"{name}: truth K={rec['truth']['keff']:.12g} extra iters={truth.iters} "
          f"({rec['truth']['seconds']:.1f} s)", flush=True)
    if name in GRAD_SAMPLES:
        rng = np.random.default_rng(GRAD_SAMPLES[name])
        idx = np.stack([rng.integers(0, s, 64) for s in kap.shape], axis=1)
        g = O.decanonical(O.keff_gradient(pb, truth.p), axis)
        rec["grad_samples"] = {"seed": GRAD_SAMPLES[name], "idx": idx.tolist(),
                               "values": [float(g[tuple(i)]) for i in idx], "max_abs": float(np.abs(g).max())}
    return rec


def main(argv):
    table = workloads()
    names = argv or list(table)
    for n in names:
        if n not in table:
            raise SystemExit(f"unknown workload {n}; known: {', '.join(table)}")
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data.setdefault("_about", {
        "oracle": "oracle/etc_oracle.py (float64 NumPy), midpoint reference parameters, p0 = 0",
        "traj": f"alg:pcg stopped at recursive relres <= {RTOL_TRAJ}",
        "truth": f"warm-started from traj, stopped at relres <= {RTOL_TRUTH}",
    })
    for n in names:
        build, axis = table[n]
        data[n] = run(n, build, axis)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:])
