"""K_eff of the named workloads against the oracle's, stored in
``tests/golden/oracle_keff.json`` by ``tests/golden/make_oracle_keff.py``
(which calls only the CPU oracle and the seeded generators).

Per workload the golden file holds the oracle's alg:pcg stopped at rtol 1e-6
(midpoint reference parameters, p0 = 0: the GPU's own schedule) and the same
iteration continued to relres 1e-10 (the solution of A p = b).  On the GPU,
in the launch configuration the benchmark times:

* float64 form at rtol 1e-6 against the oracle run to the same rtol with the
  same reference parameters and start: pass count within one, K within
  1e-8 relative where the oracle stops within 100 passes (measured: at most
  4e-12 on the 512^3 sphere RVEs, 1e-13 on the spheroids), 1e-6 beyond:
  over 140 or more passes of a contrast-1e3 field, rounding differences
  between the FFT-based transforms and the oracle's O(N^2) definitions move
  the stopping iterate by up to a few 1e-7 (3e-7 on the 48^3 ensemble RVE);
* float64 and mixed forms at rtol 1e-6 against the oracle's solution of
  A p = b: K within 1e-5 relative (the scope's target bar).  Stopping at
  relres 1e-6 itself leaves up to a few 1e-6 in K: the oracle's own rtol-1e-6
  iterate misses its solution by 3.8e-6 on the 128^3 spheroids (load y),
  so 1e-6 against the solution is not a bar the method reaches at this rtol.

Each test first checks that the regenerated conductivity has the SHA-256
recorded with the golden values.
"""

import hashlib
import json
import os

import numpy as np
import pytest

import rvegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

etc = pytest.importorskip("paper_2404_02433_amd")
GOLD_PATH = os.path.join(os.path.dirname(__file__), "golden", "oracle_keff.json")
with open(GOLD_PATH) as f:
    GOLD = {k: v for k, v in json.load(f).items() if not k.startswith("_")}


def regenerate(name, rve_inputs):
    rec = GOLD[name]
    if name.startswith("ensemble"):
        s = rec["info"]
        kap = rvegen.grf_lognormal(s["n"], s["sigma2"], s["ell"], s["seed"], 1e3, np.float32)
    else:
        kap, _ = rve_inputs(name.rsplit("_", 1)[0] if name.startswith("spheroids128_") else name)
    assert hashlib.sha256(np.ascontiguousarray(kap).tobytes()).hexdigest() == rec["sha256"], name
    return kap


def run(kap, axis, precision):
    x = torch.as_tensor(kap, device="cuda:0")
    out = etc.solve(x, axis, precision=precision, rtol=1e-6)
    del x
    return out


@pytest.mark.parametrize("name", sorted(GOLD))
def test_keff_matches_oracle(name, rve_inputs):
    rec = GOLD[name]
    print(f"golden {name}: generating {rec['shape']} {rec['dtype']}", flush=True)
    kap = regenerate(name, rve_inputs)
    axis = rec["axis"]
    traj, truth = rec["traj"], rec["truth"]
    f64 = run(kap, axis, "fp64")
    print(f"golden {name}: fp64 K={f64['keff']:.12g} iters={f64['iters']} oracle traj K={traj['keff']:.12g} "
          f"iters={traj['iters']} truth K={truth['keff']:.12g}", flush=True)
    assert f64["status"] == "ok"
    assert np.allclose(f64["kref"], rec["kref"], rtol=1e-12, atol=0.0)
    print(f"golden {name}: fp64 rel diff vs oracle traj {abs(f64['keff'] - traj['keff']) / traj['keff']:.2e}, "
          f"vs solution {abs(f64['keff'] - truth['keff']) / truth['keff']:.2e}", flush=True)
    assert abs(f64["iters"] - traj["iters"]) <= 1
    bar = 1e-8 if traj["iters"] <= 100 else 1e-6
    assert abs(f64["keff"] - traj["keff"]) <= bar * traj["keff"]
    assert abs(f64["keff"] - truth["keff"]) <= 1e-5 * truth["keff"]
    mixed = run(kap, axis, "mixed")
    print(f"golden {name}: mixed K={mixed['keff']:.12g} iters={mixed['iters']} "
          f"rel diff vs oracle traj {abs(mixed['keff'] - traj['keff']) / traj['keff']:.2e}, "
          f"vs solution {abs(mixed['keff'] - truth['keff']) / truth['keff']:.2e}", flush=True)
    assert mixed["status"] == "ok"
    assert abs(mixed["keff"] - traj["keff"]) <= 1e-5 * traj["keff"]
    assert abs(mixed["keff"] - truth["keff"]) <= 1e-5 * truth["keff"]


def test_spheres32_to_rtol_1e10_matches_oracle_solution(rve_inputs):
    """The 32^3 sphere RVE as its workload states it: one float64 solve to
    relres 1e-10, K_xx within 1e-9 of the oracle's solution."""
    kap = regenerate("spheres32", rve_inputs)
    out = etc.solve(torch.as_tensor(kap, device="cuda:0"), 0, rtol=1e-10)
    truth = GOLD["spheres32"]["truth"]["keff"]
    assert out["status"] == "ok"
    assert abs(out["keff"] - truth) <= 1e-9 * truth, (out["keff"], truth)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("mixed", 1e-5)])
def test_mixed_size_ensemble_matches_oracle(precision, tol, rve_inputs):
    """The ensemble RVEs of every edge (48 ... 160, float32 log-normal
    fields) solved together as one ensemble call: each K within the form's
    bar (1e-6 float64, 1e-5 mixed) of the oracle's rtol-1e-6 run, and within
    1e-5 of the oracle's solution."""
    names = sorted((n for n in GOLD if n.startswith("ensemble")), key=lambda n: GOLD[n]["shape"][0])
    if not names:
        pytest.skip("no ensemble goldens")
    kaps = [torch.as_tensor(regenerate(n, rve_inputs), device="cuda:0") for n in names]
    out = etc.solve_ensemble(kaps, 0, precision=precision, rtol=1e-6)
    for i, n in enumerate(names):
        traj, truth = GOLD[n]["traj"]["keff"], GOLD[n]["truth"]["keff"]
        print(f"ensemble {precision} {n}: K={out['keff'][i]:.12g} iters={out['iters'][i]} "
              f"rel vs traj {abs(out['keff'][i] - traj) / traj:.2e} vs solution {abs(out['keff'][i] - truth) / truth:.2e}",
              flush=True)
        assert out["status"][i] == "ok"
        assert abs(out["keff"][i] - traj) <= tol * traj, n
        assert abs(out["keff"][i] - truth) <= 1e-5 * truth, n
