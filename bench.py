"""Benchmark: time-to-solve of a 512^3 two-phase RVE to relative residual 1e-6,
mixed form vs float64 form, on one MI355X.

A step is one whole solve with the conductivity already resident in HBM:
etc_setup (canonical copy, extrema, reference medium, tables) + etc_solve
(PCG to rtol) + etc_keff.  Prints one JSON line (rank 0, N = 1).

Workload ("spheres512"): 512^3 voxels, non-overlapping spheres of radius 10
voxels added by random sequential addition (seed 4) until the voxel volume
fraction reaches 0.26 (8660 spheres), kappa 1 in the matrix and 100 in the
spheres, load along x, Dirichlet 1 / 0.

Extra fields: the float64 form's time, both K_eff values and iteration
counts, the achieved HBM rate of the whole solve (algorithmic bytes / time),
the roofline record of the dominant kernel (HIP-event timing around its
launches inside the timed region), a per-kernel census of all six hot
kernels per form (one extra solve per kernel after the timed region, HIP
events around that kernel's launches), the literal 2000-sphere 512^3
workload timed the same way, the mixed-size GRF ensemble (64 RVEs in one
ensemble plan: RVEs/s, passes/s, HBM rate), and the CPU oracle's time on a bounded sample
of the same workload (with the CPU model, the BLAS threads the oracle uses
and the recorded time of one whole oracle solve).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-solve 512^3 RVE at rel.res 1e-6 (mixed vs FP64); achieved HBM GB/s"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per voxel and launch of each hot kernel (reads +
# writes of the arrays it must touch), by storage precision.
#   1 operator:             w, kappa -> q                       3 vectors
#   2 residual + DCT_b:     r, q -> r, t                        4 vectors
#   3 DCT_a forward:        t -> t                              2 vectors
#   4 tridiagonal:          t -> t                              2 vectors
#   5 DCT_a backward:       t -> t                              2 vectors
#   6 DCT_b^-1, solution and direction:
#                           t, w, x -> w, x                     5 vectors (x = p in FP64,
#                                                              the float32 increment in mixed)
KERNEL_NAMES = {1: "k_apply_A_iso", 2: "k_rows_fwd (residual update + DCT_b)", 3: "k_cols (DCT_a forward)",
                4: "k_thomas", 5: "k_cols (DCT_a backward)", 6: "k_rows_inv (DCT_b^-1 + solution + direction)"}


def bytes_per_voxel(kernel: int, es: int) -> int:
    return {1: 3 * es, 2: 4 * es, 3: 2 * es, 4: 2 * es, 5: 2 * es, 6: 5 * es}[kernel]


def iteration_bytes_per_voxel(es: int, mixed: bool, refine_every: int) -> float:
    b = sum(bytes_per_voxel(k, es) for k in range(1, 7))
    if mixed and refine_every > 0:
        # flush (p double r/w, increment r/w, w read), true residual (p,
        # kappa, r), redo of DCT_b (r -> t), every refine_every passes
        b += (16 + 3 * es + 8 + 2 * es + 2 * es) / refine_every
    return b


def code_tokens(src: str) -> str:
    """C++ source without its comments and with runs of white space folded to
    one blank (string and character literals kept as they are), so that a
    change of comments or layout alone leaves the hash of the kernels as it
    was."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash() -> str:
    """Hash of the kernel and library sources (code only, see code_tokens)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2404_02433_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update(name.encode())
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: int, workload: str, precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash():
        return None
    k = rec.get("kernels", {}).get(str(kernel))
    return None if k is None else k.get("bytes_per_launch")


def run_solve(etc, kap, precision, rtol, timer_kernel=0, autotune=False):
    plan = etc.etc_setup(kap, 0, 1.0, 0.0, precision=precision, rtol=rtol, autotune=autotune)
    if timer_kernel:
        etc.etc_set_kernel_timer(plan, timer_kernel)
    out = etc.etc_solve(plan)
    out.update(etc.etc_keff(plan))
    if timer_kernel:
        out["kernel_ms"], out["kernel_launches"] = etc.etc_kernel_time(plan)
    plan.close()
    return out


def time_form(torch, etc, kap, precision, rtol, steps, warmup, timer_kernel, autotune=False):
    for _ in range(warmup):
        run_solve(etc, kap, precision, rtol, autotune=autotune)
    torch.cuda.synchronize()
    outs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        outs.append(run_solve(etc, kap, precision, rtol, timer_kernel, autotune))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, outs


def cpu_baseline(kap_np, iters_full: int, slab: int = 128, sample_iters: int = 2):
    """Oracle (float64 NumPy) on the host cores, on a bounded sample: the first
    `slab` load planes of the same RVE (all 512 x 512 transverse voxels).  Its
    setup and PCG passes are timed and scaled to the full workload: every
    oracle step (per-plane DCTs, per-line tridiagonal sweeps, stencil, vector
    updates) costs in proportion to the number of load planes."""
    from oracle import etc_oracle as O

    nL = kap_np.shape[0]
    sub = kap_np[:slab]
    t0 = time.perf_counter()
    pb = O.make_problem(sub, 0)
    kref = O.kref_mid(pb)
    t_setup = time.perf_counter() - t0
    t1 = time.perf_counter()
    res = O.pcg(pb, rtol=1e-30, max_iter=sample_iters, kref=kref)
    t_pcg = time.perf_counter() - t1
    per_pass = t_pcg / (res.iters + 1)   # initial preconditioner pass + sample passes
    scale = nL / sub.shape[0]
    est = scale * (t_setup + per_pass * (iters_full + 1))
    blas = blas_threads()
    out = {"value": est, "unit": "s", "cores": blas, "kind": "oracle",
           "sample": f"first {sub.shape[0]} of {nL} load planes of the same RVE: oracle setup + initial pass + "
                     f"{res.iters} PCG passes timed ({t_setup + t_pcg:.1f} s), scaled by {scale:g} (plane count) "
                     f"and to {iters_full} passes",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "threads_note": f"the oracle's DCTs (matrix products) use {blas} BLAS threads; its stencil, "
                           "tridiagonal sweeps and vector updates run on one thread"}
    full = measured_full_oracle_solve()
    if full:
        out["measured_full_solve"] = full
    return out


def blas_threads() -> int:
    """Threads of NumPy's BLAS (the only multi-threaded part of the oracle)."""
    try:
        import numpy as np
        from threadpoolctl import threadpool_info

        np.ones((2, 2)) @ np.ones((2, 2))
        n = [i["num_threads"] for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(n[0])
    except Exception:
        pass
    return int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", 1)))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_full_oracle_solve():
    """The whole 512^3 oracle solve (alg:pcg to rtol 1e-6, 55 passes) as
    recorded with the stored oracle K_eff values (a separate CPU run, not this
    host), for context beside the sampled estimate."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_keff.json")
    try:
        with open(path) as f:
            rec = json.load(f).get("spheres512")
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    return {"seconds": rec["traj"]["seconds"], "passes": rec["traj"]["iters"],
            "blas_threads": rec.get("blas_threads"), "where": "build container CPU (recorded in tests/golden/oracle_keff.json)"}


def _grf_one(spec):
    import numpy as np
    import rvegen

    return rvegen.grf_lognormal(spec["n"], spec["sigma2"], spec["ell"], spec["seed"], 1e3, np.float32)


def grf_ensemble_parallel(rvegen, count, workers=8):
    """The seeded GRF ensemble, each RVE generated in a worker process (the
    same arrays as rvegen.grf_ensemble, which builds them one after another).
    Called before anything touches the GPU, so the workers are forked from a
    process without device state."""
    from concurrent.futures import ProcessPoolExecutor

    print(f"bench: generating the GRF ensemble ({count} RVEs)", file=sys.stderr, flush=True)
    specs = rvegen.grf_ensemble_specs(count)
    workers = max(1, min(workers, (os.cpu_count() or 1) // 2))
    if workers == 1:
        return [_grf_one(sp) for sp in specs], specs
    with ProcessPoolExecutor(max_workers=workers) as ex:
        kaps = list(ex.map(_grf_one, specs))
    return kaps, specs


def ensemble_record(torch, etc, rvegen, args, ens, form, mode="launch", graph=False):
    """Ensemble of `count` log-normal GRF RVEs of mixed edges {48, 64, 96, 128,
    160} (per-RVE variance U[0.5, 2], correlation length U[4, 16], contrast
    <= 1e3, float32 input), load x, rtol 1e-6.  A step solves every RVE and
    reads back every K_eff; mode "launch" is one ensemble plan (every kernel
    of a pass one launch for all RVEs), "plans" the per-shape batch plans on
    concurrent streams."""
    kaps_np, specs = ens
    kaps = [torch.as_tensor(k, device="cuda:0") for k in kaps_np]
    V = sum(k.size for k in kaps_np)
    kw = dict(precision=form, rtol=args.rtol, use_graph=graph, mode=mode)
    if mode == "plans":
        kw.update(concurrent=not args.serial, max_batch_voxels=args.batch_voxels)
    print(f"bench: timing the ensemble ({form}, {mode})", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        etc.solve_ensemble(kaps, 0, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = etc.solve_ensemble(kaps, 0, **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    es = 4 if form == "mixed" else 8
    it_bytes = sum(iteration_bytes_per_voxel(es, form == "mixed", 20) * k.size * it
                   for k, it in zip(kaps_np, out["iters"]))
    gbs = it_bytes / dt / 1e9
    del kaps
    return {
        "workload": f"grf_ensemble: {len(kaps_np)} log-normal GRF RVEs, edges 48/64/96/128/160, "
                    f"{V / 1e6:.1f} M voxels in total, load x, rtol {args.rtol:g}",
        "form": form, "mode": mode, "graph": bool(graph),
        "rves_per_s": len(kaps_np) / dt, "s_per_ensemble": dt,
        "passes_per_s": sum(out["iters"]) / dt, "iters_min_max": [min(out["iters"]), max(out["iters"])],
        "all_ok": all(st == "ok" for st in out["status"]), "plans": out["plans"],
        "hbm_gbs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
    }


def ensemble_bench(torch, etc, rvegen, args):
    """Ensemble benchmark alone (RVEs/s as the metric)."""
    form = args.forms.split(",")[0]
    ens = grf_ensemble_parallel(rvegen, args.ensemble, args.gen_workers)
    rec = ensemble_record(torch, etc, rvegen, args, ens, form, args.ensemble_mode, args.graph)
    line = {
        "metric": "RVE ensemble throughput (64 mixed-size GRF RVEs to rel.res 1e-6)",
        "value": rec["rves_per_s"], "unit": "RVEs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": rec["s_per_ensemble"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage / f64 dots+tridiagonal+refinement" if form == "mixed" else "f64",
        "data": "synthetic", "config": {"workload": rec["workload"], "form": form, "mode": rec["mode"],
                                        "graph": rec["graph"]},
        "ensemble": rec,
    }
    print(json.dumps(line), flush=True)


def leg_2000(torch, etc, rvegen, args, forms):
    """The literal 2000-sphere 512^3 workload (r = 10, vf ~0.062), timed like
    the headline workload (same steps and warm-up, per form)."""
    print("bench: generating spheres512_2000", file=sys.stderr, flush=True)
    kap_np, info = rvegen.make_config("spheres512_2000")
    kap = torch.as_tensor(kap_np, device="cuda:0")
    out = {"workload": f"512^3 two-phase RVE, {info['spheres']} non-overlapping spheres r=10 (vf={info['vf']:.4f}), "
                       f"kappa 1/100, load x, rtol {args.rtol:g}"}
    for form in forms:
        print(f"bench: timing {form} (2000 spheres)", file=sys.stderr, flush=True)
        dt, outs = time_form(torch, etc, kap, form, args.rtol, args.steps, args.warmup, 0, args.autotune)
        o = outs[-1]
        out[form] = {"time_s": dt, "iters": o["iters"], "keff": o["keff"], "relres": o["relres"], "status": o["status"]}
    del kap
    return out


def copy_rate(torch, etc, mib: int = 1024, reps: int = 10) -> float:
    """HBM rate of a plain streaming copy (read + write bytes / time), the
    practical ceiling that the hot kernels are also compared with."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    best = 0.0
    # the library's grid-stride copy kernel and the runtime's device copy
    for fn in (lambda: etc.etc_copy_f64(src, dst), lambda: dst.copy_(src)):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        best = max(best, 2.0 * n * 8 / (ms * 1e-3) / 1e9)
    del src, dst
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="grid edge (default: the 512^3 workload)")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--kernel", type=int, default=6, help="hot kernel timed with HIP events (1-6)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-census", action="store_true", help="skip the per-kernel timing solves")
    ap.add_argument("--no-2000", action="store_true", help="skip the 2000-sphere workload leg")
    ap.add_argument("--forms", default="mixed,fp64")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run the plain copy kernel on MIB MiB (5 launches) and exit; the byte counters "
                         "of this run calibrate FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--ensemble", type=int, default=0, metavar="COUNT",
                    help="time the mixed-size GRF ensemble of COUNT RVEs instead (RVEs/s)")
    ap.add_argument("--graph", action="store_true", help="replay the PCG passes from captured HIP graphs")
    ap.add_argument("--serial", action="store_true", help="ensemble: run the batch plans one after another")
    ap.add_argument("--ensemble-mode", default="launch", choices=["launch", "plans"],
                    help="ensemble: one plan with multi-group launches, or per-shape batch plans")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the ensemble record of the default run")
    ap.add_argument("--gen-workers", type=int, default=8,
                    help="processes generating the ensemble's fields (1: in this process, e.g. under a profiler)")
    ap.add_argument("--autotune", action="store_true",
                    help="plans tune their launch shapes at setup (the warm-up solve pays for the tuning)")
    ap.add_argument("--batch-voxels", type=int, default=1 << 25, help="ensemble: voxel cap of one batch plan")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a design note"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2404_02433_amd as etc
    import rvegen

    # the ensemble's arrays are generated first, before any device work
    ens = grf_ensemble_parallel(rvegen, 64, args.gen_workers) if (not args.no_ensemble and not args.ensemble
                                                and not args.copy_calib) else None

    if args.copy_calib:
        n = args.copy_calib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            etc.etc_copy_f64(src, dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read": n * 8, "copy_calib_bytes_written": n * 8, "launches": 5}))
        return
    if args.ensemble:
        ensemble_bench(torch, etc, rvegen, args)
        return

    print(f"bench: generating spheres512 at n={args.n}", file=sys.stderr, flush=True)
    kap_np, info = rvegen.make_config("spheres512", args.n)
    kap = torch.as_tensor(kap_np, device="cuda:0")
    V = kap_np.size
    forms = args.forms.split(",")
    res = {}
    for form in forms:
        print(f"bench: timing {form}", file=sys.stderr, flush=True)
        dt, outs = time_form(torch, etc, kap, form, args.rtol, args.steps, args.warmup, args.kernel, args.autotune)
        o = outs[-1]
        es = 4 if form == "mixed" else 8
        it_bytes = iteration_bytes_per_voxel(es, form == "mixed", 20) * V
        kms = sum(x["kernel_ms"] for x in outs) / max(1, sum(x["kernel_launches"] for x in outs))
        res[form] = {"time_s": dt, "iters": o["iters"], "keff": o["keff"], "k_in": o["k_in"],
                     "relres": o["relres"], "status": o["status"],
                     "hbm_gbs": it_bytes * o["iters"] / dt / 1e9,
                     "kernel_avg_ms": kms}
        print(f"bench: {form} {dt:.4f} s/solve iters={o['iters']} keff={o['keff']:.8f}", file=sys.stderr, flush=True)

    # per-kernel census (outside the timed region): one solve per hot kernel
    # with HIP events around every launch of that kernel
    copy_gbs = copy_rate(torch, etc)
    if not args.no_census:
        for form in forms:
            print(f"bench: kernel census {form}", file=sys.stderr, flush=True)
            es = 4 if form == "mixed" else 8
            census = {}
            for kid in range(1, 7):
                o = run_solve(etc, kap, form, args.rtol, kid, args.autotune)
                ms = o["kernel_ms"] / max(1, o["kernel_launches"])
                bpl = bytes_per_voxel(kid, es) * V
                gbs = bpl / (ms * 1e-3) / 1e9
                census[KERNEL_NAMES[kid]] = {"avg_launch_ms": ms, "launches": o["kernel_launches"],
                                             "algorithmic_bytes_per_launch": bpl, "achieved_gbs": gbs,
                                             "frac_of_peak": gbs / HBM_PEAK_GBS, "frac_of_copy": gbs / copy_gbs,
                                             "traffic": measured_traffic(kid, "spheres512", form)}
            res[form]["kernels"] = census

    head = "mixed" if "mixed" in res else forms[0]
    es = 4 if head == "mixed" else 8
    kid = args.kernel
    bpl = bytes_per_voxel(kid, es) * V
    kms = res[head]["kernel_avg_ms"]
    achieved = bpl / (kms * 1e-3) / 1e9 if kms > 0 else None
    traffic = measured_traffic(kid, "spheres512", head)
    roof = {"bound": "hbm", "kernel": KERNEL_NAMES[kid], "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "algorithmic_bytes_per_launch": bpl, "avg_launch_ms": kms,
            "copy_gbs": copy_gbs, "frac_of_copy": (achieved / copy_gbs) if achieved else None}
    line = {
        "metric": METRIC,
        "value": res[head]["time_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res[head]["time_s"] * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage / f64 dots+tridiagonal+refinement" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"spheres512: {args.n}^3 two-phase RVE, r=10 non-overlapping spheres to "
                               f"vf>={0.26} ({info['spheres']} spheres, vf={info['vf']:.4f}), kappa 1/100, "
                               f"load x, rtol {args.rtol:g}", "form": head, "autotune": bool(args.autotune)},
        "forms": res,
        "keff_mixed_vs_fp64": (abs(res["mixed"]["keff"] - res["fp64"]["keff"]) / res["fp64"]["keff"]
                               if "mixed" in res and "fp64" in res else None),
        "hbm_gbs": res[head]["hbm_gbs"],
        "roofline": roof,
    }
    if not args.no_2000 and args.n == 512:
        line["spheres512_2000"] = leg_2000(torch, etc, rvegen, args, forms)
    if ens is not None:
        # both ensemble forms: per-shape batch plans on concurrent streams and
        # one plan whose every kernel of a pass is one launch for all RVEs
        rec = ensemble_record(torch, etc, rvegen, args, ens, "mixed", "plans")
        one = ensemble_record(torch, etc, rvegen, args, ens, "mixed", "launch")
        rec["one_launch"] = {k: one[k] for k in ("rves_per_s", "s_per_ensemble", "iters_min_max", "all_ok", "plans")}
        line["ensemble"] = rec
        del ens
    if not args.no_cpu:
        print("bench: cpu oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(kap_np, res[head]["iters"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
