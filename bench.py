"""Benchmark: MAP solves/s at 512^2 (joint E/B shear) to 1e-6 relative gradient on one MI355X.

One step is one pass of the whole hot path over one batch: simulate the quadratic
estimator's maps on the device (fiducial and band-boosted simulations, Philox draws),
solve all of them together with the data map as ONE batched L-BFGS solve (127 MAP
solves: 1 data + 6 simulations x (1 + 20 bands)), reduce the band statistics E_l and
form the noise bias, Fisher matrix and Newton step (bandpower_qe).  `value` is MAP
solves per second of that step, inputs resident in HBM.

Also reported: the same 127 solves through the plain path (one map at a time, host
check after every iteration, no graph), the batched solve alone, the roofline of the
dominant kernel (HIP events around every launch of one instrumented step; bytes are
the kernels' algorithmic bytes counted on the device), the FP64 oracle on the host
(cpu_baseline, solves of the same data map and simulations), and one line per other
workload ("secondary": 256^2 density band powers, 512^2 density maps, 1024^2 CMB maps,
the 96-map uneven batch against its plain path, the 512^2 shear catalog at the catalog level).

    python bench.py [--steps K] [--warmup W] [--nsim 6] [--n 512] [--no-cpu] [--no-plain]
                    [--no-secondary] [--catalog-only] [--density-bands-only] [--cmb-full] [--cmb-iterate]
    python bench.py --pmc-summary FETCH_CSV WRITE_CSV   # profiles/pmc_traffic.json from rocprofv3 --pmc
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MAP solves/sec at 512² to 1e-6 rel. grad, batched vs plain; % HBM roofline"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--nsim", type=int, default=6)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--m", type=int, default=10)
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-solves", type=int, default=0, help="plain-path solves to time (0 = all)")
    ap.add_argument("--no-secondary", action="store_true", help="skip the other workloads' lines")
    ap.add_argument("--lbfgs-only", action="store_true",
                    help="skip the conjugate-gradient comparison (for counter runs: only L-BFGS launches of the chain)")
    ap.add_argument("--catalog-only", action="store_true",
                    help="print only the 512^2 shear catalog line (for profiling the catalog solve)")
    ap.add_argument("--density-bands-only", action="store_true",
                    help="print only the 256^2 density band-power line (for profiling that estimate)")
    ap.add_argument("--cmb-iterate", action="store_true",
                    help="only the 1024^2 CMB estimate (64 simulations) before and after one fiducial step")
    ap.add_argument("--cmb-full", action="store_true",
                    help="only the 1024^2 CMB band-power estimate at 256 simulations (10497 solves), one JSON line")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="write profiles/pmc_traffic.json from two rocprofv3 --pmc counter files of this benchmark")
    ap.add_argument("--cpu-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-out", default="", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-cores", type=int, default=1, help=argparse.SUPPRESS)
    return ap.parse_args()


# translation unit each profiled kernel is compiled in (the PMC record is keyed to its sources)
KERNEL_UNITS = {"k_passB": "wf_solver_k.hip", "k_passA": "wf_solver_k.hip", "k_cg_pass": "wf_solver_k.hip",
                "k_cg_dir": "wf_solver_k.hip", "k_stream_copy": "wf_solver_k.hip",
                "k_colinv": "wf_chain_f32l.hip", "k_colinvr": "wf_chain_f32l.hip", "k_row": "wf_chain_f32l.hip",
                "k_rowr": "wf_chain_f32l.hip", "k_colfwd": "wf_chain_f32l.hip", "k_colfwdr": "wf_chain_f32l.hip"}


def source_closure(unit: str):
    """(files, sha1) of a kernel translation unit and every local header it includes."""
    import hashlib
    import re
    dirs = [os.path.join(ROOT, "paper_1810_00503_amd", "csrc"), os.path.join(ROOT, "include")]
    seen, todo = [], [unit]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        path = next((os.path.join(d, f) for d in dirs if os.path.exists(os.path.join(d, f))), None)
        if path is None:
            continue
        seen.append(f)
        for line in open(path):
            m = re.match(r'\s*#include\s+"([^"]+)"', line)
            if m:
                todo.append(m.group(1))
    h = hashlib.sha1()
    for f in sorted(seen):
        path = next(os.path.join(d, f) for d in dirs if os.path.exists(os.path.join(d, f)))
        h.update(f.encode() + b"\0" + open(path, "rb").read())
    return sorted(seen), h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC record
    (profiles/pmc_traffic.json), or None if the sources the kernel is compiled from changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    k = json.load(open(path)).get("kernels", {}).get("k_" + kernel)
    if k is None or "unit" not in k or source_closure(k["unit"])[1] != k.get("sources_sha1"):
        return None
    return k["traffic_bytes_per_launch"]


def pmc_summary(fetch_csv: str, write_csv: str, copy_bytes: int = 2 * 1024 ** 3):
    """Per-dispatch HBM bytes from two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch), calibrated by the library's streaming copy of copy_bytes that
    the benchmark runs (k_stream_copy reads and writes copy_bytes).  Writes
    profiles/pmc_traffic.json and prints a markdown table."""
    import csv
    from collections import defaultdict

    def load(path, counter):
        acc = defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            acc[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]) * 1024.0)
        return acc

    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")

    def short(name):
        b = name.split("(")[0].replace("void ", "").strip()
        return b.split("::")[-1].split("<")[0]

    cf = [v for (k, g), vs in fetch.items() if short(k) == "k_stream_copy" for v in vs]
    cw = [v for (k, g), vs in write.items() if short(k) == "k_stream_copy" for v in vs]
    if not cf or not cw:
        raise SystemExit("pmc-summary: no k_stream_copy dispatches in the counter files")
    ff = copy_bytes / (sum(cf) / len(cf))
    wf_ = copy_bytes / (sum(cw) / len(cw))
    rows = []
    for key in fetch:
        if key not in write:
            continue
        f = sum(fetch[key]) / len(fetch[key])
        w = sum(write[key]) / len(write[key])
        rows.append((key[0], key[1], len(fetch[key]), f, w, ff * f + wf_ * w))
    rows.sort(key=lambda r: -r[2] * r[5])
    kernels = {}
    for name, grid, disp, f, w, t in rows:
        k = short(name)
        if k not in KERNEL_UNITS or k in kernels:
            continue   # the most-dispatched traffic of each kernel (the solver's own launches)
        files, sha = source_closure(KERNEL_UNITS[k])
        kernels[k] = {"name": name.split("(")[0].replace("void ", "").strip(), "grid": grid, "dispatches": disp,
                      "traffic_bytes_per_launch": t, "unit": KERNEL_UNITS[k], "sources": files,
                      "sources_sha1": sha}
    rec = {"fetch_factor": ff, "write_factor": wf_, "copy_bytes": copy_bytes, "kernels": kernels}
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    mib = 1024.0 ** 2
    print(f"calibration: k_stream_copy of {copy_bytes / mib:.0f} MiB reads FETCH_SIZE = "
          f"{copy_bytes / ff / mib:.1f} MiB and WRITE_SIZE = {copy_bytes / wf_ / mib:.1f} MiB: read bytes = "
          f"{ff:.3f} x FETCH_SIZE, written bytes = {wf_:.3f} x WRITE_SIZE")
    print("| kernel | grid | dispatches | FETCH_SIZE avg (MiB) | WRITE_SIZE avg (MiB) | calibrated traffic avg (MiB) |")
    print("|---|---:|---:|---:|---:|---:|")
    for name, grid, disp, f, w, t in rows[:20]:
        nm = name.split("(")[0].replace("void ", "").strip()
        print(f"| `{nm}` | {grid} | {disp} | {f / mib:.1f} | {w / mib:.1f} | {t / mib:.1f} |")


def host_cores() -> int:
    """Cores this process may use: its CPU affinity, capped by OMP_NUM_THREADS where the host
    sets it (a host that shares its cores among its GPUs limits each process that way)."""
    n = len(os.sched_getaffinity(0))
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, n)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, gpu_solve=None):
    """The oracle (float64 numpy, one thread per process) on the host: solves of the data map
    and fiducial simulations of the workload at the benchmark's tolerance, on every core this
    process may use (one independent solve per process, all started together) and on one core.
    The child also writes three maps with the oracle's MAP at 1e-10 (untimed);
    gpu_solve(maps, ref_fields) -> (fields, maps, stats, E, dtheta) solves the same data on the
    GPU at the benchmark's tolerance, and the accuracy beside the throughput is the GPU against
    that reference (field relative L2; per-pixel map error on observed and on masked pixels,
    relative to the largest reference pixel; E_l of the solved fields per band; the library's
    d chi^2 / d theta_b at the reference fields per band)."""
    import tempfile

    import numpy as np
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "ref.npz")
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", "--n", str(args.n), "--tol", str(args.tol),
               "--m", str(args.m), "--seed", str(args.seed), "--cpu-out", out, "--cpu-cores", str(host_cores())]
        r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=900)
        if r.returncode != 0:
            return {"error": r.stderr[-400:]}
        res = json.loads(r.stdout.strip().splitlines()[-1])
        if gpu_solve is not None and os.path.exists(out):
            ref = np.load(out)
            k = int(ref["count"])
            s, x, st, E, th = gpu_solve([ref[f"d{i}"] for i in range(k)], [ref[f"s{i}"] for i in range(k)])
            obs = ref["observed"]
            el2, eo, em, eE, et = [], [], [], [], []
            for i in range(k):
                sr, xr = ref[f"s{i}"], ref[f"x{i}"]
                el2.append(float(np.linalg.norm(s[i] - sr) / np.linalg.norm(sr)))
                dx = np.abs(x[i] - xr) / np.abs(xr).max()
                eo.append(float(dx[:, obs].max()))
                em.append(float(dx[:, ~obs].max()))
                Er, tr = ref[f"E{i}"], ref[f"t{i}"]
                nE, nt = np.abs(Er) > 0, np.abs(tr) > 0
                eE.append(float(np.max(np.abs(E[i] - Er)[nE] / np.abs(Er)[nE])))
                et.append(float(np.max(np.abs(th[i] - tr)[nt] / np.abs(tr)[nt])))
            res["accuracy"] = {"maps": k, "reference": "oracle float64 MAP to 1e-10 of the same data",
                               "field_rel_l2_max": max(el2), "map_max_abs_observed_rel": max(eo),
                               "map_max_abs_masked_rel": max(em),
                               "gpu_rel_grad_max": max(float(x_.rel_grad) for x_ in st),
                               # E_l of the GPU's MAP against E_l of the reference MAP, per band
                               "band_E_rel_max": max(eE),
                               # the library's d chi^2 / d theta_b against the oracle's, both at
                               # the reference MAP, per band
                               "dchi2_dtheta_rel_max": max(et)}
    return res


def _cpu_maps(args, idx):
    """Map idx of the CPU sample: 0 the data map, i > 0 fiducial simulation i - 1 (Philox)."""
    import oracle as O
    from paper_1810_00503_amd import workloads as WL
    wl = WL.shear_eb(args.n)
    S_true = O.prior_S(wl.pshape, wl.band, wl.theta_true)
    S = O.prior_S(wl.pshape, wl.band, wl.theta_fid)
    if idx == 0:
        d = O.simulate(O.philox.draws_for_sims(args.seed, [0], wl.n, wl.ncomp)[0], S_true, wl.W)
    else:
        d = O.simulate(O.philox.draws_for_sims(args.seed + 1, [idx - 1], wl.n, wl.ncomp)[0], S, wl.W)
    return wl, S, d


def _cpu_worker(args, idx, barrier, q):
    import oracle as O
    wl, S, d = _cpu_maps(args, idx)
    barrier.wait()
    t0 = time.perf_counter()
    r = O.lbfgs_solve(d, wl.W, S, m=args.m, tol=args.tol)
    q.put((idx, t0, time.perf_counter(), r["iters"]))


def cpu_child(args):
    import multiprocessing as mp

    import numpy as np

    import oracle as O
    # all cores: one independent solve per process, started together (fork: this process never
    # touches the GPU)
    P = max(1, args.cpu_cores)
    ctxm = mp.get_context("fork")
    barrier = ctxm.Barrier(P)
    q = ctxm.Queue()
    procs = [ctxm.Process(target=_cpu_worker, args=(args, i, barrier, q)) for i in range(P)]
    for p in procs:
        p.start()
    res = [q.get() for _ in range(P)]
    for p in procs:
        p.join()
    t_start = min(r[1] for r in res)
    t_end = max(r[2] for r in res)
    par = P / (t_end - t_start)
    # one core: the data map and the first two fiducial simulations one after another
    maps = [_cpu_maps(args, i) for i in range(3)]
    t0 = time.perf_counter()
    its = [O.lbfgs_solve(d, wl.W, S, m=args.m, tol=args.tol)["iters"] for wl, S, d in maps]
    dt = time.perf_counter() - t0
    if args.cpu_out:   # the reference for the accuracy line (untimed)
        wl = maps[0][0]
        ref = {"count": len(maps), "observed": wl.W > 0}
        for i, (wl, S, d) in enumerate(maps):
            sr = O.lbfgs_solve(d, wl.W, S, m=args.m, tol=1e-10, max_iter=50000)["s"]
            ref[f"d{i}"], ref[f"s{i}"], ref[f"x{i}"] = d, sr, O.forward(sr)
            # band powers of the reference MAP (eq. el) and d chi^2 / d theta_b at it
            ref[f"E{i}"] = O.band_E(sr, S, wl.band, wl.theta_fid, wl.nbands)
            ref[f"t{i}"] = O.dchi2_dtheta(sr, wl.pshape, wl.band, wl.theta_fid, wl.nbands)
        np.savez(args.cpu_out, **ref)
    print(json.dumps({"value": round(par, 4), "unit": "solves/s", "cores": P, "kind": "oracle",
                      "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                      "one_core_solves_per_s": round(len(maps) / dt, 4),
                      "sample": f"{P} independent {args.n}^2 E/B shear MAP solves (the data map and "
                                f"{P - 1} fiducial simulations) to {args.tol:g} rel. grad, float64 numpy, one "
                                f"process per core started together, {t_end - t_start:.1f} s wall, iterations "
                                f"{sorted(r[3] for r in res)}; one core: 3 of them in {dt:.1f} s "
                                f"(iterations {its})"}))


def secondary_workloads(args):
    """The other workloads, one timed call each after one untimed call (inputs resident):
    the 64^2 float64 density map alone and 1024 of them, 256^2 density band powers (128 simulations, 1665 solves per estimate; then with 5 of the
    12 Fisher rows simulated, and two steps of the fiducial iteration with those), the scalar
    512^2 density variant (127 maps), 1024^2 CMB maps (preconditioned, 16 maps) and the
    96-map uneven batch (preconditioned) against its plain one-map-at-a-time path."""
    import numpy as np
    import torch

    import paper_1810_00503_amd as wf
    from paper_1810_00503_amd import workloads as WL
    dev = "cuda:0"

    def base_of(wl):
        return wf.Problem(torch.tensor(wl.W, dtype=torch.float32, device=dev), wl.pshape, wl.band, wl.theta_fid)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    def solve_line(name, probs, opts):
        (_, _, st, _), dt = timed(lambda: wf.map_wf_solve(probs, opts))
        its = [x.iters for x in st]
        conv = sum(x.status == wf.WF_SOLVE_CONVERGED for x in st)
        return {"workload": name, "maps": len(probs), "solves_per_s": round(len(probs) / dt, 2),
                "iters_mean": round(float(np.mean(its)), 1), "iters_max": int(np.max(its)),
                "converged": f"{conv}/{len(probs)}"}

    out = {}
    # 64^2 projected density in float64 (m = 10, stop at 1e-8): one map alone (the map the tests
    # compare with the dense Wiener filter), and 1024 such maps (distinct noise realisations) in
    # one batched call with preallocated outputs
    wl = WL.density64()
    b64 = wf.Problem(torch.tensor(wl.W, dtype=torch.float64, device=dev), wl.pshape, wl.band, wl.theta_fid)
    d64 = wf.wf_simulate(b64, 1024, 1100, theta_true=wl.theta_true)
    o64 = wf.LbfgsOpts(m=10, rel_grad_tol=1e-8)
    one = [b64.with_data(d64[0])]
    (_, _, st1, _), dt1 = timed(lambda: wf.map_wf_solve(one, o64))
    many = [b64.with_data(d64[i]) for i in range(1024)]
    buf = [torch.empty((1, 64, 33), dtype=torch.complex128, device=dev) for _ in many]
    (_, _, stm, _), dtm = timed(lambda: wf.map_wf_solve(many, o64, out=buf))
    out["density64_f64"] = {"workload": "64^2 projected density, float64, L-BFGS m=10 to 1e-8 rel. grad",
                            "one_map_ms": round(dt1 * 1e3, 3), "one_map_iters": st1[0].iters,
                            "batch1024_solves_per_s": round(1024 / dtm, 1),
                            "batch1024_iters_mean": round(float(np.mean([x.iters for x in stm])), 1),
                            "batch1024_converged": f"{sum(x.status == wf.WF_SOLVE_CONVERGED for x in stm)}/1024"}
    del d64, many, buf
    # 256^2 density band powers: one estimate = data + 128 simulations x (1 + 12 bands)
    wl = WL.density_bands()
    base = base_of(wl)
    prob = base.with_data(wf.wf_simulate(base, 1, 2000, theta_true=wl.theta_true)[0])
    nsim = 128
    opts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol)
    (th_all, _, _, F_all, _), dt = timed(lambda: wf.bandpower_qe(prob, nsim, 2001, opts=opts))
    ns = 1 + nsim * (1 + wl.nbands)
    # the same estimate with the optional diagonal preconditioner (same stop test, same MAPs)
    opts_pc = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, precond=1)
    (th_pc, _, _, _, _), dt_pc = timed(lambda: wf.bandpower_qe(prob, nsim, 2001, opts=opts_pc))
    sd_all = np.sqrt(np.abs(np.diag(np.linalg.inv(F_all))))
    out["density256_bandpowers"] = {"workload": f"256^2 density, {wl.nbands} bands, {nsim} simulations "
                                                f"({ns} MAP solves per estimate)",
                                    "bandpower_estimates_per_s": round(1.0 / dt, 3),
                                    "solves_per_s": round(ns / dt, 1),
                                    "preconditioned_estimates_per_s": round(1.0 / dt_pc, 3),
                                    "preconditioned_theta_max_diff_over_sigma": round(
                                        float(np.max(np.abs(th_pc - th_all) / sd_all)), 5)}
    # the same estimate with a subset of the Fisher rows simulated (the rest interpolated
    # along the diagonals), and two steps of the fiducial iteration with it
    rows = [0, 3, 6, 9, 11]
    (th_r, _, _, _, F_r, _), dt_r = timed(lambda: wf.bandpower_iterate(prob, nsim, 2001, max_iter=1, rows=rows,
                                                                       opts=opts))
    (th_i, hist_i, _, _, _, _), dt_i = timed(lambda: wf.bandpower_iterate(prob, nsim, 2001, max_iter=2, rel_tol=0.0,
                                                                          rows=rows, opts=opts))
    ns_r = 1 + nsim * (1 + len(rows))
    sig = np.diag(F_all) > 1e-6 * np.diag(F_all).max()
    sd = np.sqrt(np.abs(np.diag(np.linalg.inv(F_all))))
    out["density256_sampled_rows"] = {
        "workload": f"256^2 density, {wl.nbands} bands, {nsim} simulations, Fisher rows {rows} simulated "
                    f"({ns_r} MAP solves per estimate)",
        "bandpower_estimates_per_s": round(1.0 / dt_r, 3), "solves_per_s": round(ns_r / dt_r, 1),
        "F_rel_frobenius_diff_vs_all_rows": round(float(np.linalg.norm(F_r - F_all) / np.linalg.norm(F_all)), 5),
        # Theta_hat differences in units of its statistical error sqrt((F^-1)_ll) from all rows, over
        # the bands carrying signal (F_ll above 1e-6 of the largest; the damping tail's are undetermined)
        "signal_bands": int(sig.sum()),
        "theta_max_diff_over_sigma_vs_all_rows": round(float(np.max(np.abs(th_r - th_all)[sig] / sd[sig])), 4),
        "fiducial_iteration_2_estimates_s": round(dt_i, 4),
        "fiducial_iteration_2nd_step_change_over_sigma": round(float(np.max(np.abs(hist_i[2] - hist_i[1])[sig] /
                                                                           sd[sig])), 4)}
    # posterior error maps of the 512^2 shear workload: 127 simulations in one batched solve
    wl = WL.shear_eb()
    base = base_of(wl)
    # B-mode band powers with the leakage as a bias against the full estimate (6 simulations)
    nb_e = wl.nbands // 2
    bband = list(range(nb_e, wl.nbands))
    dsh = wf.wf_simulate(base, 1, 2300, theta_true=wl.theta_true)[0]
    pdat = base.with_data(dsh)
    (thl, _, _, Fbb, _), dt_l = timed(lambda: wf.bmode_leakage_qe(pdat, 6, 2301, bband, opts=opts))
    (thf, _, _, Ff, _), dt_f = timed(lambda: wf.bandpower_qe(pdat, 6, 2301, opts=opts))
    sdf = np.sqrt(np.abs(np.diag(np.linalg.inv(Ff))))[bband]
    out["shear512_bmode_leakage"] = {
        "workload": f"512^2 E/B shear, {len(bband)} B bands, 6 simulations: leakage bias "
                    f"({6 * (2 + len(bband)) + 1} solves) vs the full estimate ({6 * (1 + wl.nbands) + 1})",
        "leakage_seconds": round(dt_l, 4), "full_seconds": round(dt_f, 4),
        "theta_B_max_diff_over_sigma_full": round(float(np.max(np.abs(thl - thf[bband]) / sdf)), 4)}
    (vm, vp, _), dt_pe = timed(lambda: wf.posterior_error(base, 127, 2200, opts=opts))
    out["shear512_posterior_error"] = {"workload": "512^2 E/B shear, residual variance per mode and per pixel from 127 "
                                                   "simulations (127 MAP solves)",
                                       "estimates_per_s": round(1.0 / dt_pe, 3), "solves_per_s": round(127 / dt_pe, 1),
                                       "mean_pixel_variance": float(vp.double().mean().item())}
    del vm, vp
    # scalar 512^2 density variant
    wl = WL.density_bands(512)
    base = base_of(wl)
    d = wf.wf_simulate(base, 127, 2100, theta_true=wl.theta_true)
    out["density512_maps"] = solve_line("512^2 density (the 256^2 band-power generator at 512^2)",
                                        [base.with_data(d[i]) for i in range(127)], opts)
    del d
    # 1024^2 CMB patch (the diagonal preconditioner: unpreconditioned L-BFGS needs > 4000 iterations)
    wl = WL.cmb_patch()
    base = base_of(wl)
    d = wf.wf_simulate(base, 16, 4100, theta_true=wl.theta_true)
    popts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, max_iter=4000, precond=1)
    out["cmb1024_maps"] = solve_line("1024^2 CMB, preconditioned L-BFGS", [base.with_data(d[i]) for i in range(16)],
                                     popts)
    # the paper's method on the same maps: no preconditioner (same stop test)
    uopts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, max_iter=20000)
    out["cmb1024_maps_unpreconditioned"] = solve_line("1024^2 CMB, L-BFGS without preconditioner",
                                                      [base.with_data(d[i]) for i in range(16)], uopts)
    # 1024^2 CMB band powers (40 linear bands): N_sim = 6 at the 1e-6 stop (247 solves per
    # estimate), and N_sim = 1 with float64 refinement to 3e-11 (42 solves; the stop that gives
    # maps within 1e-5 on this spectrum); both extrapolated to N_sim = 256 (10497 solves, in
    # chunks of 256) by solve count
    prob4 = base.with_data(d[0])
    nsim4 = 6
    ns4 = 1 + nsim4 * (1 + wl.nbands)
    (_, _, _, _, rc4), dt4 = timed(lambda: wf.bandpower_qe(prob4, nsim4, 4201, opts=popts))
    ropts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, max_iter=4000, precond=1, refine=4, refine_tol=3e-11)
    ns4r = 1 + 1 * (1 + wl.nbands)
    wf.bandpower_qe(prob4, 1, 4201, opts=popts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, _, rc4r = wf.bandpower_qe(prob4, 1, 4201, opts=ropts)
    torch.cuda.synchronize()
    dt4r = time.perf_counter() - t0
    n256 = 1 + 256 * (1 + wl.nbands)
    line4 = {"workload": f"1024^2 CMB, {wl.nbands} linear bands, preconditioned L-BFGS",
             "nsim": nsim4, "solves_per_estimate": ns4, "seconds": round(dt4, 3), "solves_per_s": round(ns4 / dt4, 1),
             "all_converged": rc4 == wf.WF_OK,
             "refined": {"nsim": 1, "refine_tol": 3e-11, "solves_per_estimate": ns4r, "seconds": round(dt4r, 3),
                         "solves_per_s": round(ns4r / dt4r, 1), "all_converged": rc4r == wf.WF_OK},
             "extrapolated_nsim256": {"solves": n256, "estimates_per_s_1e-6": round(ns4 / dt4 / n256, 5),
                                      "estimates_per_s_refined": round(ns4r / dt4r / n256, 5)}}
    # the refined solve of the committed oracle reference's data map (the same white normals,
    # simulated here in float32) against that reference
    gpath = os.path.join(ROOT, "tests", "golden", "cmb1024_map.npy")
    if os.path.exists(gpath):
        gmeta = json.load(open(gpath.replace(".npy", ".json")))
        seed_g = int(gmeta["data"].split("white_draws(1024, 1, 1, ")[1].split(")")[0])
        dr = torch.tensor(WL.white_draws(1024, 1, 1, seed_g), dtype=torch.float32, device=dev)
        dg = wf.wf_simulate(base, 1, 0, draws=dr, theta_true=wl.theta_true)[0]
        sg, _, stg, _ = wf.map_wf_solve([base.with_data(dg)], ropts)
        ref = np.load(gpath).astype(np.complex128)
        got = sg[0].cpu().numpy().astype(np.complex128)
        line4["refined_map_vs_oracle"] = {"field_rel_l2": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                                          "iters": stg[0].iters, "rel_grad": stg[0].rel_grad,
                                          "reference": "tests/golden/cmb1024_map.npy (oracle MAP to 1e-11)"}
    out["cmb1024_bandpowers"] = line4
    # convergence by scale of one CMB map (appendix B): reference 1e-6, looser 1e-2 .. 1e-4
    ctols = [1e-2, 1e-3, 1e-4]
    (cpow, cerr, ccv, cits, _, _), dt_c = timed(lambda: wf.convergence_by_band(base.with_data(d[0]), ctols, popts))
    ok = cpow[0] > 0
    out["cmb1024_convergence_by_scale"] = {
        "workload": "1024^2 CMB map, preconditioned, solved to 1e-6 and to 1e-2, 1e-3, 1e-4 in one batch",
        "seconds": round(dt_c, 3), "iterations": [int(x) for x in cits],
        # per tolerance: the largest band-power change |P_t / P_ref - 1| in units of the cosmic-variance scale
        "max_power_change_over_cv": [round(float(np.max(np.abs(cpow[t + 1][ok] / cpow[0][ok] - 1.0) / ccv[ok])), 4)
                                     for t in range(len(ctols))]}
    del d
    # 96-map uneven batch
    wls = WL.uneven_batch(96)
    probs = []
    for i, w in enumerate(wls):
        b0 = base_of(w)
        probs.append(b0.with_data(wf.wf_simulate(b0, 1, 5100 + i, theta_true=w.theta_true)[0]))
    line = solve_line("96 uneven maps (sides 128..1024, density / shear / CMB), preconditioned", probs, popts)
    plain_opts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, max_iter=4000, precond=1, use_graph=0,
                              iters_per_poll=1)
    # the same 96 maps one at a time (same tolerance and stop test)
    res, dtp = timed(lambda: [wf.map_wf_solve([p], plain_opts) for p in probs])
    line["plain_solves_per_s"] = round(len(probs) / dtp, 2)
    line["plain_converged"] = f"{sum(r[2][0].status == wf.WF_SOLVE_CONVERGED for r in res)}/{len(probs)}"
    line["speedup_batched_vs_plain"] = round(line["solves_per_s"] / line["plain_solves_per_s"], 2)
    # band-power estimates of the same 96 maps (one simulation each, every Fisher column): all
    # estimates' solves shared among batched solves, against one bandpower_qe call per map
    nsol = sum(2 + w.nbands for w in wls)
    # untimed first calls: the tiles of every (side, components, batch-size bucket) class are
    # tuned on a context's first solve of it, once for the shared batch and once per map kind
    # and side for the per-map path
    wf.bandpower_qe_batch(probs, 1, 5300, opts=popts)
    seen = set()
    for i, (w, p) in enumerate(zip(wls, probs)):
        if (w.n, w.ncomp, w.nbands) not in seen:
            seen.add((w.n, w.ncomp, w.nbands))
            wf.bandpower_qe(p, 1, 5300 + i, opts=popts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, _, rcb = wf.bandpower_qe_batch(probs, 1, 5300, opts=popts)
    torch.cuda.synchronize()
    dtb = time.perf_counter() - t0
    t0 = time.perf_counter()
    rcs = [wf.bandpower_qe(p, 1, 5300 + i, opts=popts)[4] for i, p in enumerate(probs)]
    torch.cuda.synchronize()
    dtm = time.perf_counter() - t0
    line["bandpower_estimates"] = {"nsim": 1, "solves": nsol, "batched_estimates_per_s": round(len(probs) / dtb, 3),
                                   "per_map_estimates_per_s": round(len(probs) / dtm, 3),
                                   "batched_solves_per_s": round(nsol / dtb, 1),
                                   "speedup_batched_vs_per_map": round(dtm / dtb, 2),
                                   "all_converged": rcb == wf.WF_OK and all(r == wf.WF_OK for r in rcs)}
    out["uneven96"] = line
    out["shear512_catalog"] = catalog_line(args)
    return out


def _deviation_from_truth(th, F, theta_true):
    """|theta_hat - theta_true| in units of each band's conditional error 1 / sqrt(F_bb), and of
    the marginal error sqrt((F^-1)_bb) over the bands carrying signal (F_bb above 1e-6 of the
    largest) when that block of F is positive definite (the conditional error ignores the
    mask's couplings between neighbouring bands)."""
    import numpy as np
    fd = np.diag(F)
    okb = fd > 0
    z = np.abs(th - theta_true)[okb] * np.sqrt(fd[okb])
    cond = {"median": round(float(np.median(z)), 3) if z.size else None,
            "max": round(float(np.max(z)), 3) if z.size else None,
            "worst_band": int(np.flatnonzero(okb)[np.argmax(z)]) if z.size else None, "bands": int(okb.sum())}
    sig = fd > 1e-6 * fd.max()
    Fs = 0.5 * (F[np.ix_(sig, sig)] + F[np.ix_(sig, sig)].T)
    marg = None
    if sig.any() and np.linalg.eigvalsh(Fs).min() > 0:
        zm = np.abs(th - theta_true)[sig] / np.sqrt(np.diag(np.linalg.inv(Fs)))
        marg = {"median": round(float(np.median(zm)), 3), "max": round(float(np.max(zm)), 3),
                "bands": int(sig.sum())}
    return cond, marg


def cmb_full_line(args):
    """The 1024^2 CMB band-power estimate at its full size: 40 linear bands, 256 simulations
    (1 + 256 x 41 = 10497 MAP solves, run in batches of 256), preconditioned L-BFGS to the
    bench's tolerance; one untimed estimate with 2 simulations first (tile tuning, graph capture)."""
    import torch

    import paper_1810_00503_amd as wf
    from paper_1810_00503_amd import workloads as WL
    wf.load()
    dev = "cuda:0"
    wl = WL.cmb_patch()
    base = wf.Problem(torch.tensor(wl.W, dtype=torch.float32, device=dev), wl.pshape, wl.band, wl.theta_fid)
    d = wf.wf_simulate(base, 1, 4100, theta_true=wl.theta_true)[0]
    prob = base.with_data(d)
    popts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, max_iter=4000, precond=1)
    nsim = 256
    wf.bandpower_qe(prob, 2, 4201, opts=popts)
    torch.cuda.synchronize()
    print(f"cmb-full: warm-up done, {nsim} simulations next", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    th, E, b, F, rc = wf.bandpower_qe(prob, nsim, 4201, opts=popts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ns = 1 + nsim * (1 + wl.nbands)
    # deviation from the truth (the damping tail's bands carry almost no signal, so the full
    # inverse of F is dominated by noise there)
    cond, marg = _deviation_from_truth(th, F, wl.theta_true)
    return {"workload": f"1024^2 CMB (cmb_patch generator), {wl.nbands} linear bands, {nsim} simulations, "
                        f"preconditioned L-BFGS m={args.m} to {args.tol:g} rel. grad",
            "nsim": nsim, "solves": ns, "seconds": round(dt, 2), "estimates_per_s": round(1.0 / dt, 5),
            "solves_per_s": round(ns / dt, 1), "all_converged": rc == wf.WF_OK,
            "theta_hat_first_bands": [round(float(x), 4) for x in th[:5]],
            "theta_hat_minus_truth_over_cond_sigma": cond,
            "theta_hat_minus_truth_over_marginal_sigma": marg}


def cmb_iterate_line(args):
    """The 1024^2 CMB band-power estimate with 64 simulations (2625 MAP solves per estimate),
    once at the workload's fiducial (the truth scaled band by band by U(0.01, 1)) and after one
    step of the fiducial iteration (sec. 2.3: the fiducial reset to the first estimate), each
    with its deviation from the truth in the errors of its own F."""
    import torch

    import paper_1810_00503_amd as wf
    from paper_1810_00503_amd import workloads as WL
    wf.load()
    dev = "cuda:0"
    wl = WL.cmb_patch()
    base = wf.Problem(torch.tensor(wl.W, dtype=torch.float32, device=dev), wl.pshape, wl.band, wl.theta_fid)
    prob = base.with_data(wf.wf_simulate(base, 1, 4200, theta_true=wl.theta_true)[0])
    popts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, max_iter=4000, precond=1)
    nsim = 64
    t0 = time.perf_counter()
    th1, _, _, F1, rc1 = wf.bandpower_qe(prob, nsim, 4201, opts=popts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    th2, hist, _, _, F2, rc2 = wf.bandpower_iterate(prob, nsim, 4201, max_iter=2, rel_tol=0.0, opts=popts)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    c1, m1 = _deviation_from_truth(th1, F1, wl.theta_true)
    c2, m2 = _deviation_from_truth(th2, F2, wl.theta_true)
    return {"workload": f"1024^2 CMB (cmb_patch generator), {wl.nbands} linear bands, {nsim} simulations per "
                        f"estimate, preconditioned L-BFGS m={args.m} to {args.tol:g} rel. grad",
            "one_estimate_seconds": round(t1 - t0, 2), "two_step_iteration_seconds": round(t2 - t1, 2),
            "all_converged": rc1 == wf.WF_OK and rc2 == wf.WF_OK, "iteration_steps": int(len(hist) - 1),
            "at_workload_fiducial": {"cond_sigma": c1, "marginal_sigma": m1},
            "after_one_fiducial_step": {"cond_sigma": c2, "marginal_sigma": m2}}


def catalog_line(args):
    """512^2 E/B shear at the catalog level (sec. 3.4): ~10 galaxies per observed pixel at
    their own positions, the field evaluated at each galaxy by the library's non-uniform
    transform.  Data: a field drawn from the truth (complex normals times sqrt(S_true / 2) on
    the half plane), evaluated at the galaxies by the library, plus shape noise sigma_e.  One
    catalog, then a batch of 8 catalogs (same positions, other noise), and the binned-map solve
    of the same galaxies (mean shape per pixel, weight = count / sigma_e^2) for reference."""
    import numpy as np
    import torch

    import paper_1810_00503_amd as wf
    from paper_1810_00503_amd import workloads as WL
    dev = "cuda:0"
    n = 512
    cat = WL.shear_catalog(n, 5100, ngal_mean=10.0)
    S_true = np.where(cat.band >= 0, cat.theta_true[np.maximum(cat.band, 0)], 1.0) * cat.pshape   # band -1: amplitude 1
    g = torch.Generator(device="cpu").manual_seed(5101)
    z = torch.complex(torch.randn(S_true.shape, generator=g, dtype=torch.float64),
                      torch.randn(S_true.shape, generator=g, dtype=torch.float64))
    s_true = (z * torch.from_numpy(np.sqrt(S_true / 2.0))).to(torch.complex64).to(dev)
    prob = wf.Problem.for_catalog(n, cat.pshape, cat.band, cat.theta_fid, device=dev)
    pos = torch.tensor(cat.pos, device=dev)
    gam = wf.catalog_forward(prob, wf.GalaxyCatalog(pos), s_true)
    sig = float(1.0 / np.sqrt(cat.wgt[0]))
    wgt = torch.tensor(cat.wgt, dtype=torch.float32, device=dev)
    cats = [wf.GalaxyCatalog(pos, gam + sig * torch.randn(gam.shape, generator=torch.Generator(device=dev).manual_seed(
        5200 + i), device=dev), wgt) for i in range(8)]
    opts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    (_, st1, _), dt1 = timed(lambda: wf.map_wf_solve_catalog([prob], cats[:1], opts))
    (_, st8, _), dt8 = timed(lambda: wf.map_wf_solve_catalog([prob] * 8, cats, opts))
    # where one solve's device time goes (HIP events around every launch: graphs off, so this
    # call is slower than the timed one; the split is what it reports)
    wf.set_profiling(True)
    wf.reset_kernel_stats()
    wf.map_wf_solve_catalog([prob], cats[:1], opts)
    torch.cuda.synchronize()
    ks = wf.kernel_stats()
    wf.set_profiling(False)
    split = {"galaxy_passes_ms": ks["catalog"]["ms"],
             "transforms_2n_ms": ks["colinv"]["ms"] + ks["row"]["ms"] + ks["colfwd"]["ms"],
             "solver_vector_passes_ms": sum(ks[k]["ms"] for k in ("passA", "passB", "post", "coef", "misc")),
             "galaxy_pass_launches": ks["catalog"]["launches"]}
    # the same galaxies binned: mean shape per pixel, weight count / sigma_e^2
    iy = torch.floor(pos[:, 0]).long().clamp_(0, n - 1)
    ix = torch.floor(pos[:, 1]).long().clamp_(0, n - 1)
    pix = iy * n + ix
    cnt = torch.zeros(n * n, dtype=torch.float32, device=dev).index_add_(0, pix, torch.ones_like(pix, dtype=torch.float32))
    dmap = torch.stack([torch.zeros(n * n, device=dev).index_add_(0, pix, cats[0].e[c]) for c in range(2)])
    dmap = torch.where(cnt > 0, dmap / cnt.clamp(min=1.0), torch.zeros_like(dmap)).reshape(2, n, n)
    W = (cnt / sig ** 2).reshape(n, n)
    pb = wf.Problem(W, cat.pshape, cat.band, cat.theta_fid, d=dmap)
    (_, _, stb, _), dtb = timed(lambda: wf.map_wf_solve([pb], opts))
    return {"workload": f"512^2 E/B shear catalog, Poisson(10) galaxies per observed pixel ({cat.ngal} galaxies), "
                        f"catalog-level response (non-uniform transform on a 1024^2 grid)",
            "galaxies": cat.ngal, "solves_per_s": round(1.0 / dt1, 2), "ms_per_solve": round(dt1 * 1e3, 2),
            "iters": st1[0].iters, "batch8_solves_per_s": round(8 / dt8, 2),
            "batch8_iters_mean": round(float(np.mean([x.iters for x in st8])), 1),
            "galaxy_evaluations_per_s": round(cat.ngal * 2 * (st1[0].iters + st1[0].ngrad) / dt1, 1),
            "binned_map_solves_per_s": round(1.0 / dtb, 2), "binned_map_iters": stb[0].iters,
            "device_time_split": {k: round(v, 3) if isinstance(v, float) else v for k, v in split.items()}}


def density_bands_line(args):
    """The 256^2 density band-power estimate alone (12 bands, 128 simulations, 1665 MAP solves
    per estimate, L-BFGS to the benchmark's tolerance): one untimed estimate, then --steps
    timed ones, the same inputs as the secondary line."""
    import numpy as np
    import torch

    import paper_1810_00503_amd as wf
    from paper_1810_00503_amd import workloads as WL
    wf.load()
    dev = "cuda:0"
    wl = WL.density_bands()
    base = wf.Problem(torch.tensor(wl.W, dtype=torch.float32, device=dev), wl.pshape, wl.band, wl.theta_fid)
    prob = base.with_data(wf.wf_simulate(base, 1, 2000, theta_true=wl.theta_true)[0])
    nsim = 128
    opts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol)
    wf.bandpower_qe(prob, nsim, 2001, opts=opts)
    torch.cuda.synchronize()
    ts = []
    for _ in range(max(1, args.steps)):
        t0 = time.perf_counter()
        wf.bandpower_qe(prob, nsim, 2001, opts=opts)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    ns = 1 + nsim * (1 + wl.nbands)
    return {"workload": f"256^2 density, {wl.nbands} bands, {nsim} simulations ({ns} MAP solves per estimate)",
            "estimates": len(ts), "bandpower_estimates_per_s": round(1.0 / dt, 3), "solves_per_s": round(ns / dt, 1)}


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.cpu_child:
        cpu_child(args)
        return
    if args.catalog_only:
        print(json.dumps({"shear512_catalog": catalog_line(args)}), flush=True)
        return
    if args.cmb_full:
        print(json.dumps({"cmb1024_bandpowers_nsim256": cmb_full_line(args)}), flush=True)
        return
    if args.cmb_iterate:
        print(json.dumps({"cmb1024_fiducial_iteration": cmb_iterate_line(args)}), flush=True)
        return
    if args.density_bands_only:
        print(json.dumps({"density256_bandpowers": density_bands_line(args)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the simulation batches would shard "
              f"across GPUs with one all-reduce of E and F, which is not implemented.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1810_00503_amd as wf
    from paper_1810_00503_amd import workloads as WL

    wf.load()
    dev = "cuda:0"
    wl = WL.shear_eb(args.n)
    W = torch.tensor(wl.W, dtype=torch.float32, device=dev)
    base = wf.Problem(W, wl.pshape, wl.band, wl.theta_fid)
    # the observed map: a simulation from the truth (Theta = 1), Philox stream 0
    d = wf.wf_simulate(base, 1, args.seed, sim0=0, theta_true=wl.theta_true)[0]
    prob = base.with_data(d)
    opts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol)
    nb = wl.nbands
    nsolve = 1 + args.nsim * (1 + nb)
    sim_seed = args.seed + 1

    def step():
        return wf.bandpower_qe(prob, args.nsim, sim_seed, opts=opts)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        th, E, b, F, rc = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    value = nsolve * args.steps / elapsed

    # the step's solves as separate problems (for the solve-only and plain comparisons)
    sims = [prob]
    dsim = wf.wf_simulate(base, args.nsim, sim_seed, sim0=0)
    for i in range(args.nsim):
        sims.append(base.with_data(dsim[i]))
        for l in range(nb):
            di = wf.wf_simulate(base, 1, sim_seed, sim0=i, boost_band=l, boost_factor=2.0)[0]
            sims.append(base.with_data(di))
    torch.cuda.synchronize()
    wf.map_wf_solve(sims, opts)
    torch.cuda.synchronize()
    tb = []
    for _ in range(3):   # median of three calls
        t0 = time.perf_counter()
        _, _, st_b, _ = wf.map_wf_solve(sims, opts)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    t_batch = float(np.median(tb))
    iters = [s.iters for s in st_b]
    # the same batch with conjugate gradients (same operator, tolerance and stop test)
    cg_line = None
    if not args.lbfgs_only:
        copts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, method=wf.WF_METHOD_CG)
        wf.map_wf_solve(sims, copts)
        torch.cuda.synchronize()
        tc = []
        for _ in range(3):
            t0 = time.perf_counter()
            _, _, st_c, _ = wf.map_wf_solve(sims, copts)
            torch.cuda.synchronize()
            tc.append(time.perf_counter() - t0)
        cg_line = {"solves_per_s": round(nsolve / float(np.median(tc)), 2),
                   "iters_mean": round(float(np.mean([x.iters for x in st_c])), 1),
                   "iters_max": int(max(x.iters for x in st_c)),
                   "exact_gradients_mean": round(float(np.mean([x.ngrad for x in st_c])), 1),
                   "converged": f"{sum(x.status == wf.WF_SOLVE_CONVERGED for x in st_c)}/{nsolve}"}
    # the same batch with the optional diagonal noise-aware preconditioner (off by default: the method
    # solves without one); the stop test stays the exact whitened relative gradient
    # (with the secondary lines: it would mix shorter-history pass-B launches into a profile of the step)
    pc_line = None
    if not args.no_secondary and not args.lbfgs_only:
        pcopts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, precond=1)
        wf.map_wf_solve(sims, pcopts)
        torch.cuda.synchronize()
        tp = []
        for _ in range(3):
            t0 = time.perf_counter()
            _, _, st_p, _ = wf.map_wf_solve(sims, pcopts)
            torch.cuda.synchronize()
            tp.append(time.perf_counter() - t0)
        pc_line = {"solves_per_s": round(nsolve / float(np.median(tp)), 2),
                   "iters_mean": round(float(np.mean([x.iters for x in st_p])), 1),
                   "iters_max": int(max(x.iters for x in st_p)),
                   "rel_grad_max": float(max(x.rel_grad for x in st_p)),
                   "converged": f"{sum(x.status == wf.WF_SOLVE_CONVERGED for x in st_p)}/{nsolve}"}
    # the same batch at other history lengths (the paper does not fix m): per iteration the solver
    # moves about 3m + 11 field vectors, so the history length trades traffic per iteration
    # against the iterations it saves
    m_sweep = None
    if not args.no_secondary and not args.lbfgs_only:
        m_sweep = {}
        for mm in (3, 5, 10, 16):
            mopts = wf.LbfgsOpts(m=mm, rel_grad_tol=args.tol)
            wf.map_wf_solve(sims, mopts)
            torch.cuda.synchronize()
            tm = []
            for _ in range(3):
                t0 = time.perf_counter()
                _, _, st_m, _ = wf.map_wf_solve(sims, mopts)
                torch.cuda.synchronize()
                tm.append(time.perf_counter() - t0)
            m_sweep[f"m={mm}"] = {"solves_per_s": round(nsolve / float(np.median(tm)), 2),
                                  "iters_mean": round(float(np.mean([x.iters for x in st_m])), 1),
                                  "iters_max": int(max(x.iters for x in st_m)),
                                  "converged": f"{sum(x.status == wf.WF_SOLVE_CONVERGED for x in st_m)}/{nsolve}"}
    conv = sum(s.status == wf.WF_SOLVE_CONVERGED for s in st_b)

    plain = plain_graph = None
    if not args.no_plain:
        npl = len(sims) if args.plain_solves <= 0 else min(args.plain_solves, len(sims))
        popts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, use_graph=0, iters_per_poll=1)
        wf.map_wf_solve(sims[:1], popts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in sims[:npl]:
            wf.map_wf_solve([p], popts)
        torch.cuda.synchronize()
        plain = npl / (time.perf_counter() - t0)
        # one map at a time, but with the batch's graph replay (8 iterations between host polls):
        # separates what batching gains from what the captured iterations gain
        gopts = wf.LbfgsOpts(m=args.m, rel_grad_tol=args.tol, iters_per_poll=8)
        wf.map_wf_solve(sims[:1], gopts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in sims[:npl]:
            wf.map_wf_solve([p], gopts)
        torch.cuda.synchronize()
        plain_graph = npl / (time.perf_counter() - t0)

    # one instrumented step: events around every launch, device-counted algorithmic bytes
    wf.reset_kernel_stats()
    wf.set_profiling(True)
    step()
    torch.cuda.synchronize()
    ks = wf.kernel_stats()
    wf.set_profiling(False)
    dom = max(ks, key=lambda k: ks[k]["ms"])
    kd = ks[dom]
    achieved = kd["bytes"] / (kd["ms"] * 1e-3) / 1e9 if kd["ms"] > 0 else 0.0
    per_kernel = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                      "GB_per_s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 and v["bytes"] > 0
                      else None} for k, v in ks.items()}
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
            "avg_launch_us": round(1e3 * kd["ms"] / max(kd["launches"], 1), 2),
            "bytes_per_launch": kd["bytes"] / max(kd["launches"], 1)}

    # the fused transform chain of one gradient / curvature product (column inverse, row pass with
    # the mask and noise weights, column forward with the prior scale and the solver's dots)
    chain_k = ("colinv", "row", "colfwd")
    cb = sum(ks[k]["bytes"] for k in chain_k)
    cm = sum(ks[k]["ms"] for k in chain_k)
    ca = cb / (cm * 1e-3) / 1e9 if cm > 0 else 0.0
    roof_chain = {"bound": "hbm", "kernels": "+".join(chain_k), "achieved": round(ca, 1), "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": round(ca / HBM_PEAK_GBS, 4), "ms_per_step": round(cm, 3),
                  "bytes_per_step": cb}
    # the same chain against its algorithmic minimum: per curvature product read p and write Dp
    # (2 vectors), per exact gradient read w and d and write g (3 vectors); W and the prior tables
    # are shared by the batch (one field vector = ncomp n^2 float32 = the [ncomp][n][n/2] complex field)
    vb = 2 * args.n * args.n * 4
    alg = sum((2.0 * x.iters + 3.0 * x.ngrad) * vb for x in st_b)
    aa = alg / (cm * 1e-3) / 1e9 if cm > 0 else 0.0
    roof_chain["algorithmic_bytes_per_step"] = alg
    roof_chain["algorithmic_GBps"] = round(aa, 1)
    roof_chain["algorithmic_frac"] = round(aa / HBM_PEAK_GBS, 4)
    # counting as algorithmic also the L-BFGS Gram reads that the column-forward pass does for
    # the solver (g and the other kept Dp_j: min(k, m) vectors at iteration k), which the
    # vector algebra would otherwise need in a pass of its own
    gram = sum(sum(min(k, args.m) for k in range(x.iters)) * vb for x in st_b)
    ag = (alg + gram) / (cm * 1e-3) / 1e9 if cm > 0 else 0.0
    roof_chain["algorithmic_with_gram_bytes_per_step"] = alg + gram
    roof_chain["algorithmic_with_gram_frac"] = round(ag / HBM_PEAK_GBS, 4)

    # the chain's HBM bytes by the committed counters (rocprofv3 FETCH_SIZE / WRITE_SIZE of the
    # L-BFGS launches of these kernels, calibrated by the streaming copy), per step: each
    # kernel's counted bytes per launch times its launches in the instrumented step; null when
    # any of the three kernels' sources changed since the counters were taken
    tiles = wf.get_chain_tiles(args.n, 2, wf.WF_F32, nsolve)
    names = {"colinv": "colinvr" if tiles[3] & 2 else "colinv", "row": "rowr" if tiles[3] & 1 else "row",
             "colfwd": "colfwdr" if tiles[3] & 4 else "colfwd"}
    per_launch = {k: measured_traffic(v) for k, v in names.items()}
    if all(v is not None for v in per_launch.values()):
        tb = sum(per_launch[k] * ks[k]["launches"] for k in chain_k)
        roof_chain["traffic"] = tb
        roof_chain["traffic_GBps"] = round(tb / (cm * 1e-3) / 1e9, 1) if cm > 0 else None
        roof_chain["traffic_frac"] = round(tb / (cm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if cm > 0 else None
    else:
        roof_chain["traffic"] = None

    # measured copy ceiling (context for the roofline): the library's streaming copy of 2 GiB
    roof["copy_ceiling_GBps"] = round(wf.copy_bandwidth(2 * 1024 ** 3, 5), 1)
    roof_chain["copy_ceiling_GBps"] = roof["copy_ceiling_GBps"]
    # the same rates as fractions of that measured ceiling (context beside the peak fraction)
    if roof["copy_ceiling_GBps"] > 0:
        roof["frac_of_copy_ceiling"] = round(achieved / roof["copy_ceiling_GBps"], 4)
        roof_chain["frac_of_copy_ceiling"] = round(ca / roof["copy_ceiling_GBps"], 4)

    def gpu_solve(ds, srefs):
        probs = [base.with_data(torch.tensor(np.asarray(d), dtype=torch.float32, device=dev)) for d in ds]
        s_, x_, st_, _ = wf.map_wf_solve(probs, opts, want_maps=True)
        E_ = [wf.wf_band_E(p, t) for p, t in zip(probs, s_)]
        th_ = [wf.wf_chi2_dtheta(p, torch.tensor(np.asarray(sr), dtype=torch.complex64, device=dev))
               for p, sr in zip(probs, srefs)]
        return [t.cpu().numpy() for t in s_], [t.cpu().numpy() for t in x_], st_, E_, th_

    cpu = None if args.no_cpu else cpu_baseline(args, gpu_solve)
    accuracy = cpu.pop("accuracy", None) if isinstance(cpu, dict) else None
    secondary = None if args.no_secondary else secondary_workloads(args)
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.n}^2 joint E/B shear (shear_eb generator), {nb} bands; one bandpower_qe "
                               f"step = {nsolve} MAP solves (1 data + {args.nsim} sims x (1 + {nb} bands)) in one "
                               f"batch to {args.tol:g} rel. grad, L-BFGS m={args.m}",
                   "n": args.n, "ncomp": 2, "batch": nsolve, "nsim": args.nsim, "nbands": nb,
                   "rel_grad_tol": args.tol, "m": args.m},
        "roofline": roof,
        "roofline_gradient_chain": roof_chain,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "batched_solve_only_solves_per_s": round(len(sims) / t_batch, 2),
        "batched_solve_only_cg": cg_line,
        "batched_solve_only_precond": pc_line,
        "batched_solve_only_m_sweep": m_sweep,
        "plain_solves_per_s": None if plain is None else round(plain, 2),
        "plain_graph_solves_per_s": None if plain_graph is None else round(plain_graph, 2),
        "speedup_batched_vs_plain": None if plain is None else round(len(sims) / t_batch / plain, 2),
        "bandpower_estimates_per_s": round(args.steps / elapsed, 3),
        "iters_mean": round(float(np.mean(iters)), 1), "iters_max": int(np.max(iters)),
        "chain_tiles": {"rows_per_wg": tiles[0], "col_blocks_per_wg": tiles[1], "instances_per_launch": tiles[2],
                        "register_staged": {"row": bool(tiles[3] & 1), "column_inverse": bool(tiles[3] & 2),
                                            "column_forward": bool(tiles[3] & 4)},
                        "autotuned": tiles[4]},
        "converged": f"{conv}/{len(sims)}",
        "per_kernel": per_kernel,
        "secondary": secondary,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
