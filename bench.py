"""Benchmark of the RSRR hot path on one MI355X.

A step is one full solve (Alg. 2 around Alg. 1: assembly, batched LU + solves
with refinement, basis, projection, reduced problem, eigenpair recovery and
residual filter) of one synthetic workload whose inputs are already resident
in device memory.  The default workload is the largest single-GPU
configuration: the dense Helmholtz BEM matrix on a Fibonacci sphere, n = 8192,
entries assembled on the fly at every node, ellipse centre 3 with semi-axes
(1.5, 0.3), N = 40 nodes, L = 64 probing vectors, complex64 factorisations
with fp64 refinement.

Prints one JSON line.  `value` = resolvent samples per second of the whole
step (N samples per solve); eigenpairs per second and per-step latency
percentiles are reported beside it.  Kernel statistics come from one extra
solve with every kernel timer on, outside the timed region; the timed steps
record HIP events only around the launches of the kernel function that took
most device time in that pass, and the roofline object is computed from
those events.  `cpu_baseline` is the CPU oracle timed on a bounded sample of
the same workload (a few of its sampling nodes), with the oracle's end-to-end
time on the small QEP beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "hbm": 8.0e12}

def kernel_bound(sym: str):
    """(bound, peak) for a kernel function, or None if it has no model."""
    if sym.startswith("gemm_kernel<double"):
        return "mfma", PEAK["fp64_mfma"]
    if sym.startswith("gemm_kernel<float"):
        return "mfma", PEAK["fp32_mfma"]
    if sym.startswith(("bj_gram_kernel", "bj_apply_kernel")):
        return "mfma", PEAK["fp64_mfma"]    # FP64 MFMA 16x16x4 Gram and apply
    if sym.startswith(("lu_panel_kernel", "pchol_panel_kernel", "lu_permute_kernel")):
        return "hbm", PEAK["hbm"]          # panels are latency bound; priced on their bytes
    return None



def sources_sha256() -> str:
    """Hash of every library source: the kernels and the drivers that decide
    the launch mix a per-launch traffic figure averages over."""
    d = os.path.join(ROOT, "paper_1510_07522_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def traffic_record(sym: str):
    """HBM bytes per launch from the committed counter summary of this kernel
    function, if no library source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(sym)
    if not rec or rec.get("sources_sha256") != sources_sha256():
        return None
    return rec.get("hbm_bytes_per_launch")


def _pmc_rows(folder: str):
    """Per-dispatch counter values of one rocprofv3 --pmc output folder, as
    {"Kernel_Name", "Counter_Value"} rows: from its counter_collection.csv
    (--output-format csv) or from its results database (the default format)."""
    import csv
    import glob
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if len(files) == 1:
        return list(csv.DictReader(open(files[0])))
    dbs = glob.glob(os.path.join(folder, "**", "*results.db"), recursive=True)
    if len(files) == 0 and len(dbs) == 1:
        import sqlite3
        con = sqlite3.connect(dbs[0])
        rows = con.execute("select name, counter_value from pmc_events").fetchall()
        con.close()
        return [{"Kernel_Name": n, "Counter_Value": v} for n, v in rows]
    raise SystemExit(f"{folder}: expected one counter_collection.csv or one results database")


def _kernel_sym(name: str) -> str:
    """Kernel function as the library's timers name it: no return type,
    namespace or argument list."""
    name = name.replace("void ", "", 1).replace("rsrr::", "")
    depth = 0
    for i, ch in enumerate(name):
        depth += ch == "<"
        depth -= ch == ">"
        if ch == "(" and depth == 0:
            return name[:i]
    return name


def write_traffic(dirs, sym: str, copy_mib: int, workload_desc: str):
    """HBM bytes per launch of one kernel function from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for a plain device copy of copy_mib MiB (the copy reads and writes exactly
    that many bytes)."""
    f_dir, w_dir, cf_dir, cw_dir = dirs
    per = {}
    for tag, folder in (("fetch", f_dir), ("write", w_dir)):
        vals = [float(r["Counter_Value"]) * 1024.0 for r in _pmc_rows(folder)
                if _kernel_sym(r["Kernel_Name"]) == sym]
        if not vals:
            raise SystemExit(f"{folder}: no dispatch of {sym}")
        per[tag] = (sum(vals) / len(vals), len(vals))
    true_bytes = float(copy_mib) * (1 << 20)
    scale = {}
    for tag, folder in (("fetch", cf_dir), ("write", cw_dir)):
        vals = [float(r["Counter_Value"]) * 1024.0 for r in _pmc_rows(folder)
                if "copyBuffer" in r["Kernel_Name"]]
        if not vals:
            raise SystemExit(f"{folder}: no copy dispatch")
        scale[tag] = true_bytes / (sum(vals) / len(vals))
    fetch = per["fetch"][0] * scale["fetch"]
    write = per["write"][0] * scale["write"]
    path = os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    rec[sym] = {"sources_sha256": sources_sha256(),
                "hbm_bytes_per_launch": fetch + write, "fetch_bytes_per_launch": fetch,
                "write_bytes_per_launch": write, "launches": per["fetch"][1],
                "fetch_scale": scale["fetch"], "write_scale": scale["write"],
                "workload": workload_desc}
    json.dump(rec, open(path, "w"), indent=1)
    print(json.dumps(rec[sym], indent=1))


def roofline_of(sym: str, t: dict, steps: int):
    bp = kernel_bound(sym)
    if bp is None or t["launches"] == 0:
        return None
    bound, peak = bp
    avg_s = t["ms"] / 1e3 / t["launches"]
    if bound == "hbm":
        work, unit, scale = t["bytes"] / t["launches"], "GB/s", 1e9
    else:
        work, unit, scale = t["flops"] / t["launches"], "TFLOP/s", 1e12
    if work <= 0:
        return None
    ach = work / avg_s
    # Gauss 3M products (last template argument true) count 8 real flops per
    # complex multiply-add like any complex product but execute 6 of them
    executed = 0.75 if sym.startswith("gemm_kernel<") and sym.endswith(", true>") else 1.0
    return {"kernel": sym, "bound": bound, "achieved": ach / scale, "peak": peak / scale, "unit": unit,
            "frac": ach / peak, "executed_frac": executed * ach / peak if bound == "mfma" else None,
            "traffic": traffic_record(sym), "algorithmic_per_launch": work,
            "algorithmic_bytes_per_launch": t["bytes"] / t["launches"],
            "launches_per_step": t["launches"] / steps, "avg_launch_ms": avg_s * 1e3,
            "ms_per_step": t["ms"] / steps}


def kernel_roofline(timers: dict, steps: int):
    """Roofline of the kernel function with the most device time (HIP events
    around each of its launches), and of the next few."""
    rows = [r for r in (roofline_of(k[4:], v, steps) for k, v in timers.items() if k.startswith("sym:"))
            if r is not None]
    rows.sort(key=lambda r: -r["ms_per_step"])
    if not rows:
        return None, []
    return rows[0], [{k: r[k] for k in ("kernel", "bound", "frac", "executed_frac", "achieved", "unit", "ms_per_step")}
                     for r in rows[1:8]]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name: str):
    import nep_inputs as ni
    if name == "c1":
        p, c, N, L, U = ni.config_c1()
        return dict(prob=p, contour=c, N=N, L=L, U=U,
                    desc="delay NEP -zI + A0 + A1 exp(-z), n=2048, circle |z|<3, N=48, L=48")
    if name == "c0":
        p, c, N, L, U = ni.config_c0()
        return dict(prob=p, contour=c, N=N, L=L, U=U,
                    desc="dense QEP z^2 I + z C + K, n=200, circle centre 5i r=2, N=32, L=20")
    if name == "c3":
        p, c, N, L, U = ni.config_c3()
        return dict(prob=p, contour=c, N=N, L=L, U=U,
                    desc="Helmholtz BEM sphere n=8192, ellipse centre 3 (1.5, 0.3), N=40, L=64")
    if name.startswith("c1n"):           # reduced-size variant of c1, e.g. c1n1024
        n = int(name[3:])
        p, c, N, L, U = ni.config_c1(n=n)
        return dict(prob=p, contour=c, N=N, L=L, U=U, desc=f"delay NEP as c1 with n={n}")
    raise SystemExit(f"unknown workload {name}")


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 0) for d in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count()


def cpu_baseline(name: str, w, max_nodes: int, budget_s: float):
    """The oracle on the host: (1) Alg. 2 Step 2 (LAPACK LU solve per node,
    complex128) on as many of the workload's own nodes as fit the budget,
    converted to samples/s (an upper bound on the oracle's end-to-end rate:
    the basis, projection and reduced problem come on top); (2) the oracle
    end to end on the small QEP (n = 200), timed here; (3) the oracle end to
    end on this workload as recorded by tests/golden/make_oracle_golden.py
    (host and thread count stated in the record)."""
    import nep_inputs as ni
    from oracle import rsrr_ref as R
    z, _ = R.contour_quadrature(w["contour"], w["N"])
    t0 = time.perf_counter()
    done = 0
    for zj in z[:max_nodes]:
        R.sample_resolvent(w["prob"], [zj], w["U"])
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    p0, c0, N0, L0, U0 = ni.config_c0()
    t1 = time.perf_counter()
    ref0 = R.rsrr(p0, c0, N0, L0, U0)
    dt0 = time.perf_counter() - t1
    out = {"value": done / dt, "unit": "resolvent samples/s", "cores": _blas_threads(),
           "kind": "oracle",
           "sample": f"Alg. 2 Step 2 only (LAPACK LU solve per node, complex128) on {done} of the "
                     f"{w['N']} sampling nodes of this workload ({dt:.1f} s); the basis, projection "
                     f"and reduced problem are not included, so this bounds the oracle's end-to-end "
                     f"samples/s from above",
           "end_to_end_c0": {"seconds": dt0, "resolvent_samples_per_s": N0 / dt0,
                             "eigenpairs_per_s": len(ref0["lam"]) / dt0, "n_eig": len(ref0["lam"]),
                             "what": "oracle end to end on the small QEP n=200, N=32, L=20, timed here"}}
    gold = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.json")
    if os.path.exists(gold):
        g = json.load(open(gold))
        out["end_to_end_recorded"] = {
            "seconds": g["oracle_seconds"], "resolvent_samples_per_s": g["N"] / g["oracle_seconds"],
            "eigenpairs_per_s": g["count"] / g["oracle_seconds"], "n_eig": g["count"],
            "host": g["host"], "what": "oracle end to end on this workload, recorded by "
                                       "tests/golden/make_oracle_golden.py (not on this host)"}
    return out


def batched_bench(a, P):
    """The batched-instance workload: sixteen dense QEPs of uneven order
    (n ~ U{512..4096}, k ~ U[1,400], circle centre 10i radius 4, N = 64,
    L = 32) solved by one rsrr_solve_batched call per step: all 1024
    (instance, node) LUs factored together, then each instance's later
    stages.  value = resolvent samples per second over all instances."""
    import torch
    import nep_inputs as ni
    insts = ni.config_c2()
    sizes = [p.n for p, *_ in insts]
    log(f"workload c2: 16 QEPs, n = {sizes}, N=64, L=32")
    # LU panel width from the autotuner: one factorisation of an instance's
    # 64 matrices at the largest order per candidate width
    nb_tuned, ms_tuned = P.tune_lu(a.precision, max(sizes), 64)
    log(f"autotuned LU panel width {nb_tuned} ({ms_tuned:.1f} ms for 64 matrices of order {max(sizes)})")
    hs = [P.Problem(p) for p, *_ in insts]
    cts = [P.contour(c.center, c.a, c.b) for _, c, _, _, _ in insts]
    prms = [P.default_params(N=N, L=L, precision=a.precision, nb=0) for _, _, N, L, _ in insts]
    Us = [P.to_device(U) for *_, U in insts]
    samples = sum(N for _, _, N, _, _ in insts)
    for i in range(a.warmup):
        t0 = time.perf_counter()
        outs = P.solve_batched(hs, cts, prms, Us)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t0:.3f}s n_eig={sum(o['info']['n_eig'] for o in outs)}")
    P.timers_only(None)
    P.timers_reset()
    P.timers_enable(True)
    P.solve_batched(hs, cts, prms, Us)
    torch.cuda.synchronize()
    P.timers_enable(False)
    stats = P.timers_read()
    classes = {k: v for k, v in stats.items() if not k.startswith("sym:")}
    dev_ms = sum(t["ms"] for t in classes.values())
    pre_roof, roof_next = kernel_roofline(stats, 1)
    dominant = pre_roof["kernel"] if pre_roof else None
    log(f"kernel statistics pass: {dev_ms:.1f} ms of timed device work; dominant kernel {dominant}")
    P.timers_reset()
    if dominant:
        P.timers_only(dominant)
        P.timers_enable(True)
    lat, n_eig = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(a.steps):
        t0 = time.perf_counter()
        outs = P.solve_batched(hs, cts, prms, Us)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        n_eig.append(sum(o["info"]["n_eig"] for o in outs))
        log(f"step {i}: {lat[-1]:.3f}s n_eig={n_eig[-1]}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    P.timers_enable(False)
    timed = P.timers_read()
    P.timers_only(None)
    roof, _ = kernel_roofline(timed, a.steps)
    if roof is not None:
        roof["share_of_timed_device_ms"] = pre_roof["ms_per_step"] / max(dev_ms, 1e-9)
        roof["events"] = "HIP events around each launch of this kernel function in the timed steps"
    for h in hs:
        h.close()
    cpu = None
    if not a.no_cpu:
        log("cpu baseline (oracle) ...")
        p, c, N, L, U = max(insts, key=lambda i: i[0].n)
        cpu = cpu_baseline("c2", dict(prob=p, contour=c, N=N, L=L, U=U), a.cpu_nodes, a.cpu_budget)
        cpu["sample"] = cpu["sample"].replace("this workload", f"the largest instance (n={p.n})")
    lat_s = np.array(lat)
    res = {
        "metric": "resolvent samples/sec + eigenpairs/sec at residual<=1e-10; p50/p99 solve latency",
        "value": samples * a.steps / elapsed, "unit": "resolvent samples/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": elapsed / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64" if a.precision == "c64_ir" else "c128",
        "data": "synthetic (seeded)",
        "config": {"workload": "c2", "description": "16 dense QEPs z^2 I + z C + K of uneven order, "
                   "circle centre 10i r=4, N=64, L=32, one batched solve per step", "n": sizes, "N": 64,
                   "L": 32, "precision": a.precision, "nb_autotuned": nb_tuned, "parallelism": "single GPU"},
        "eigenpairs_per_s": sum(n_eig) / elapsed, "n_eig": n_eig[-1],
        "latency_s": {"p50": float(np.percentile(lat_s, 50)), "p99": float(np.percentile(lat_s, 99))},
        "n_eig_per_instance": [o["info"]["n_eig"] for o in outs],
        "kernel_ms_per_step": {k: v["ms"] for k, v in sorted(classes.items(), key=lambda kv: -kv[1]["ms"])},
        "kernel_ms_source": "one batched solve with every kernel timer on, outside the timed steps",
        "roofline": roof, "roofline_next_kernels": roof_next, "cpu_baseline": cpu,
    }
    print(json.dumps(res))


def serve_bench(a, P):
    """Serving workload: a Poisson stream of mixed solves (QEP, delay, BEM,
    random circles, L in {16, 32, 64}) submitted at their arrival times to a
    server with `slots` concurrent slots and an HBM budget; latency is
    arrival to result."""
    import collections

    import nep_inputs as ni
    reqs = ni.config_c4(count=a.requests)
    log(f"serving: {len(reqs)} requests over {reqs[-1]['t']:.2f}s, "
        f"{dict(collections.Counter(r['family'] for r in reqs))}")
    handles, Us = [], []
    for r in reqs:
        handles.append(P.Problem(ni.build_c4_problem(r)))
        Us.append(ni.probing_matrix(r["n"], r["L"], seed=r["useed"]))
    srv = P.Server(int(a.budget_gib * (1 << 30)), a.slots)
    tickets = []
    t0 = time.perf_counter()
    for r, h, U in zip(reqs, handles, Us):
        dt = t0 + r["t"] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        c = r["contour"]
        prm = P.default_params(N=r["N"], L=r["L"], precision="c64_ir")
        tickets.append((time.perf_counter() - t0, srv.submit(h, P.contour(c.center, c.a, c.b), prm, U)))
    lat, n_eig, done, fails = [], 0, 0.0, 0
    warn = collections.Counter()
    for (ts, t), r in zip(tickets, reqs):
        try:
            out, l = srv.wait(t, timeout_s=a.wait_timeout)
        except P.RsrrError as e:
            if e.code == -7:            # bounded wait ended: the message carries the server state
                log(f"request {r['family']} n={r['n']} not finished after {a.wait_timeout:.0f}s: {e}")
                raise SystemExit(3)
            fails += 1
            log(f"request {r['family']} n={r['n']} failed: {e}")
            continue
        lat.append(l)
        n_eig += int(np.sum(out["res"] <= 1e-10))
        st = out["status"]
        warn["rank_saturated"] += bool(st & 1)
        warn["count_mismatch"] += bool(st & 2)
        warn["ir_fallback"] += bool(st & 4)
        warn["no_pair"] += out["info"]["n_eig"] == 0
        done = max(done, ts + l)
        log(f"request {len(lat)}: {r['family']} n={r['n']} L={r['L']} n_eig={out['info']['n_eig']} "
            f"latency {l:.3f}s")
    srv.close()
    for h in handles:
        h.close()
    lat = np.array(lat)
    res = {"metric": "serving: p50/p99 latency (arrival to result), eigenpairs/s at residual<=1e-10",
           "value": n_eig / done, "unit": "eigenpairs/s", "n_gpus": 1, "higher_is_better": True,
           "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                         "max": float(lat.max())},
           "requests": len(reqs), "failed": fails, "requests_per_s": len(lat) / done,
           "wall_s": done, "eigenpairs": n_eig, "warnings": dict(warn),
           "dtype": "c64+f64", "data": "synthetic (seeded)",
           "config": {"workload": "c4", "rate_per_s": 20.0, "slots": a.slots,
                      "budget_gib": a.budget_gib,
                      "mix": dict(collections.Counter(r["family"] for r in reqs))}}
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--precision", default="c64_ir", choices=["c64_ir", "c128"])
    ap.add_argument("--scheme", default="sampling", choices=["sampling", "moment"],
                    help="subspace of Alg. 2 Step 3: sampling matrix (RSRR) or moment matrix (SSRR, K' = N)")
    ap.add_argument("--contour", default="ellipse", choices=["ellipse", "rect"],
                    help="rect: the square inscribed in the workload's circle, Gauss-Legendre sides")
    ap.add_argument("--cpu-nodes", type=int, default=8)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sample-compare", type=int, default=3,
                    help="repetitions of the sampling stage alone in both precisions")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of this many MiB 5 times (reference "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--nb", type=int, default=None,
                    help="LU panel width of the sampling and reduced-problem factorisations (default 64)")
    ap.add_argument("--graph", type=int, default=0, choices=[0, 1],
                    help="capture the sampling launches in a HIP graph replayed by later steps")
    ap.add_argument("--chunk-gib", type=float, default=None,
                    help="device memory per batch of reduced-problem inverses (library default if unset)")
    ap.add_argument("--requests", type=int, default=600, help="serving workload (c4): requests")
    ap.add_argument("--wait-timeout", type=float, default=600.0,
                    help="serving workload (c4): bound of each wait for a result, seconds")
    ap.add_argument("--slots", type=int, default=2, help="serving workload (c4): concurrent slots")
    ap.add_argument("--budget-gib", type=float, default=200.0, help="serving workload (c4): HBM budget")
    ap.add_argument("--traffic-from", nargs=4, default=None,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write profiles/traffic.json from four rocprofv3 --pmc output folders "
                         "(FETCH_SIZE / WRITE_SIZE of the kernel, then of the copy calibration) and exit")
    ap.add_argument("--traffic-kernel", default="gemm_kernel<double, 0, 0, false, true>")
    a = ap.parse_args()
    if a.traffic_from:
        write_traffic(a.traffic_from, a.traffic_kernel, a.copy_calibration or 1024,
                      f"{a.workload}: one solve (bench.py --workload {a.workload} --steps 1 "
                      f"--warmup 0 --no-cpu --sample-compare 0)")
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.copy_calibration > 0:
        nbytes = a.copy_calibration << 20
        x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": nbytes, "launches": 5}))
        return
    import paper_1510_07522_amd as P

    if a.workload == "c4":
        serve_bench(a, P)
        return
    if a.workload == "c2":
        batched_bench(a, P)
        return
    w = workload(a.workload)
    prob, c, N, L = w["prob"], w["contour"], w["N"], w["L"]
    if a.contour == "rect":
        r = min(c.a, c.b) / np.sqrt(2.0)
        w["desc"] += f"; contour: inscribed square, half-side {r:.4f}, Gauss-Legendre sides"
        ct = P.contour(c.center, r, r, kind="rect")
    else:
        ct = P.contour(c.center, c.a, c.b)
    if a.scheme == "moment":
        w["desc"] += "; moment scheme (SSRR), K' = N"
    log(f"workload {a.workload}: {w['desc']}")
    h = P.Problem(prob)
    U = P.to_device(w["U"])
    prm = P.default_params(N=N, L=L, precision=a.precision, scheme=a.scheme, graph=a.graph)
    if a.chunk_gib is not None:
        prm.chunk_gib = a.chunk_gib
    if a.nb is not None:
        prm.nb = a.nb

    for i in range(a.warmup):
        t0 = time.perf_counter()
        out = h.solve(ct, prm, U)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t0:.3f}s n_eig={out['info']['n_eig']}")

    # kernel statistics: one solve with every kernel timer on (outside the
    # timed region; the events cost a few percent of a step)
    P.timers_only(None)
    P.timers_reset()
    P.timers_enable(True)
    h.solve(ct, prm, U)
    torch.cuda.synchronize()
    P.timers_enable(False)
    stats = P.timers_read()
    classes = {k: v for k, v in stats.items() if not k.startswith("sym:")}
    dev_ms = sum(t["ms"] for t in classes.values())
    pre_roof, _ = kernel_roofline(stats, 1)
    dominant = pre_roof["kernel"] if pre_roof else None
    log(f"kernel statistics pass: {dev_ms:.1f} ms of timed device work; dominant kernel {dominant}")

    # timed region: HIP events only around the dominant kernel function (none
    # when the sampling launches replay a captured graph: a capture takes no
    # timer events, so the roofline then comes from the statistics pass)
    P.timers_reset()
    if dominant and not a.graph:
        P.timers_only(dominant)
        P.timers_enable(True)
    lat = []
    n_eig = []
    infos = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(a.steps):
        t0 = time.perf_counter()
        out = h.solve(ct, prm, U)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        n_eig.append(out["info"]["n_eig"])
        infos.append(out["info"])
        log(f"step {i}: {lat[-1]:.3f}s n_eig={n_eig[-1]} res_max="
            f"{(out['res'].max() if len(out['res']) else 0):.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    P.timers_enable(False)
    timed = P.timers_read()
    P.timers_only(None)
    ms_step = elapsed / a.steps * 1e3
    samples_s = N * a.steps / elapsed
    eig_s = sum(n_eig) / elapsed
    roof, _ = kernel_roofline(timed, a.steps) if not a.graph else (pre_roof, None)
    _, roof_next = kernel_roofline(stats, 1)
    if roof is not None:
        roof["share_of_timed_device_ms"] = pre_roof["ms_per_step"] / max(dev_ms, 1e-9)
        roof["events"] = "HIP events around each launch of this kernel function in the timed steps"

    # sampling stage alone, both precisions (the c64 + refinement vs complex128 comparison)
    ws_bound = h.workspace_bound(ct, prm)
    stage = {}
    if a.sample_compare > 0:
        S = P.empty_device(prob.n, N * L)
        for prec in ("c128", "c64_ir"):
            pp = P.default_params(N=N, L=L, precision=prec)
            h.sample(ct, pp, U, S)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.sample_compare):
                _, info, _ = h.sample(ct, pp, U, S)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / a.sample_compare
            stage[prec] = {"samples_per_s": N / dt, "ms": dt * 1e3, "ir_iters": info.ir_iters,
                           "ir_fallback": info.ir_fallback}
            log(f"sampling stage {prec}: {dt * 1e3:.2f} ms ({N / dt:.1f} samples/s)")
        del S
    h.close()

    cpu = None
    if not a.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(a.workload, w, a.cpu_nodes, a.cpu_budget)

    lat_s = np.array(lat)
    res = {
        "metric": "resolvent samples/sec + eigenpairs/sec at residual<=1e-10; p50/p99 solve latency",
        "value": samples_s,
        "unit": "resolvent samples/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64" if a.precision == "c64_ir" else "c128",
        "data": "synthetic (seeded)",
        "config": {"workload": a.workload, "description": w["desc"], "n": prob.n, "N": N, "L": L,
                   "NS": prm.NS, "K": prm.K, "precision": a.precision, "scheme": a.scheme,
                   "contour": a.contour, "nb": int(prm.nb), "graph": a.graph, "parallelism": "single GPU"},
        "eigenpairs_per_s": eig_s,
        "n_eig": n_eig[-1],
        "latency_s": {"p50": float(np.percentile(lat_s, 50)), "p99": float(np.percentile(lat_s, 99))},
        "stages_s": {k: infos[-1][k] for k in ("t_sample", "t_basis", "t_project", "t_reduced",
                                                "t_residual")},
        "solve_info": {k: infos[-1][k] for k in ("k_S", "m", "n_wind", "n_gap", "n_eig",
                                                  "n_candidates", "ir_iters", "ir_fallback")},
        "workspace_bytes": infos[-1]["ws_bytes"],
        "workspace_bound_bytes": ws_bound,
        "sampling_stage": stage,
        "sampling_c64ir_over_c128": (stage["c64_ir"]["samples_per_s"] / stage["c128"]["samples_per_s"]
                                     if len(stage) == 2 else None),
        "kernel_ms_per_step": {k: v["ms"] for k, v in sorted(
            classes.items(), key=lambda kv: -kv[1]["ms"])},
        "kernel_ms_source": "one solve with every kernel timer on, outside the timed steps",
        "roofline": roof,
        "roofline_next_kernels": roof_next,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
