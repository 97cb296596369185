"""Writes the oracle's results at the benchmark sizes to tests/golden/.

Calls only ``oracle`` (the plain FP64 CPU implementation of Alg. 2 around
Alg. 1) and ``nep_inputs`` (the seeded generators).  For each workload it
stores the eigenvalues strictly inside the contour that the oracle extracts
(all candidates, with their residuals ||T(l)v|| / (||T(l)||_F ||v||), so that
a later cut at any tolerance can be taken from the file), the count at the
default acceptance level 1e-10, the winding integral (eq. eq-ncs), the gap
count (eq. eq-gap), the retained Hankel rank m, the basis dimension k_S
(Alg. 2 Step 3) and the oracle's wall time on this host.

Usage:  python tests/golden/make_oracle_golden.py c1 c3 c2_723 c2_1183 [c0]
Each workload takes minutes (c1, c3: the oracle's 512 reduced LU solves of
order k_S, or 40 LU solves of order 8192); results go to
tests/golden/oracle_<name>.json.
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import nep_inputs as ni  # noqa: E402
from oracle import rsrr_ref as R  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
TOL_RES = 1e-10


def workloads():
    """name -> (description, problem, contour, N, L, U)."""
    def c2(n):
        for p, c, N, L, U in ni.config_c2():
            if p.n == n:
                return (f"batched-QEP instance n={n} (16 QEPs of uneven size, k ~ U[1,400], "
                        f"circle centre 10i radius 4, N=64, L=32)", p, c, N, L, U)
        raise KeyError(n)
    return {
        "c0": lambda: ("dense QEP z^2 I + z C + K, n=200, circle centre 5i r=2, N=32, L=20",
                       *ni.config_c0()),
        "c1": lambda: ("delay NEP -zI + A0 + A1 exp(-z), n=2048, circle |z|<3, N=48, L=48",
                       *ni.config_c1()),
        "c3": lambda: ("Helmholtz BEM sphere n=8192, ellipse centre 3 (1.5, 0.3), N=40, L=64, "
                       "Chebyshev degree 40", *ni.config_c3()),
        "c2_723": lambda: c2(723),
        "c2_1183": lambda: c2(1183),
    }


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def run(name: str):
    desc, p, c, N, L, U = workloads()[name]()
    print(f"[golden] {name}: {desc}", flush=True)
    t0 = time.perf_counter()
    # every extracted eigenvalue inside the contour, with its residual
    out = R.rsrr(p, c, N, L, U, tol_res=np.inf)
    dt = time.perf_counter() - t0
    lam, res = out["lam"], out["res"]
    keep = res <= TOL_RES
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 0) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    rec = {
        "workload": name,
        "description": desc,
        "n": int(p.n), "N": int(N), "L": int(L), "NS": 512, "K": 2, "delta": 1e-14,
        "hankel_tol": 1e-13, "tol_res": TOL_RES,
        "k_S": int(out["kS"]), "m": int(out["m"]), "n_gap": int(out["n_gap"]),
        "wind": [float(out["wind"].real), float(out["wind"].imag)],
        "n_wind": int(out["n_wind"]),
        "n_candidates": int(len(lam)),
        "count": int(keep.sum()),
        # candidates sorted by (Re, Im): [re, im, residual]
        "candidates": [[float(l.real), float(l.imag), float(r)] for l, r in zip(lam, res)],
        "sigma_S_first_last": [float(out["sigma_S"][0]), float(out["sigma_S"][-1])],
        "oracle_seconds": dt,
        "host": {"cpu": cpu_model(), "os_cpu_count": os.cpu_count(), "blas_threads": threads,
                 "numpy": np.__version__},
        "writer": "tests/golden/make_oracle_golden.py (oracle.rsrr_ref.rsrr with tol_res=inf)",
    }
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=0)
    print(f"[golden] {name}: k_S={rec['k_S']} m={rec['m']} n_wind={rec['n_wind']} "
          f"candidates={rec['n_candidates']} count={rec['count']} in {dt:.1f}s -> {path}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["c0"]
    for nm in names:
        run(nm)
