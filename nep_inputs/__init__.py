"""Seeded synthetic inputs for nonlinear eigenvalue problems T(z) v = 0.

This module only *draws* problem data (coefficient matrices, point sets,
probing matrices, contours).  It holds none of the eigensolver's arithmetic:
no quadrature, no factorisation, no projection.  Both the CPU oracle and the
GPU library are fed from here, so that they see bit-identical inputs.

A coefficient-form problem is T(z) = sum_k f_k(z) A_k (coefficient form of the
paper, eq. eq-Z-expr).  Each f_k is described by a small *spec* tuple that both
sides evaluate with their own code:

    ("pow",  c, p)          f(z) = c * z**p
    ("exp",  c, p, tau)     f(z) = c * z**p * exp(tau * z)
    ("rat",  c, p, b)       f(z) = c * z**p / (z - b)
    ("callable", fn)        any f given by a Python function: fn(z) -> (f(z), f'(z))
                            for a complex array z (f'(z) may be None: no derivative)

Each A_k carries a storage kind: "dense" (complex128 n x n, column-major when
flattened), "real" (float64 n x n), "identity" (no data) or "diag" (complex128
length-n vector).

The BEM family (Helmholtz single layer on a sphere) is not in coefficient form;
it is described by its point set and the spacing h.

Random streams use numpy's PCG64 through ``numpy.random.default_rng(seed)``;
the draw order of every family is fixed and documented per function.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "CoeffProblem", "BemProblem", "Contour",
    "probing_matrix", "qep_dense", "qep_diag", "delay_dense", "delay_diag", "sqrt_coupled",
    "bem_sphere", "acoustic_1d", "loaded_string", "viscoelastic_synth",
    "config_c0", "config_c1", "config_c2", "config_c3", "config_small_qep",
    "config_small_delay",
]


@dataclasses.dataclass
class Contour:
    """Closed contour.  kind "ellipse": phi(t) = center + a cos t + i b sin t
    (eq. eq-contour), a the semi-axis along the real direction, b along the
    imaginary one (a circle of radius r has a = b = r).  kind "rect": the
    rectangle center + [-a, a] x i[-b, b] with nh sampling nodes on each
    horizontal side and nv on each vertical side (0, 0: split in proportion to
    the side lengths)."""
    center: complex
    a: float
    b: float
    kind: str = "ellipse"
    nh: int = 0
    nv: int = 0


@dataclasses.dataclass
class CoeffProblem:
    n: int
    kinds: List[str]          # "dense" | "real" | "identity" | "diag"
    mats: List[Optional[np.ndarray]]
    fspecs: List[tuple]
    name: str = ""

    @property
    def J(self) -> int:
        return len(self.kinds)


@dataclasses.dataclass
class BemProblem:
    n: int
    xyz: np.ndarray           # (n, 3) float64 points on the unit sphere
    h: float                  # mean nearest-neighbour spacing
    name: str = ""


def _cgauss(rng: np.random.Generator, shape) -> np.ndarray:
    """i.i.d. (x + i y)/sqrt(2), x, y ~ N(0,1); x drawn first, then y."""
    x = rng.standard_normal(shape)
    y = rng.standard_normal(shape)
    return (x + 1j * y) / math.sqrt(2.0)


def probing_matrix(n: int, L: int, seed: int) -> np.ndarray:
    """Complex Gaussian n x L probing matrix U (Alg. 2, Step 1), Fortran order."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(_cgauss(rng, (n, L)))


# ---------------------------------------------------------------- QEP family
def qep_dense(n: int, kmax: float, seed: int, cscale: float = 0.05) -> CoeffProblem:
    """T(z) = z^2 I + z C + K with K = diag(k), k ~ U[1, kmax],
    C = cscale * (X + iY)/sqrt(2)/sqrt(n).  Draw order: k, then X, then Y."""
    rng = np.random.default_rng(seed)
    k = rng.uniform(1.0, kmax, size=n)
    G = _cgauss(rng, (n, n)) / math.sqrt(n)
    C = np.asfortranarray(cscale * G)
    return CoeffProblem(
        n=n, kinds=["identity", "dense", "diag"],
        mats=[None, C, k.astype(np.complex128)],
        fspecs=[("pow", 1.0, 2), ("pow", 1.0, 1), ("pow", 1.0, 0)],
        name=f"qep_dense(n={n},kmax={kmax},seed={seed})")


def qep_diag(m: np.ndarray, c: np.ndarray, k: np.ndarray) -> CoeffProblem:
    """Diagonal QEP T(z) = z^2 diag(m) + z diag(c) + diag(k) (closed-form roots)."""
    n = len(k)
    return CoeffProblem(
        n=n, kinds=["diag", "diag", "diag"],
        mats=[np.asarray(m, np.complex128), np.asarray(c, np.complex128),
              np.asarray(k, np.complex128)],
        fspecs=[("pow", 1.0, 2), ("pow", 1.0, 1), ("pow", 1.0, 0)],
        name=f"qep_diag(n={n})")


# -------------------------------------------------------------- delay family
def delay_dense(n: int, seed: int) -> CoeffProblem:
    """T(z) = -z I + A0 + A1 exp(-z); A0, A1 real N(0,1)/sqrt(n), A0 drawn first."""
    rng = np.random.default_rng(seed)
    A0 = np.asfortranarray(rng.standard_normal((n, n)) / math.sqrt(n))
    A1 = np.asfortranarray(rng.standard_normal((n, n)) / math.sqrt(n))
    return CoeffProblem(
        n=n, kinds=["identity", "real", "real"], mats=[None, A0, A1],
        fspecs=[("pow", -1.0, 1), ("pow", 1.0, 0), ("exp", 1.0, 0, -1.0)],
        name=f"delay_dense(n={n},seed={seed})")


def delay_diag(a: np.ndarray, b: np.ndarray) -> CoeffProblem:
    """T(z) = -z I + diag(a) + diag(b) exp(-z) (roots via Lambert W)."""
    n = len(a)
    return CoeffProblem(
        n=n, kinds=["identity", "diag", "diag"],
        mats=[None, np.asarray(a, np.complex128), np.asarray(b, np.complex128)],
        fspecs=[("pow", -1.0, 1), ("pow", 1.0, 0), ("exp", 1.0, 0, -1.0)],
        name=f"delay_diag(n={n})")


def sqrt_coupled(n: int, seed: int, derivatives: bool = True) -> CoeffProblem:
    """T(z) = -z I + A0 + sqrt(z + 4) A1 (principal branch, cut on (-inf, -4]),
    A0, A1 real N(0,1)/sqrt(n) drawn in that order: a coefficient form whose
    third scalar function is outside the pow/exp/rat menu, given as Python
    functions ("callable" specs; without derivatives when derivatives=False)."""
    rng = np.random.default_rng(seed)
    A0 = np.asfortranarray(rng.standard_normal((n, n)) / math.sqrt(n))
    A1 = np.asfortranarray(rng.standard_normal((n, n)) / math.sqrt(n))

    def f0(z):
        return -z, (-np.ones_like(z) if derivatives else None)

    def f1(z):
        return np.ones_like(z), (np.zeros_like(z) if derivatives else None)

    def f2(z):
        r = np.sqrt(z + 4.0)
        return r, (0.5 / r if derivatives else None)
    return CoeffProblem(
        n=n, kinds=["identity", "real", "real"], mats=[None, A0, A1],
        fspecs=[("callable", f0), ("callable", f1), ("callable", f2)],
        name=f"sqrt_coupled(n={n},seed={seed},derivatives={derivatives})")


# ---------------------------------------------------------------- BEM family
def bem_sphere(n: int) -> BemProblem:
    """Fibonacci points on the unit sphere: z_i = 1 - (2i+1)/n,
    r_i = sqrt(1 - z_i^2), phi_i = i * pi * (3 - sqrt 5); h is the mean
    nearest-neighbour distance (brute force, chunked)."""
    i = np.arange(n, dtype=np.float64)
    zc = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - zc * zc))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    xyz = np.stack([r * np.cos(phi), r * np.sin(phi), zc], axis=1)
    nn = np.empty(n)
    step = 1024
    for s in range(0, n, step):
        d2 = ((xyz[s:s + step, None, :] - xyz[None, :, :]) ** 2).sum(-1)
        d2[np.arange(d2.shape[0]), np.arange(s, min(s + step, n))] = np.inf
        nn[s:s + step] = np.sqrt(d2.min(axis=1))
    return BemProblem(n=n, xyz=np.ascontiguousarray(xyz), h=float(nn.mean()),
                      name=f"bem_sphere(n={n})")


# ------------------------------------------------- the paper's own examples
def acoustic_1d(n: int = 1000, zeta: float = 1.0) -> CoeffProblem:
    """Acoustic-1D QEP (Sec. 'Three benchmark examples'): T = z^2 M + z C + Ks,
    M = -(4 pi^2/n)(I - e_n e_n^T / 2), C = (2 pi i/zeta) e_n e_n^T,
    Ks = n * tridiag(-1, 2, -1) with last diagonal entry 1."""
    M = np.full(n, -4.0 * math.pi ** 2 / n, dtype=np.complex128)
    M[-1] *= 0.5
    Cd = np.zeros(n, np.complex128)
    Cd[-1] = 2.0j * math.pi / zeta
    K = np.zeros((n, n))
    K[np.arange(n), np.arange(n)] = 2.0 * n
    K[np.arange(n - 1), np.arange(1, n)] = -1.0 * n
    K[np.arange(1, n), np.arange(n - 1)] = -1.0 * n
    K[-1, -1] = 1.0 * n
    return CoeffProblem(
        n=n, kinds=["diag", "diag", "real"], mats=[M, Cd, np.asfortranarray(K)],
        fspecs=[("pow", 1.0, 2), ("pow", 1.0, 1), ("pow", 1.0, 0)],
        name=f"acoustic_1d(n={n})")


def loaded_string(n: int = 5000, last_diag_t1: float = 1.0) -> CoeffProblem:
    """Loaded string rational NEP: T = T1 + z/(z-1) e_n e_n^T - z T3,
    T1 = n tridiag(-1, 2, -1) (last diagonal entry last_diag_t1 * n),
    T3 = (1/(6n)) tridiag(1, 4, 1) with last diagonal entry 2/(6n)."""
    T1 = np.zeros((n, n))
    T1[np.arange(n), np.arange(n)] = 2.0 * n
    T1[np.arange(n - 1), np.arange(1, n)] = -1.0 * n
    T1[np.arange(1, n), np.arange(n - 1)] = -1.0 * n
    T1[-1, -1] = last_diag_t1 * n
    T3 = np.zeros((n, n))
    T3[np.arange(n), np.arange(n)] = 4.0 / (6.0 * n)
    T3[np.arange(n - 1), np.arange(1, n)] = 1.0 / (6.0 * n)
    T3[np.arange(1, n), np.arange(n - 1)] = 1.0 / (6.0 * n)
    T3[-1, -1] = 2.0 / (6.0 * n)
    E = np.zeros(n, np.complex128)
    E[-1] = 1.0
    return CoeffProblem(
        n=n, kinds=["real", "diag", "real"],
        mats=[np.asfortranarray(T1), E, np.asfortranarray(T3)],
        fspecs=[("pow", 1.0, 0), ("rat", 1.0, 1, 1.0), ("pow", -1.0, 1)],
        name=f"loaded_string(n={n})")


def viscoelastic_synth(n: int, seed: int) -> CoeffProblem:
    """Synthetic viscoelastic NEP T = z^2 M + G(z) Kv + Ks with the paper's
    three-term Biot modulus G(z) = Ginf * sum_k a_k z/(z + b_k) (eq.
    eq-ne-dampingmodel), split into three rational terms sharing Kv.  M, Ks, Kv
    are random SPD matrices (draw order: M, Ks, Kv), scaled so that the
    undamped spectrum lies in the paper's frequency band."""
    rng = np.random.default_rng(seed)

    def spd(scale):
        X = rng.standard_normal((n, n)) / math.sqrt(n)
        return np.asfortranarray(scale * (X @ X.T + np.eye(n)))

    M = spd(1.0)
    Ks = spd(1.0e5)
    Kv = spd(1.0e-1)
    ginf = 3.441e5
    a = (2.06, 67.1985, 506.9457)
    b = (193.39, 16345.0, 485918.4)
    kinds = ["real", "real"] + ["real"] * 3
    mats = [M, Ks, Kv, Kv, Kv]
    fspecs = [("pow", 1.0, 2), ("pow", 1.0, 0)] + [
        ("rat", ginf * ak, 1, -bk) for ak, bk in zip(a, b)]
    return CoeffProblem(n=n, kinds=kinds, mats=mats, fspecs=fspecs,
                        name=f"viscoelastic_synth(n={n},seed={seed})")


# ------------------------------------------------------ benchmark workloads
def config_c0():
    """Dense complex QEP, n=200, circle centre 5i radius 2, N=32, L=20."""
    p = qep_dense(200, 100.0, seed=1000)
    return p, Contour(5j, 2.0, 2.0), 32, 20, probing_matrix(200, 20, seed=2000)


def config_c1(n: int = 2048):
    """Dense delay NEP, n=2048, circle centre 0 radius 3, N=48, L=48."""
    p = delay_dense(n, seed=1001)
    return p, Contour(0.0, 3.0, 3.0), 48, 48, probing_matrix(n, 48, seed=2001)


def config_c2(count: int = 16, nmin: int = 512, nmax: int = 4096):
    """Sixteen dense QEPs of uneven size (k ~ U[1,400]), circle 10i radius 4,
    N=64, L=32.  The sizes are drawn first from one stream."""
    rng = np.random.default_rng(1002)
    sizes = rng.integers(nmin, nmax + 1, size=count)
    out = []
    for i, n in enumerate(sizes):
        n = int(n)
        p = qep_dense(n, 400.0, seed=3000 + i)
        out.append((p, Contour(10j, 4.0, 4.0), 64, 32,
                    probing_matrix(n, 32, seed=4000 + i)))
    return out


def config_c4(count: int = 600, rate: float = 20.0, seed: int = 1004):
    """Request stream of the serving workload: Poisson arrivals (exponential
    gaps, `rate` per second); family uniform over
      QEP   n ~ U{256..4096}, N = 32, k ~ U[1,100], centre i U[2,9], radius U[0.5,2]
      delay n ~ U{512..2048}, N = 48, centre uniform in |c| <= 1, radius U[0.5,1.5]
      BEM   n ~ U{1024..4096}, N = 40, centre U[2.5,4.0] (real), radius U[0.3,0.8]
    and L uniform in {16, 32, 64}.  Returns dicts with the arrival time, the
    family, n, a problem seed, the contour, N, L and the seed of U; problems
    are built by the caller (build_c4_problem) so that they can be cached."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        fam = ("qep", "delay", "bem")[int(rng.integers(0, 3))]
        L = int((16, 32, 64)[int(rng.integers(0, 3))])
        if fam == "qep":
            n, N = int(rng.integers(256, 4097)), 32
            c = Contour(1j * rng.uniform(2.0, 9.0), *([rng.uniform(0.5, 2.0)] * 2))
        elif fam == "delay":
            n, N = int(rng.integers(512, 2049)), 48
            rad, ang = math.sqrt(rng.uniform()), rng.uniform(0, 2 * math.pi)
            c = Contour(rad * complex(math.cos(ang), math.sin(ang)), *([rng.uniform(0.5, 1.5)] * 2))
        else:
            n, N = int(rng.integers(1024, 4097)), 40
            c = Contour(complex(rng.uniform(2.5, 4.0)), *([rng.uniform(0.3, 0.8)] * 2))
        out.append(dict(t=t, family=fam, n=n, pseed=5000 + i, contour=c, N=N, L=L, useed=6000 + i))
    return out


def build_c4_problem(req):
    """The problem of one serving request (see config_c4)."""
    if req["family"] == "qep":
        return qep_dense(req["n"], 100.0, seed=req["pseed"])
    if req["family"] == "delay":
        return delay_dense(req["n"], seed=req["pseed"])
    return bem_sphere(req["n"])


def config_c3(n: int = 8192):
    """Helmholtz single-layer BEM on a Fibonacci sphere, ellipse centre 3,
    semi-axes 1.5 and 0.3, N=40, L=64."""
    p = bem_sphere(n)
    return p, Contour(3.0, 1.5, 0.3), 40, 64, probing_matrix(n, 64, seed=2003)


def config_small_qep(n: int = 48, seed: int = 7):
    """A C0-shaped QEP small enough for brute-force checks."""
    p = qep_dense(n, 100.0, seed=seed)
    return p, Contour(5j, 2.0, 2.0), 16, 8, probing_matrix(n, 8, seed=seed + 1)


def config_small_delay(n: int = 32, seed: int = 11):
    """A C1-shaped delay problem small enough for brute-force checks."""
    p = delay_dense(n, seed=seed)
    return p, Contour(0.0, 1.5, 1.5), 24, 8, probing_matrix(n, 8, seed=seed + 1)
