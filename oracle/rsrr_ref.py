"""Plain, slow FP64 CPU oracle of the resolvent-sampling Rayleigh-Ritz method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the GPU library: it reads problem data
from ``nep_inputs`` (seeded generators, no solver arithmetic) and does every
step of the method itself, in complex128, with NumPy/SciPy-LAPACK primitives
(``solve`` = LU with partial pivoting, ``svd``, ``eig``) as single steps.

Method (Xiao, Meng, Zhang, Zheng, "Resolvent sampling based Rayleigh-Ritz
method for large-scale nonlinear eigenvalue problems", arXiv 1510.07522):

  Alg. 2 (RSRR)
    Step 1  contour, N, L, random U, sampling nodes z_i            contour_quadrature
    Step 2  Y_i = T(z_i)^{-1} U                                     sample_resolvent
    Step 3  S_hat = [Y_0 ... Y_{N-1}] (eq. eq-hatS), truncated SVD  truncated_basis
    Step 4  T_S(z) = S^H T(z) S (eq. eq-Ts-NEP, eq-Zs-expr)         project_coefficients
            (BEM: Chebyshev interpolation, eq. eq-Ts-coefs,         chebyshev_projection
             or the interpolant on a circle, R14)                   circle_projection
            reduced NEP by Alg. 1                                   solve_reduced
    Step 5  v = S g                                                 rsrr
  Alg. 1 (modified block Sakurai-Sugiura)
    Step 2  moments A_alpha of T_S^{-1} (eq. eq-Ap, eq-Ap-num),
            Hankel H, H^< (eq. eq-HH)                               reduced_moments, hankel
    Step 3  SVD of H (eq. eq-svdH), count by winding number
            (eq. eq-ncs) and by singular-value gap (eq. eq-gap)     count_gap
    Step 4  A = V0^H H^< W0 S0^-1 (eq. eq-A), eig, recovery
            (eq. eq-eigens)                                         extract_pairs

Readings taken where the paper is silent or ambiguous (each is listed in the
design notes with its reason):
  R1  trapezoid angles theta_j = 2 pi (j + 1/2)/N for j = 0..N-1 (N points).
  R2  a, b are the real and imaginary semi-axes; rho = max(a, b).
  R3  "larger than delta sigma_1" is strict; Ŝ is not column-scaled.
  R4  the gap search runs over j = 1..len(sigma)-1 restricted to
      sigma_{j+1} > 10 u len(sigma) sigma_1; ties go to the smallest j.
  R5  the Hankel truncation keeps every singular value above
      hankel_tol * sigma_1; all extracted eigenvalues strictly inside the
      contour whose residual is at most tol_res are returned.  The winding
      and gap counts are reported beside the final count.
  R6  the Chebyshev coefficient P_0 carries weight 1/(d+1) (standard
      interpolant), the interval is [center - a, center + a].
  R7  residual = ||T(l) v||_2 / (||T(l)||_F ||v||_2); the paper's
      ||T(l) v||_2 / ||v||_2 is reported too.
  R8  eigenvectors are scaled to unit 2-norm with the entry of largest modulus
      real and positive.
  R12 rectangular contours (the paper's Sec. 7 examples): Gauss-Legendre
      nodes on each side, counter-clockwise from the lower-left corner
      (bottom, right, top, left); the sampling split (nh per horizontal side,
      nv per vertical side) is given, or N/2 is split in proportion to the
      side lengths, nh = round(N/2 a/(a+b)) clamped to [1, N/2-1]; the moment
      nodes are always split that way.  Moments and the winding number use
      the quadrature weights dz/(2 pi i) and rho = max(a, b) as for the
      ellipse.
  R14 matrices without a coefficient form (BEM) are interpolated in z
      (Sec. 6.2): on the Chebyshev points of [center - a, center + a] when
      the contour hugs that interval (b <= a/4), otherwise on d+1 equispaced
      points of a circle around the contour, in the basis ((z-center)/R)^j.
  R13 the moment scheme (SSRR, Sec. 3.1-3.2) uses the shifted and scaled
      monomials s^alpha, s = (z - gamma)/rho, as the paper's own moment
      formula eq. eq-Ap-num does; over alpha < K' they span the same
      polynomials as z^alpha, so span(M_hat) is unchanged in exact arithmetic.
      The weights are the contour's dz/(2 pi i); K' = N by default (the
      paper's comparisons use K' = N).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np
import scipy.linalg as sla

from nep_inputs import BemProblem, CoeffProblem, Contour

U_ROUND = np.finfo(np.float64).eps / 2.0


# --------------------------------------------------------------------------
# Problem evaluation: T(z) and T'(z) from the coefficient form (eq. eq-Z-expr)
# or from the BEM kernel entries (cf. eq. eq-nyes).
# --------------------------------------------------------------------------
def eval_scalar(spec: tuple, z):
    """f(z) and f'(z) for one scalar-function spec (see nep_inputs)."""
    z = np.asarray(z, dtype=np.complex128)
    kind = spec[0]
    if kind == "pow":
        c, p = complex(spec[1]), int(spec[2])
        f = c * z ** p
        df = c * p * z ** (p - 1) if p > 0 else np.zeros_like(z)
        return f, df
    if kind == "exp":
        c, p, tau = complex(spec[1]), int(spec[2]), complex(spec[3])
        e = np.exp(tau * z)
        f = c * z ** p * e
        dzp = p * z ** (p - 1) if p > 0 else np.zeros_like(z)
        df = c * e * (dzp + tau * z ** p)
        return f, df
    if kind == "callable":
        # a caller-supplied scalar function (any f_k of the coefficient form)
        f, df = spec[1](z)
        f = np.asarray(f, np.complex128)
        df = np.full_like(f, np.nan) if df is None else np.asarray(df, np.complex128)
        return f, df
    if kind == "rat":
        c, p, b = complex(spec[1]), int(spec[2]), complex(spec[3])
        f = c * z ** p / (z - b)
        dzp = p * z ** (p - 1) if p > 0 else np.zeros_like(z)
        df = c * (dzp * (z - b) - z ** p) / (z - b) ** 2
        return f, df
    raise ValueError(f"unknown scalar function kind {kind!r}")


def dense_coefficient(prob: CoeffProblem, k: int) -> np.ndarray:
    kind, A = prob.kinds[k], prob.mats[k]
    if kind == "identity":
        return np.eye(prob.n, dtype=np.complex128)
    if kind == "diag":
        return np.diag(np.asarray(A, np.complex128))
    return np.asarray(A, np.complex128)


def bem_matrix(prob: BemProblem, z: complex, derivative: bool = False) -> np.ndarray:
    """Helmholtz single-layer entries exp(i z r)/(4 pi r) off the diagonal and
    i z/(4 pi) + 1/(2h) on it (derivative=True gives dT/dz)."""
    x = prob.xyz
    r = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    n = prob.n
    np.fill_diagonal(r, 1.0)
    if derivative:
        T = 1j * np.exp(1j * z * r) / (4.0 * math.pi)
        np.fill_diagonal(T, 1j / (4.0 * math.pi))
    else:
        T = np.exp(1j * z * r) / (4.0 * math.pi * r)
        np.fill_diagonal(T, 1j * z / (4.0 * math.pi) + 1.0 / (2.0 * prob.h))
    return T.astype(np.complex128)


def T_matrix(prob, z: complex) -> np.ndarray:
    """T(z) as a dense complex128 matrix."""
    if isinstance(prob, BemProblem):
        return bem_matrix(prob, z)
    T = np.zeros((prob.n, prob.n), np.complex128)
    for k in range(prob.J):
        f, _ = eval_scalar(prob.fspecs[k], z)
        T += complex(f) * dense_coefficient(prob, k)
    return T


def dT_matrix(prob, z: complex) -> np.ndarray:
    if isinstance(prob, BemProblem):
        return bem_matrix(prob, z, derivative=True)
    T = np.zeros((prob.n, prob.n), np.complex128)
    for k in range(prob.J):
        _, df = eval_scalar(prob.fspecs[k], z)
        T += complex(df) * dense_coefficient(prob, k)
    return T


# --------------------------------------------------------------------------
# Alg. 2, Step 1: contour and sampling nodes (eq. eq-contour, eq-Ap-num).
# --------------------------------------------------------------------------
def contour_nodes(c: Contour, N: int):
    """Angles theta_j = 2 pi (j+1/2)/N, nodes phi(theta_j) and phi'(theta_j)."""
    theta = 2.0 * math.pi * (np.arange(N) + 0.5) / N
    z = c.center + c.a * np.cos(theta) + 1j * c.b * np.sin(theta)
    dz = -c.a * np.sin(theta) + 1j * c.b * np.cos(theta)
    return theta, z.astype(np.complex128), dz.astype(np.complex128)


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [-1, 1]: the nodes are the eigenvalues of
    the symmetric tridiagonal Jacobi matrix of the Legendre polynomials
    (off-diagonal k / sqrt(4k^2 - 1)), polished by two Newton steps on P_n;
    the weights are 2 / ((1 - x^2) P_n'(x)^2)."""
    if n == 1:
        return np.zeros(1), np.full(1, 2.0)
    k = np.arange(1, n)
    x = sla.eigvalsh_tridiagonal(np.zeros(n), k / np.sqrt(4.0 * k * k - 1.0))

    def p_and_dp(t):
        p_prev, p = np.ones_like(t), t.copy()
        for j in range(2, n + 1):
            p_prev, p = p, ((2 * j - 1) * t * p - (j - 1) * p_prev) / j
        return p, n * (t * p - p_prev) / (t * t - 1.0)

    for _ in range(2):
        p, dp = p_and_dp(x)
        x = x - p / dp
    x = np.sort(x)
    x = 0.5 * (x - x[::-1])                       # exact symmetry
    _, dp = p_and_dp(x)
    w = 2.0 / ((1.0 - x) * (1.0 + x) * dp * dp)
    w = 0.5 * (w + w[::-1])
    return x, w


def rect_split(c: Contour, N: int, sampling: bool):
    """Nodes per horizontal and per vertical side of a rectangle (R12)."""
    if sampling and (c.nh or c.nv):
        assert c.nh > 0 and c.nv > 0 and N == 2 * (c.nh + c.nv), "N = 2 (nh + nv)"
        return c.nh, c.nv
    assert N >= 4 and N % 2 == 0, "rectangle needs an even node count >= 4"
    half = N // 2
    nh = min(max(int(math.floor(half * c.a / (c.a + c.b) + 0.5)), 1), half - 1)
    return nh, half - nh


def contour_quadrature(c: Contour, N: int, sampling: bool = True):
    """Nodes z_j and weights dz_j with  integral of g(z) dz ~ sum_j dz_j g(z_j).
    Ellipse: trapezoid rule in theta, dz_j = (2 pi / N) phi'(theta_j).
    Rectangle: Gauss-Legendre on each side (R12)."""
    if c.kind == "ellipse":
        _, z, dphi = contour_nodes(c, N)
        return z, (2.0 * math.pi / N) * dphi
    assert c.kind == "rect"
    nh, nv = rect_split(c, N, sampling)
    g, a, b = complex(c.center), c.a, c.b
    z, dz = [], []
    # (midpoint, half-side vector) of bottom, right, top, left, counter-clockwise
    for mid, half, cnt in ((g - 1j * b, a, nh), (g + a, 1j * b, nv),
                           (g + 1j * b, -a, nh), (g - a, -1j * b, nv)):
        x, w = gauss_legendre(cnt)
        z.append(mid + half * x)
        dz.append(half * w)
    return np.concatenate(z).astype(np.complex128), np.concatenate(dz).astype(np.complex128)


def inside(c: Contour, lam) -> np.ndarray:
    lam = np.asarray(lam, np.complex128)
    xr = (lam.real - np.real(c.center)) / c.a
    xi = (lam.imag - np.imag(c.center)) / c.b
    if c.kind == "rect":
        return (np.abs(xr) < 1.0) & (np.abs(xi) < 1.0)
    return xr ** 2 + xi ** 2 < 1.0


# --------------------------------------------------------------------------
# Alg. 2, Step 2: probed resolvent at the sampling nodes (eq. eq-hatS).
# --------------------------------------------------------------------------
def sample_resolvent(prob, z_nodes, U: np.ndarray) -> np.ndarray:
    """S_hat = [T(z_0)^{-1} U, ..., T(z_{N-1})^{-1} U]; each block by LU with
    partial pivoting."""
    n, L = U.shape
    S_hat = np.empty((n, len(z_nodes) * L), np.complex128, order="F")
    for i, zi in enumerate(z_nodes):
        S_hat[:, i * L:(i + 1) * L] = sla.solve(T_matrix(prob, zi), U)
    return S_hat


def moment_matrix(S_hat: np.ndarray, c: Contour, N: int, L: int, Kp: int) -> np.ndarray:
    """Moment scheme (SSRR): M_hat = [M_0 ... M_{K'-1}] with
    M_alpha = sum_i w_i s_i^alpha T(z_i)^{-1} U (eq. eq-malpha-qud, eq-hatM),
    w_i = dz_i / (2 pi i), s_i = (z_i - gamma)/rho (R13); the same matrix as
    S_hat D Z (eq. eq-hatMS)."""
    z, dz = contour_quadrature(c, N, sampling=True)
    rho = max(c.a, c.b)
    w = dz / (2j * math.pi)
    s = (z - c.center) / rho
    n = S_hat.shape[0]
    M = np.zeros((n, Kp * L), np.complex128, order="F")
    for alpha in range(Kp):
        for i in range(N):
            M[:, alpha * L:(alpha + 1) * L] += (w[i] * s[i] ** alpha) * S_hat[:, i * L:(i + 1) * L]
    return M


# --------------------------------------------------------------------------
# Alg. 2, Step 3: truncated SVD basis (delta rule of the parameter guidance).
# --------------------------------------------------------------------------
def numerical_rank(sigma: np.ndarray, tol: float) -> int:
    """Number of singular values strictly larger than tol * sigma_1."""
    if len(sigma) == 0 or sigma[0] == 0.0:
        return 0
    return int(np.count_nonzero(sigma > tol * sigma[0]))


def truncated_basis(S_hat: np.ndarray, delta: float = 1e-14):
    """Left singular vectors of S_hat whose singular values exceed delta*s1."""
    Uq, sigma, _ = sla.svd(S_hat, full_matrices=False, lapack_driver="gesdd")
    kS = numerical_rank(sigma, delta)
    return np.asfortranarray(Uq[:, :kS]), sigma, kS


# --------------------------------------------------------------------------
# Alg. 2, Step 4: reduced coefficients (eq. eq-Zs-expr) and the Chebyshev
# variant for matrices without a coefficient form (eq. eq-Ts-coefs).
# --------------------------------------------------------------------------
def project_coefficients(prob: CoeffProblem, S: np.ndarray) -> List[np.ndarray]:
    SH = S.conj().T
    return [SH @ dense_coefficient(prob, k) @ S for k in range(prob.J)]


def chebyshev_nodes(d: int):
    theta = (np.arange(d + 1) + 0.5) * math.pi / (d + 1)
    return theta, np.cos(theta)


def chebyshev_projection(prob, S: np.ndarray, center: float, a: float, d: int):
    """P_hat_j for j = 0..d from S^H T(x_k) S at the d+1 first-kind Chebyshev
    points x_k mapped onto [center - a, center + a]."""
    theta, t = chebyshev_nodes(d)
    SH = S.conj().T
    proj = [SH @ T_matrix(prob, center + a * tk) @ S for tk in t]
    P = []
    for j in range(d + 1):
        w = (1.0 if j == 0 else 2.0) / (d + 1)
        P.append(w * sum(np.cos(j * theta[k]) * proj[k] for k in range(d + 1)))
    return P


def chebyshev_values(t, d: int):
    """tau_0..tau_d and their t-derivatives at a (complex) point t."""
    tau = np.zeros(d + 1, np.complex128)
    dtau = np.zeros(d + 1, np.complex128)
    tau[0] = 1.0
    if d >= 1:
        tau[1] = t
        dtau[1] = 1.0
    for j in range(2, d + 1):
        tau[j] = 2.0 * t * tau[j - 1] - tau[j - 2]
        dtau[j] = 2.0 * tau[j - 1] + 2.0 * t * dtau[j - 1] - dtau[j - 2]
    return tau, dtau


class ReducedNEP:
    """T_S(z) = sum_j B_j g_j(z) with its derivative (coefficient or Chebyshev)."""

    def __init__(self, B: List[np.ndarray], scal):
        self.B = B
        self.scal = scal            # z -> (g(z) array, g'(z) array)

    @property
    def k(self) -> int:
        return self.B[0].shape[0]

    def T(self, z):
        g, _ = self.scal(z)
        return sum(gj * Bj for gj, Bj in zip(g, self.B))

    def dT(self, z):
        _, dg = self.scal(z)
        return sum(dgj * Bj for dgj, Bj in zip(dg, self.B))


def reduced_from_coefficients(prob: CoeffProblem, S: np.ndarray) -> ReducedNEP:
    B = project_coefficients(prob, S)

    def scal(z):
        vals = [eval_scalar(s, z) for s in prob.fspecs]
        return (np.array([v[0] for v in vals], np.complex128),
                np.array([v[1] for v in vals], np.complex128))
    return ReducedNEP(B, scal)


def circle_projection(prob, S: np.ndarray, center: complex, R: float, d: int):
    """P_hat_j, j = 0..d, of the interpolant T_S(z) ~ sum_j P_hat_j s^j,
    s = (z - center)/R, through the d+1 equispaced points z_k = center +
    R w^k, w = exp(2 pi i/(d+1)) (R14): P_hat_j = (1/(d+1)) sum_k w^(-jk)
    S^H T(z_k) S, the discrete Fourier transform of the samples."""
    nd = d + 1
    SH = S.conj().T
    zk = center + R * np.exp(2j * math.pi * np.arange(nd) / nd)
    proj = [SH @ T_matrix(prob, z) @ S for z in zk]
    P = []
    for j in range(nd):
        P.append(sum(np.exp(-2j * math.pi * j * k / nd) * proj[k] for k in range(nd)) / nd)
    return P


def reduced_from_circle(prob, S, center: complex, R: float, d: int) -> ReducedNEP:
    P = circle_projection(prob, S, center, R, d)

    def scal(z):
        s = (z - center) / R
        g = s ** np.arange(d + 1)
        dg = np.zeros(d + 1, np.complex128)
        dg[1:] = np.arange(1, d + 1) * s ** np.arange(d) / R
        return g.astype(np.complex128), dg
    return ReducedNEP(P, scal)


def interpolation_kind(c: Contour, interp: str = "auto") -> str:
    """R14: the Chebyshev interpolant on [center - a, center + a] (the paper's)
    for contours that hug that interval (b <= a/4); otherwise the interpolant
    through equispaced points of a circle around the contour (radius max(a, b)
    for an ellipse, sqrt(a^2 + b^2) for a rectangle).  A Chebyshev series
    evaluated a distance of order a off its interval multiplies the rounding
    of its high coefficients by |tau_j| ~ (1 + sqrt 2)^j."""
    if interp != "auto":
        return interp
    return "chebyshev" if c.b <= 0.25 * c.a else "circle"


def circle_radius(c: Contour) -> float:
    return math.hypot(c.a, c.b) if c.kind == "rect" else max(c.a, c.b)


def reduced_from_chebyshev(prob, S, center: float, a: float, d: int) -> ReducedNEP:
    P = chebyshev_projection(prob, S, center, a, d)

    def scal(z):
        tau, dtau = chebyshev_values((z - center) / a, d)
        return tau, dtau / a
    return ReducedNEP(P, scal)


# --------------------------------------------------------------------------
# Alg. 1: modified block SS for the reduced NEP.
# --------------------------------------------------------------------------
def reduced_moments(red: ReducedNEP, c: Contour, NS: int, K: int):
    """Moments A_alpha, alpha < 2K, of T_S^{-1} by the N_S-point quadrature of
    the contour (trapezoid rule on the ellipse = eq. eq-Ap-num; Gauss-Legendre
    on a rectangle, R12) and the winding-number count (eq. eq-ncs)."""
    zeta, dz = contour_quadrature(c, NS, sampling=False)
    rho = max(c.a, c.b)
    k = red.k
    A = [np.zeros((k, k), np.complex128) for _ in range(2 * K)]
    wind = 0.0 + 0.0j
    I = np.eye(k, dtype=np.complex128)
    for m in range(NS):
        X = sla.solve(red.T(zeta[m]), I)            # T_S(zeta_m)^{-1}
        s = (zeta[m] - c.center) / rho
        w = dz[m] / (2j * math.pi)
        for alpha in range(2 * K):
            A[alpha] += (w * s ** alpha) * X
        # tr(X T_S') = sum_ij X_ij T_S'_ji
        wind += w * np.sum(X * red.dT(zeta[m]).T)
    return A, wind


def hankel(A: Sequence[np.ndarray], K: int):
    """Block Hankel H = [A_{i+j}], shifted H^< = [A_{i+j+1}] and the block row
    H_r = [A_0 ... A_{K-1}] (eq. eq-HH, eq-eigens)."""
    H = np.block([[A[i + j] for j in range(K)] for i in range(K)])
    Hs = np.block([[A[i + j + 1] for j in range(K)] for i in range(K)])
    Hr = np.hstack([A[j] for j in range(K)])
    return H, Hs, Hr


def count_gap(sigma: np.ndarray, tol_gap: float = 1e3):
    """Largest ratio sigma_j/sigma_{j+1} (eq. eq-gap).  Returns (count, gmax);
    count is -1 when gmax < tol_gap."""
    s = np.asarray(sigma)
    if len(s) < 2 or s[0] == 0.0:
        return -1, 0.0
    floor = 10.0 * U_ROUND * len(s) * s[0]
    best, bj = 0.0, -1
    for j in range(len(s) - 1):
        if s[j + 1] <= floor:
            break
        r = s[j] / s[j + 1]
        if r > best:
            best, bj = r, j + 1
    if best >= tol_gap:
        return bj, best
    return -1, best


def extract_pairs(H, Hs, Hr, m: int, c: Contour):
    """A = V0^H H^< W0 S0^-1 (eq. eq-A); eigenpairs of A; lambda = rho l' + gamma
    and g = H_r W0 S0^-1 g' (eq. eq-eigens)."""
    V, sigma, Wh = sla.svd(H, lapack_driver="gesdd")
    V0 = V[:, :m]
    W0 = Wh[:m, :].conj().T
    Sinv = 1.0 / sigma[:m]
    A = (V0.conj().T @ Hs @ W0) * Sinv[None, :]
    lp, Gp = sla.eig(A)
    rho = max(c.a, c.b)
    lam = rho * lp + c.center
    G = Hr @ (W0 * Sinv[None, :]) @ Gp
    return lam, G, sigma


def normalise_vectors(V: np.ndarray) -> np.ndarray:
    V = V / np.linalg.norm(V, axis=0, keepdims=True)
    idx = np.argmax(np.abs(V), axis=0)
    ph = V[idx, np.arange(V.shape[1])]
    return V * (np.abs(ph) / ph)[None, :]


def residuals(prob, lam, V):
    """R7: ||T(l)v|| / (||T(l)||_F ||v||) and the paper's ||T(l)v|| / ||v||."""
    rel = np.empty(len(lam))
    raw = np.empty(len(lam))
    for i, l in enumerate(lam):
        T = T_matrix(prob, l)
        v = V[:, i]
        nv = np.linalg.norm(v)
        r = np.linalg.norm(T @ v)
        raw[i] = r / nv
        rel[i] = r / (np.linalg.norm(T, "fro") * nv)
    return rel, raw


def solve_reduced(red: ReducedNEP, c: Contour, NS: int, K: int,
                  tol_gap: float = 1e3, hankel_tol: float = 1e-13):
    """Alg. 1 on the reduced NEP.  Returns candidate (lambda, g) pairs and the
    diagnostics (winding count, gap count, Hankel singular values)."""
    A, wind = reduced_moments(red, c, NS, K)
    H, Hs, Hr = hankel(A, K)
    sigma = sla.svdvals(H)
    n_gap, gmax = count_gap(sigma, tol_gap)
    m = numerical_rank(sigma, hankel_tol)
    lam, G, _ = extract_pairs(H, Hs, Hr, m, c)
    n_wind = int(round(wind.real)) if np.isfinite(wind.real) else -1   # -1: no derivatives given
    return dict(lam=lam, G=G, n_wind=n_wind, wind=wind,
                n_gap=n_gap, gmax=gmax, m=m, hankel_sigma=sigma)


def rsrr(prob, c: Contour, N: int, L: int, U: np.ndarray, NS: int = 512,
         K: int = 2, delta: float = 1e-14, tol_gap: float = 1e3,
         tol_res: float = 1e-10, hankel_tol: float = 1e-13,
         cheb_degree: int = 40, scheme: str = "sampling", Kp: int = 0,
         interp: str = "auto") -> Dict:
    """Alg. 2 end to end.  Returns eigenvalues strictly inside the contour with
    residual <= tol_res, sorted by (Re, Im), their eigenvectors and residuals,
    plus every intermediate the GPU path is compared against.  scheme
    "moment" replaces S_hat by the moment matrix M_hat in Step 3 (SSRR; K'
    moments, 0 = N)."""
    assert U.shape == (prob.n, L)
    z, _ = contour_quadrature(c, N, sampling=True)
    S_hat = sample_resolvent(prob, z, U)
    M_hat = None
    if scheme == "moment":
        M_hat = moment_matrix(S_hat, c, N, L, Kp if Kp > 0 else N)
        S, sig_S, kS = truncated_basis(M_hat, delta)
    else:
        assert scheme == "sampling"
        S, sig_S, kS = truncated_basis(S_hat, delta)
    if isinstance(prob, BemProblem):
        if interpolation_kind(c, interp) == "chebyshev":
            red = reduced_from_chebyshev(prob, S, float(np.real(c.center)), c.a, cheb_degree)
        else:
            red = reduced_from_circle(prob, S, complex(c.center), circle_radius(c), cheb_degree)
    else:
        red = reduced_from_coefficients(prob, S)
    out = solve_reduced(red, c, NS, K, tol_gap, hankel_tol)
    lam_all, G = out["lam"], out["G"]
    keep = inside(c, lam_all)
    lam = lam_all[keep]
    V = normalise_vectors(S @ G[:, keep]) if lam.size else np.zeros((prob.n, 0), complex)
    rel, raw = residuals(prob, lam, V) if lam.size else (np.zeros(0), np.zeros(0))
    ok = rel <= tol_res
    lam, V, rel, raw = lam[ok], V[:, ok], rel[ok], raw[ok]
    order = np.lexsort((lam.imag, lam.real))
    return dict(lam=lam[order], V=V[:, order], res=rel[order], res_paper=raw[order],
                n_wind=out["n_wind"], wind=out["wind"], n_gap=out["n_gap"],
                gmax=out["gmax"], m=out["m"], kS=kS, sigma_S=sig_S, S_hat=S_hat, M_hat=M_hat,
                S=S, nodes=z, hankel_sigma=out["hankel_sigma"],
                n_inside_candidates=int(keep.sum()))
