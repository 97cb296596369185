"""BEM matrices on contours that do not hug the real axis: the interpolant
through points of a circle around the contour (rsrr_params.interp) against
the oracle's -- the projected coefficients element by element, and full
solves (count, eigenvalues, residuals) on circles of the serving workload's
BEM shape at reduced n."""
import numpy as np
import pytest

import nep_inputs as ni
from oracle import rsrr_ref as R
from tests._util import match_sets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1510_07522_amd as P
    P.load()
    return P


def test_project_bem_circle_matches_oracle(P):
    p = ni.bem_sphere(200)
    c = ni.Contour(3.25, 0.6, 0.6)
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((200, 30)) + 1j * rng.standard_normal((200, 30)))
    d = 16
    h = P.Problem(p)
    try:
        B, J = h.project(P.contour(c.center, c.a, c.b), P.default_params(N=8, L=8, cheb_degree=d),
                         P.to_device(Q), 30)
    finally:
        h.close()
    assert J == d + 1
    Bh = P.from_device(B).T.reshape(J, 30, 30)
    ref = R.circle_projection(p, Q, 3.25, 0.6, d)
    for j in range(J):
        assert np.linalg.norm(Bh[j].T - ref[j]) <= 1e-12 * max(1.0, np.linalg.norm(ref[0])), j


_REF = {}


def _oracle(n, center, r, L):
    key = (n, center, r, L)
    if key not in _REF:
        p = ni.bem_sphere(n)
        c = ni.Contour(center, r, r)
        U = ni.probing_matrix(n, L, seed=n + 1)
        _REF[key] = (p, c, U, R.rsrr(p, c, 40, L, U, NS=256, K=2, cheb_degree=40))
    return _REF[key]


@pytest.mark.parametrize("precision", ["c128", "c64_ir"])
@pytest.mark.parametrize("n,center,r,L", [(512, 3.25, 0.6, 16), (640, 2.69, 0.79, 16)])
def test_bem_circle_solve_matches_oracle(P, precision, n, center, r, L):
    p, c, U, ref = _oracle(n, center, r, L)
    h = P.Problem(p)
    try:
        out = h.solve(P.contour(c.center, c.a, c.b),
                      P.default_params(N=40, L=L, NS=256, precision=precision), P.to_device(U))
    finally:
        h.close()
    info = out["info"]
    print(n, center, r, "oracle", len(ref["lam"]), ref["n_wind"], ref["lam"], "gpu", info["n_eig"], info["n_wind"])
    assert len(ref["lam"]) >= 1 and ref["n_wind"] == len(ref["lam"])
    assert info["n_wind"] == ref["n_wind"] and info["n_eig"] == len(ref["lam"])
    assert match_sets(out["lam"], ref["lam"]) <= 1e-9 * max(center, r)
    assert np.all(out["res"] <= 1e-10)
