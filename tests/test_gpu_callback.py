"""Scalar functions supplied by the caller (rsrr_create_fn, eq. eq-Z-expr
allows any f_k): T(z) = -zI + A0 + sqrt(z + 4) A1, whose third function is
outside the pow/exp/rat menu, through a ctypes callback, against the oracle
evaluating the same Python functions."""
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


def _solve(P, p, c, N, L, U, **kw):
    h = P.Problem(p)
    try:
        return h.solve(P.contour(c.center, c.a, c.b), P.default_params(N=N, L=L, **kw), P.to_device(U))
    finally:
        h.close()


@pytest.mark.parametrize("precision", ["c128", "c64_ir"])
def test_callback_problem_matches_oracle(P, precision):
    p = ni.sqrt_coupled(96, seed=41)
    c = ni.Contour(0.0, 1.5, 1.5)
    N, L = 32, 8
    U = ni.probing_matrix(p.n, L, seed=42)
    ref = R.rsrr(p, c, N, L, U)
    out = _solve(P, p, c, N, L, U, precision=precision)
    print("oracle", len(ref["lam"]), ref["n_wind"], "gpu", len(out["lam"]), out["info"]["n_wind"])
    assert len(ref["lam"]) > 5
    assert len(out["lam"]) == len(ref["lam"])
    assert out["info"]["n_wind"] == ref["n_wind"]
    assert match_sets(out["lam"], ref["lam"]) <= 1e-9 * 1.5
    assert np.all(out["res"] <= 1e-10)
    # residuals recomputed on the host from the same callable
    rel, _ = R.residuals(p, out["lam"], out["V"])
    assert np.all(rel <= 1e-10)


def test_callback_without_derivatives_skips_the_winding_count(P):
    from paper_1510_07522_amd._binding import WARN_NO_WINDING
    p = ni.sqrt_coupled(96, seed=41, derivatives=False)
    c = ni.Contour(0.0, 1.5, 1.5)
    N, L = 32, 8
    U = ni.probing_matrix(p.n, L, seed=42)
    ref = R.rsrr(p, c, N, L, U)
    out = _solve(P, p, c, N, L, U, precision="c64_ir")
    assert out["info"]["n_wind"] == -1 and ref["n_wind"] == -1
    assert out["status"] & WARN_NO_WINDING
    assert len(out["lam"]) == len(ref["lam"]) > 5
    assert match_sets(out["lam"], ref["lam"]) <= 1e-9 * 1.5


def test_callback_error_is_reported(P):
    from paper_1510_07522_amd import RsrrError

    def bad(z):
        raise ValueError("no value here")
    p = ni.sqrt_coupled(16, seed=43)
    q = ni.CoeffProblem(n=p.n, kinds=p.kinds, mats=p.mats,
                        fspecs=[p.fspecs[0], p.fspecs[1], ("callable", bad)])
    U = ni.probing_matrix(16, 4, seed=44)
    with pytest.raises(RsrrError) as e:
        _solve(P, q, ni.Contour(0.0, 1.5, 1.5), 16, 4, U)
    assert e.value.code == -1 and "callback" in str(e.value)
