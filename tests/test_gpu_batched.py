"""rsrr_solve_batched: several QEPs of uneven order whose sampling LUs are
factored together (one set of launches per panel step, the trailing updates
as one persistent launch over all problems' tiles).  Each problem's result
must be bit-identical to its solve alone, and match the oracle."""
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


def _instances(sizes, N=32, L=16):
    out = []
    for i, n in enumerate(sizes):
        p = ni.qep_dense(n, 400.0, seed=3100 + i)
        out.append((p, ni.Contour(10j, 4.0, 4.0), N, L, ni.probing_matrix(n, L, seed=4100 + i)))
    return out


def _same(a, b):
    return (np.array_equal(a["lam"], b["lam"]) and np.array_equal(a["V"], b["V"])
            and np.array_equal(a["res"], b["res"]) and a["info"]["n_eig"] == b["info"]["n_eig"]
            and a["info"]["k_S"] == b["info"]["k_S"])


@pytest.mark.parametrize("precision", ["c64_ir", "c128"])
def test_batched_equals_alone_and_oracle(P, precision):
    # uneven orders, ragged against the panel width, one of them below one
    # pair; N L = 512 exceeds every order, so the sampled space is the whole
    # space and every eigenvalue inside is returned
    insts = _instances([77, 150, 203, 333, 130])
    hs = [P.Problem(i[0]) for i in insts]
    try:
        cts = [P.contour(c.center, c.a, c.b) for _, c, _, _, _ in insts]
        prms = [P.default_params(N=N, L=L, precision=precision) for _, _, N, L, _ in insts]
        Us = [P.to_device(U) for *_, U in insts]
        batched = P.solve_batched(hs, cts, prms, Us)
        alone = [h.solve(ct, prm, U) for h, ct, prm, U in zip(hs, cts, prms, Us)]
    finally:
        for h in hs:
            h.close()
    for (p, c, N, L, U), b, a in zip(insts, batched, alone):
        print(p.n, "batched", b["info"]["n_eig"], "alone", a["info"]["n_eig"])
        assert _same(a, b), p.n
    # the largest against the oracle
    p, c, N, L, U = insts[3]
    ref = R.rsrr(p, c, N, L, U)
    got = batched[3]
    assert len(got["lam"]) == len(ref["lam"]) > 0
    assert match_sets(got["lam"], ref["lam"]) <= 1e-9 * 14.0
    assert np.all(got["res"] <= 1e-10)


@pytest.mark.parametrize("precision", ["c64_ir", "c128"])
def test_batched_equals_alone_with_tall_panels(P, precision):
    # orders above 1024 (several blocks of four panels with look-ahead): the
    # segmented launches factor every matrix as it is factored alone
    insts = _instances([1100, 1300, 700])
    hs = [P.Problem(i[0]) for i in insts]
    try:
        cts = [P.contour(c.center, c.a, c.b) for _, c, _, _, _ in insts]
        prms = [P.default_params(N=N, L=L, precision=precision) for _, _, N, L, _ in insts]
        Us = [P.to_device(U) for *_, U in insts]
        batched = P.solve_batched(hs, cts, prms, Us)
        alone = [h.solve(ct, prm, U) for h, ct, prm, U in zip(hs, cts, prms, Us)]
    finally:
        for h in hs:
            h.close()
    for (p, c, N, L, U), b, a in zip(insts, batched, alone):
        print(p.n, "batched", b["info"]["n_eig"], "alone", a["info"]["n_eig"])
        assert _same(a, b), p.n


def test_batched_rejects_mixed_precision(P):
    insts = _instances([40, 50])
    hs = [P.Problem(i[0]) for i in insts]
    try:
        cts = [P.contour(c.center, c.a, c.b) for _, c, _, _, _ in insts]
        prms = [P.default_params(N=16, L=4, precision="c64_ir"), P.default_params(N=16, L=4, precision="c128")]
        with pytest.raises(P.RsrrError):
            P.solve_batched(hs, cts, prms)
    finally:
        for h in hs:
            h.close()


def test_autotuned_panel_width(P, tmp_path):
    # the tuner picks one of its candidate widths; a solve with nb = 0 uses it
    # (bit-identical to a solve with that width given); the table round-trips
    # through its JSON file
    nb, ms = P.tune_lu("c64_ir", 300, 8)
    assert nb in (16, 32, 64) and ms > 0
    path = str(tmp_path / "tune.json")
    P.tune_save(path)
    assert P.tune_load(path) >= 1
    p, c, N, L, U = _instances([300])[0]
    h = P.Problem(p)
    try:
        ct = P.contour(c.center, c.a, c.b)
        a = h.solve(ct, P.default_params(N=N, L=L, precision="c64_ir", nb=0), P.to_device(U))
        b = h.solve(ct, P.default_params(N=N, L=L, precision="c64_ir", nb=nb), P.to_device(U))
    finally:
        h.close()
    assert _same(a, b)
