"""Orders above 8192: complex64 factorisations with 16 rows per thread in the
LU panel (up to order 16384), alone and in the segmented launches of an
uneven batch; complex128 factorisations stay limited to order 8192."""
import numpy as np
import pytest

import nep_inputs as ni
from oracle import rsrr_ref as R
from tests.test_gpu_dense import batch_to_dev, dev_to_batch, rnd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1510_07522_amd as P
    P.load()
    return P


def test_c64_gesv_above_8192(P):
    n, nrhs, batch = 9000, 3, 2
    rng = np.random.default_rng(9000)
    # a general matrix (rows interchanged at every panel) and a diagonally
    # dominant one (none)
    A = [rnd(rng, n, n), rnd(rng, n, n) + 2 * np.sqrt(n) * np.eye(n)]
    B = [rnd(rng, n, nrhs) for _ in range(batch)]
    dA = batch_to_dev(P, [a.astype(np.complex64) for a in A])
    dB = batch_to_dev(P, [x.astype(np.complex64) for x in B])
    st, info = P.gesv(dA, dB, n, nrhs, batch, 64)
    assert st == 0 and info == [0] * batch
    del dA
    X = dev_to_batch(dB, batch, n, nrhs)
    for b in range(batch):
        Ab = A[b].astype(np.complex64).astype(np.complex128)
        Xb = X[b].astype(np.complex128)
        eta = np.linalg.norm(B[b].astype(np.complex64) - Ab @ Xb) / (
            np.linalg.norm(Ab) * np.linalg.norm(Xb) + np.linalg.norm(B[b]))
        print(f"matrix {b}: backward error {eta:.2e}")
        assert eta < 2e-7 * np.sqrt(n), (b, eta)


def _solve(P, probs, prm_kw, batched):
    # the interval [2, 4] holds the eigenvalue near pi, away from the contour
    c = ni.Contour(3.0, 1.0, 0.3)
    hs = [P.Problem(p) for p in probs]
    try:
        cts = [P.contour(c.center, c.a, c.b) for _ in probs]
        prms = [P.default_params(**prm_kw) for _ in probs]
        Us = [P.to_device(ni.probing_matrix(p.n, prm_kw["L"], seed=8800 + i)) for i, p in enumerate(probs)]
        if batched:
            return P.solve_batched(hs, cts, prms, Us)
        return [h.solve(ct, prm, U) for h, ct, prm, U in zip(hs, cts, prms, Us)]
    finally:
        for h in hs:
            h.close()


def test_bem_above_8192_batched_equals_alone(P):
    # a BEM sphere of order 8400 beside one of order 700 in one uneven batch:
    # the segmented launches factor the large one with the 16-row panels, and
    # every result is the one the problem gets alone; the large problem's
    # pairs are checked by their residuals recomputed on the host and its
    # count against the winding number
    probs = [ni.bem_sphere(8400), ni.bem_sphere(700)]
    kw = dict(N=16, L=16, precision="c64_ir")
    batched = _solve(P, probs, kw, True)
    alone = _solve(P, probs, kw, False)
    for p, b, a in zip(probs, batched, alone):
        print(p.n, "n_eig", b["info"]["n_eig"], "winding", b["info"]["n_wind"], "lam", b["lam"])
        assert (np.array_equal(a["lam"], b["lam"]) and np.array_equal(a["V"], b["V"])
                and np.array_equal(a["res"], b["res"]))
    big = batched[0]
    assert big["info"]["n_eig"] == big["info"]["n_wind"] == 1
    assert np.all(big["res"] <= 1e-10)
    rel, _ = R.residuals(probs[0], big["lam"], big["V"])
    print("host residuals", rel)
    assert np.all(rel <= 1e-10)


def test_complex128_above_8192_is_refused(P):
    with pytest.raises(P.RsrrError):
        _solve(P, [ni.bem_sphere(8300)], dict(N=8, L=8, precision="c128"), False)
