"""Sampling launches captured in a HIP graph (rsrr_params.graph = 1): every
replay, with eager solves and synchronisations between the replays, returns
results bit-identical to the eager path; a change of size captures again."""
import numpy as np
import pytest

import nep_inputs as ni

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1510_07522_amd as P
    P.load()
    return P


def _same(a, b):
    return (np.array_equal(a["lam"], b["lam"]) and np.array_equal(a["V"], b["V"])
            and np.array_equal(a["res"], b["res"]) and a["info"]["n_eig"] == b["info"]["n_eig"])


@pytest.mark.parametrize("precision", ["c64_ir", "c128"])
@pytest.mark.parametrize("family", ["qep", "bem"])
def test_graph_replays_equal_eager(P, precision, family):
    import torch
    if family == "qep":
        p, c, N, L, U = ni.config_c0()
    else:
        p, c, N, L, U = ni.bem_sphere(256), ni.Contour(3.0, 1.5, 0.3), 24, 16, ni.probing_matrix(256, 16, seed=61)
    h = P.Problem(p)
    try:
        ct = P.contour(c.center, c.a, c.b)
        Ud = P.to_device(U)
        eager = h.solve(ct, P.default_params(N=N, L=L, precision=precision, NS=256), Ud)
        g = P.default_params(N=N, L=L, precision=precision, NS=256, graph=1)
        for rep in range(4):
            out = h.solve(ct, g, Ud)                 # first call captures, later ones replay
            torch.cuda.synchronize()
            assert _same(out, eager), rep
            other = h.solve(ct, P.default_params(N=N, L=L, precision=precision, NS=256), Ud)
            assert _same(other, eager), rep
        # another node count: captured again, still equal to the eager path
        e2 = h.solve(ct, P.default_params(N=N + 8, L=L, precision=precision, NS=256), Ud)
        g2 = h.solve(ct, P.default_params(N=N + 8, L=L, precision=precision, NS=256, graph=1), Ud)
        assert _same(e2, g2)
        g3 = h.solve(ct, g, Ud)
        assert _same(g3, eager)
    finally:
        h.close()
