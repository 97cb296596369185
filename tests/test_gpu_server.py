"""Serving loop (rsrr_server_*): solves of mixed problems admitted by memory
budget into concurrent slots.  Each result must be bit-identical to the same
solve run alone; the workspace bound used for admission must cover what a
solve allocates; uneven batches of QEP instances (the shape of the batched
workload, at sizes the oracle finishes quickly) match the oracle."""
import time

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


def ct(P, c):
    return P.contour(c.center, c.a, c.b, kind=c.kind, n_h=c.nh, n_v=c.nv)


def mixed_requests():
    """(problem, contour, params kwargs, U) of different families and sizes."""
    reqs = []
    p, c, N, L, U = ni.config_c0()
    reqs.append((p, c, dict(N=N, L=L, precision="c64_ir"), U))
    p, c, N, L, U = ni.config_small_qep(n=96, seed=21)
    reqs.append((p, c, dict(N=N, L=L, precision="c128"), U))
    p, c, N, L, U = ni.config_small_delay(n=64, seed=23)
    reqs.append((p, c, dict(N=N, L=L, precision="c64_ir"), U))
    p = ni.bem_sphere(256)
    reqs.append((p, ni.Contour(3.0, 1.5, 0.3), dict(N=24, L=16, precision="c64_ir", cheb_degree=24),
                 ni.probing_matrix(256, 16, seed=25)))
    p, _, N, L, U = ni.config_c0()
    reqs.append((p, ni.Contour(5j, 1.5, 2.0, kind="rect"), dict(N=N, L=L, precision="c128"), U))
    p, c, N, L, U = ni.config_small_qep(n=120, seed=27)
    reqs.append((p, c, dict(N=N, L=L, precision="c64_ir", scheme="moment"), U))
    return reqs


def same_result(a, b):
    return (np.array_equal(a["lam"], b["lam"]) and np.array_equal(a["V"], b["V"])
            and np.array_equal(a["res"], b["res"]) and a["info"]["n_eig"] == b["info"]["n_eig"])


def solve_alone(P, prob, c, kw, U):
    h = P.Problem(prob)
    try:
        return h.solve(ct(P, c), P.default_params(**kw), P.to_device(U))
    finally:
        h.close()


def test_server_results_equal_alone_and_in_mix(P):
    reqs = mixed_requests()
    alone = [solve_alone(P, *r) for r in reqs]
    handles = [P.Problem(r[0]) for r in reqs]
    srv = P.Server(64 << 30, 4)
    try:
        # every request twice, interleaved, so that slots run different problems at once
        tickets = []
        for rep in range(2):
            for h, (prob, c, kw, U) in zip(handles, reqs):
                tickets.append(srv.submit(h, ct(P, c), P.default_params(**kw), U))
        q, r = srv.pending()
        assert q + r <= len(tickets) and r <= 4
        outs = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
        for h in handles:
            h.close()
    for i, (out, lat) in enumerate(outs):
        ref = alone[i % len(reqs)]
        assert lat > 0
        assert same_result(out, ref), i
        assert out["info"]["n_eig"] > 0 and np.all(out["res"] <= 1e-10)


def test_server_budget_admits_one_at_a_time(P):
    # three copies of one request with a budget of 1.5x its workspace bound:
    # never two at once, whatever the slot count
    reqs = mixed_requests()[:1] * 3
    handles = [P.Problem(r[0]) for r in reqs]
    bounds = [h.workspace_bound(ct(P, c), P.default_params(**kw))
              for h, (prob, c, kw, U) in zip(handles, reqs)]
    alone = [solve_alone(P, *r) for r in reqs]
    budget = bounds[0] * 3 // 2
    srv = P.Server(budget, 3)
    try:
        tickets = [srv.submit(h, ct(P, c), P.default_params(**kw), U)
                   for h, (prob, c, kw, U) in zip(handles, reqs)]
        max_running = 0
        t0 = time.time()
        while time.time() - t0 < 60:
            q, r = srv.pending()
            max_running = max(max_running, r)
            if q == 0 and r == 0:
                break
            time.sleep(0.001)
        outs = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
        for h in handles:
            h.close()
    assert max_running <= 1
    for (out, _), ref in zip(outs, alone):
        assert same_result(out, ref)


def test_server_refuses_request_over_budget(P):
    p, c, N, L, U = ni.config_c0()
    h = P.Problem(p)
    srv = P.Server(1 << 20, 2)
    try:
        with pytest.raises(P.RsrrError, match="budget"):
            srv.submit(h, ct(P, c), P.default_params(N=N, L=L), U)
    finally:
        srv.close()
        h.close()


@pytest.mark.parametrize("case", ["c0", "delay", "moment", "bem"])
def test_workspace_bound_covers_solve(P, case):
    if case == "c0":
        p, c, N, L, U = ni.config_c0()
        kw = dict(N=N, L=L)
    elif case == "delay":
        p, c, N, L, U = ni.config_c1(n=256)
        kw = dict(N=N, L=L)
    elif case == "moment":
        p, c, N, L, U = ni.config_small_qep(n=120, seed=27)
        kw = dict(N=N, L=L, scheme="moment")
    else:
        p = ni.bem_sphere(256)
        c, U = ni.Contour(3.0, 1.5, 0.3), ni.probing_matrix(256, 16, seed=25)
        kw = dict(N=24, L=16, cheb_degree=24)
    h = P.Problem(p)
    try:
        bound = h.workspace_bound(ct(P, c), P.default_params(**kw))
        out = h.solve(ct(P, c), P.default_params(**kw), P.to_device(U))
    finally:
        h.close()
    used = out["info"]["ws_bytes"]
    print(case, "workspace", used, "bound", bound, "ratio", bound / used)
    assert 0 < used <= bound


def test_server_uneven_qep_batch_matches_oracle(P):
    # sixteen QEPs of uneven size as in the batched workload (k ~ U[1,400],
    # circle 10i radius 4, N = 64, L = 32), at n in [64, 200]
    insts = ni.config_c2(count=16, nmin=64, nmax=200)
    handles = [P.Problem(i[0]) for i in insts]
    srv = P.Server(64 << 30, 4)
    try:
        tickets = [srv.submit(h, ct(P, c), P.default_params(N=N, L=L, precision="c64_ir"), U)
                   for h, (p, c, N, L, U) in zip(handles, insts)]
        outs = [srv.wait(t)[0] for t in tickets]
    finally:
        srv.close()
        for h in handles:
            h.close()
    for (p, c, N, L, U), out in zip(insts, outs):
        ref = R.rsrr(p, c, N, L, U)
        assert out["info"]["n_eig"] == len(ref["lam"]) > 0, p.n
        assert out["info"]["n_wind"] == ref["n_wind"]
        assert match_sets(out["lam"], ref["lam"]) <= 1e-9 * 14.0
        assert np.all(out["res"] <= 1e-10)


def test_bounded_wait_times_out_then_returns_the_result(P):
    # a wait shorter than the solve ends with RSRR_ETIMEDOUT and the slot /
    # queue state; the ticket stays valid and a later wait returns the result
    from paper_1510_07522_amd._binding import ETIMEDOUT
    p, c, N, L, U = ni.config_small_delay(n=256, seed=29)
    alone = solve_alone(P, p, c, dict(N=48, L=16, precision="c64_ir"), ni.probing_matrix(256, 16, seed=30))
    h = P.Problem(p)
    srv = P.Server(64 << 30, 2)
    try:
        t = srv.submit(h, ct(P, c), P.default_params(N=48, L=16, precision="c64_ir"),
                       ni.probing_matrix(256, 16, seed=30))
        with pytest.raises(P.RsrrError) as e:
            srv.wait(t, timeout_s=1e-4)
        assert e.value.code == ETIMEDOUT and "slot 0" in str(e.value)
        out, lat = srv.wait(t, timeout_s=120.0)
    finally:
        srv.close()
        h.close()
    assert same_result(out, alone)
