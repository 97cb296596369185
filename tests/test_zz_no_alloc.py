"""rsrr_gesv_batched_noalloc (the batched LU solve whose work space is the
library's fixed device array) against rsrr_gesv_batched (the same kernels with
allocated work space), through the C ABI: two calls in a row, the second with
a smaller input, bit-identical factors and solutions; a request beyond the
fixed array is refused without touching its buffers; a singular matrix is
reported with its pivot index."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1510_07522_amd as P
    P.load()
    return P


def _batch(rng, n, nrhs, batch, dt):
    import torch
    A = [(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 2 * np.sqrt(n) * np.eye(n) * (b % 2))
         .astype(dt) for b in range(batch)]
    B = [(rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs))).astype(dt) for _ in range(batch)]
    flat = lambda ms: torch.from_numpy(np.concatenate([np.asfortranarray(m).T.reshape(-1) for m in ms])).to("cuda")
    return A, B, flat(A), flat(B)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_noalloc_matches_allocating_entry_on_two_calls(P, prec):
    import torch
    dt = np.complex128 if prec == "c128" else np.complex64
    for call, (n, nrhs, batch, nb, seed) in enumerate([(700, 5, 6, 64, 11), (123, 3, 3, 32, 12)]):
        rng = np.random.default_rng(seed)
        A, B, dA, dB = _batch(rng, n, nrhs, batch, dt)
        dA2, dB2 = dA.clone(), dB.clone()
        st1, info1 = P.gesv(dA, dB, n, nrhs, batch, nb)
        st2, info2 = P.gesv(dA2, dB2, n, nrhs, batch, nb, noalloc=True)
        torch.cuda.synchronize()
        print(f"call {call}: n={n} batch={batch} nb={nb} {prec}: status {st1} / {st2}", flush=True)
        assert st1 == st2 == 0 and info1 == info2 == [0] * batch
        assert torch.equal(dA, dA2), "factors differ"
        assert torch.equal(dB, dB2), "solutions differ"
        X = dB2.cpu().numpy().reshape(batch, nrhs, n)
        for b in range(batch):
            Ab = A[b].astype(np.complex128)
            Xb = X[b].T.astype(np.complex128)
            eta = np.linalg.norm(B[b] - Ab @ Xb) / (np.linalg.norm(Ab) * np.linalg.norm(Xb) + np.linalg.norm(B[b]))
            assert eta < (2e-15 if prec == "c128" else 2e-7) * np.sqrt(n), (b, eta)


def test_noalloc_refuses_work_beyond_the_fixed_array(P):
    import torch
    n, batch = 4096, 10                       # complex128: about 80 MiB of work space > 64 MiB
    dA = torch.ones(batch * n * n, dtype=torch.complex128, device="cuda")
    dB = torch.ones(batch * n, dtype=torch.complex128, device="cuda")
    st, _ = P.gesv(dA, dB, n, 1, batch, 64, noalloc=True)
    assert st == -1
    assert "64" in P.load().rsrr_last_error().decode() or "scratch" in P.load().rsrr_last_error().decode()
    assert bool(torch.all(dA == 1)) and bool(torch.all(dB == 1))


def test_noalloc_reports_exact_singularity(P):
    import torch
    n = 50
    rng = np.random.default_rng(1)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A[:, 7] = 0.0
    mats = [A, np.eye(n, dtype=complex)]
    dA = torch.from_numpy(np.concatenate([np.asfortranarray(m).T.reshape(-1) for m in mats])).to("cuda")
    dB = torch.ones(2 * n, dtype=torch.complex128, device="cuda")
    st, info = P.gesv(dA, dB, n, 1, 2, 16, noalloc=True)
    assert st == -4 and info[0] == 8 and info[1] == 0


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_noalloc_without_status_enqueues_only_and_replays_in_a_graph(P, prec):
    """With no status buffer the allocation-free call only enqueues kernels: it
    gives the same bits as with one, and it can be captured in a HIP graph
    (the inputs restored by a copy inside the graph); every replay, with
    eager work and synchronisations between replays, equals the eager call."""
    import torch
    dt = np.complex128 if prec == "c128" else np.complex64
    n, nrhs, batch, nb = 300, 4, 3, 32
    rng = np.random.default_rng(21)
    A, B, dA0, dB0 = _batch(rng, n, nrhs, batch, dt)
    ref_A, ref_B = dA0.clone(), dB0.clone()
    st, info = P.gesv(ref_A, ref_B, n, nrhs, batch, nb, noalloc=True)
    assert st == 0 and info == [0] * batch
    dA, dB = dA0.clone(), dB0.clone()
    st, info = P.gesv(dA, dB, n, nrhs, batch, nb, noalloc=True, status=False)
    torch.cuda.synchronize()
    assert st == 0 and info == []
    assert torch.equal(dA, ref_A) and torch.equal(dB, ref_B)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            dA.copy_(dA0)
            dB.copy_(dB0)
            st = P.gesv(dA, dB, n, nrhs, batch, nb, noalloc=True, status=False)[0]
    assert st == 0
    for rep in range(3):
        dA.fill_(0)
        dB.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"{prec} replay {rep}", flush=True)
        assert torch.equal(dA, ref_A), f"replay {rep}: factors differ"
        assert torch.equal(dB, ref_B), f"replay {rep}: solutions differ"
