"""GPU parity of the dense building blocks (batched complex GEMM on the matrix
cores, batched blocked LU with partial pivoting) against plain numpy."""
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


def rnd(rng, *shape, dtype=np.complex128):
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return a.astype(dtype)


def batch_to_dev(P, mats):
    """list of column-major n x m arrays -> one device buffer (batch strided)."""
    import torch
    arrs = [np.asfortranarray(m) for m in mats]
    flat = np.concatenate([a.T.reshape(-1) for a in arrs])
    return torch.from_numpy(flat).to("cuda")


def dev_to_batch(t, batch, rows, cols):
    a = t.cpu().numpy().reshape(batch, cols, rows)
    return [a[b].T for b in range(batch)]


OPF = {"N": lambda x: x, "T": lambda x: x.T, "C": lambda x: x.conj().T}


@pytest.mark.parametrize("opA,opB", [("N", "N"), ("N", "T"), ("C", "N"), ("T", "C"), ("C", "C")])
@pytest.mark.parametrize("prec", ["c128", "c64", "c64_3m"])
def test_gemm_matches_numpy(P, opA, opB, prec):
    rng = np.random.default_rng(hash((opA, opB, prec)) % 2**31)
    M, N, K, batch = 70, 131, 45, 3             # ragged in every dimension
    dt = np.complex128 if prec == "c128" else np.complex64
    A = [rnd(rng, *( (M, K) if opA == "N" else (K, M)), dtype=dt) for _ in range(batch)]
    B = [rnd(rng, *( (K, N) if opB == "N" else (N, K)), dtype=dt) for _ in range(batch)]
    Cc = [rnd(rng, M, N, dtype=dt) for _ in range(batch)]
    alpha, beta = 0.7 - 0.2j, -1.1 + 0.4j
    dA, dB, dC = batch_to_dev(P, A), batch_to_dev(P, B), batch_to_dev(P, Cc)
    P.gemm(opA, opB, dA, dB, dC, M, N, K, alpha, beta, batch=batch,
           sA=A[0].size, sB=B[0].size, sC=M * N, gauss3m=(prec == "c64_3m"))
    out = dev_to_batch(dC, batch, M, N)
    for b in range(batch):
        A64, B64, C64 = (x.astype(np.complex128) for x in (A[b], B[b], Cc[b]))
        ref = alpha * OPF[opA](A64) @ OPF[opB](B64) + beta * C64
        scale = np.abs(OPF[opA](A64)) @ np.abs(OPF[opB](B64)) + np.abs(C64)
        err = np.max(np.abs(out[b] - ref) / scale)
        tol = 1e-14 if prec == "c128" else 2e-6
        assert err < tol, (b, err)


# 24- and 32-column panels (those of the divide-and-conquer inverses), also
# with a batch of 50
@pytest.mark.parametrize("n,nrhs,batch,nb", [(1, 3, 2, 64), (37, 5, 3, 16), (200, 20, 4, 64),
                                             (333, 7, 2, 64), (1100, 9, 2, 64), (2100, 4, 1, 64),
                                             (300, 6, 5, 32), (777, 3, 3, 24), (2600, 5, 2, 32),
                                             (600, 3, 50, 32), (1500, 6, 3, 16)])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_batched_lu_solve(P, n, nrhs, batch, nb, prec):
    import torch
    rng = np.random.default_rng(n * 7 + nrhs)
    dt = np.complex128 if prec == "c128" else np.complex64
    A = [rnd(rng, n, n) + 2 * np.sqrt(n) * np.eye(n) * (b % 2) for b in range(batch)]
    B = [rnd(rng, n, nrhs) for _ in range(batch)]
    dA = batch_to_dev(P, [a.astype(dt) for a in A])
    dB = batch_to_dev(P, [x.astype(dt) for x in B])
    st, info = P.gesv(dA, dB, n, nrhs, batch, nb)
    assert st == 0 and info == [0] * batch
    X = dev_to_batch(dB, batch, n, nrhs)
    for b in range(batch):
        Ab = A[b].astype(dt).astype(np.complex128)
        Xb = X[b].astype(np.complex128)
        # normwise backward error of the computed solution
        eta = np.linalg.norm(B[b].astype(dt) - Ab @ Xb) / (np.linalg.norm(Ab) * np.linalg.norm(Xb)
                                                          + np.linalg.norm(B[b]))
        assert eta < (2e-15 * np.sqrt(n) if prec == "c128" else 2e-7 * np.sqrt(n)), eta
        if prec == "c128":
            ref = np.linalg.solve(Ab, B[b])
            cond = np.linalg.cond(Ab)
            assert np.linalg.norm(Xb - ref) / np.linalg.norm(ref) < 1e-15 * cond * n


def test_batched_lu_reports_exact_singularity(P):
    n = 50
    rng = np.random.default_rng(1)
    A = rnd(rng, n, n)
    A[:, 7] = 0.0                               # column 7 is zero: pivot 8 vanishes
    dA = batch_to_dev(P, [A, np.eye(n, dtype=complex)])
    dB = batch_to_dev(P, [np.ones((n, 1), complex), np.ones((n, 1), complex)])
    st, info = P.gesv(dA, dB, n, 1, 2, 16)
    assert st == -4
    assert info[0] == 8 and info[1] == 0


def test_batched_lu_reports_zero_pivot_in_later_blocks(P):
    # an exactly zero column gives the status of its own step, in the first
    # panel and in the panel at column 1024, after four blocks of panels
    n = 2100
    rng = np.random.default_rng(2)
    A0 = rnd(rng, n, n)
    A0[:, 7] = 0.0
    A1 = rnd(rng, n, n)
    A1[:, 1030] = 0.0
    A2 = rnd(rng, n, n) + 2 * np.sqrt(n) * np.eye(n)
    dA = batch_to_dev(P, [A0, A1, A2])
    dB = batch_to_dev(P, [np.ones((n, 1), complex)] * 3)
    st, info = P.gesv(dA, dB, n, 1, 3, 64)
    assert st == -4
    assert info == [8, 1031, 0]
