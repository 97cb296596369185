"""ctypes binding of librsrr.so (the C ABI in include/rsrr.h).

Argument marshalling only: every step of the method runs inside the library.
PyTorch supplies device memory (and the current HIP stream); matrices cross
the boundary column-major, i.e. a column-major n x m matrix is a contiguous
torch tensor of shape (m, n) (see ``to_device`` / ``from_device``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsrr.so")


class RsrrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rsrr error {code}: {msg}")
        self.code = code


class cplx(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class fn_t(C.Structure):
    _fields_ = [("kind", C.c_int), ("p", C.c_int), ("c", cplx), ("t", cplx)]


class contour_t(C.Structure):
    _fields_ = [("center", cplx), ("a", C.c_double), ("b", C.c_double), ("kind", C.c_int),
                ("n_h", C.c_int), ("n_v", C.c_int)]


CONTOUR_KIND = {"ellipse": 0, "rect": 1}


class params_t(C.Structure):
    _fields_ = [("N", C.c_int), ("L", C.c_int), ("NS", C.c_int), ("K", C.c_int),
                ("delta", C.c_double), ("tol_gap", C.c_double), ("tol_res", C.c_double),
                ("hankel_tol", C.c_double), ("precision", C.c_int), ("ir_max_iter", C.c_int),
                ("ir_tol", C.c_double), ("cheb_degree", C.c_int), ("nb", C.c_int),
                ("seed", C.c_uint64), ("scheme", C.c_int), ("Kp", C.c_int), ("chunk_gib", C.c_double),
                ("interp", C.c_int), ("graph", C.c_int), ("nb_reduced", C.c_int)]


class info_t(C.Structure):
    _fields_ = [("n", C.c_int), ("N", C.c_int), ("L", C.c_int), ("k_S", C.c_int), ("m", C.c_int),
                ("n_wind", C.c_int), ("n_gap", C.c_int), ("n_eig", C.c_int),
                ("n_candidates", C.c_int), ("ir_iters", C.c_int), ("ir_fallback", C.c_int),
                ("status", C.c_int), ("wind_re", C.c_double), ("wind_im", C.c_double),
                ("t_sample", C.c_double), ("t_basis", C.c_double), ("t_project", C.c_double),
                ("t_reduced", C.c_double), ("t_residual", C.c_double), ("ws_bytes", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PREC_C128, PREC_C64_IR = 0, 1
SCHEME = {"sampling": 0, "moment": 1}
INTERP = {"auto": 0, "chebyshev": 1, "circle": 2}
MAT_KIND = {"identity": 0, "diag": 1, "real": 2, "dense": 3}
FN_KIND = {"pow": 0, "exp": 1, "rat": 2}
WARN_RANK_SATURATED, WARN_COUNT_MISMATCH, WARN_IR_FALLBACK = 1, 2, 4
WARN_HANKEL_FULL, WARN_NO_WINDING = 8, 16
ETIMEDOUT = -7

# int (*rsrr_scalar_fn)(void* ctx, const rsrr_complex* z, size_t m, rsrr_complex* f, rsrr_complex* df)
SCALAR_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.POINTER(cplx), C.c_size_t, C.POINTER(cplx),
                        C.POINTER(cplx))

# Every symbol declared in include/rsrr.h, with its ctypes signature.
_vp, _i, _d, _ll = C.c_void_p, C.c_int, C.c_double, C.c_longlong
SIGNATURES = {
    "rsrr_default_params": (None, [C.POINTER(params_t)]),
    "rsrr_create": (_i, [C.POINTER(_vp), _i, _i, C.POINTER(_i), C.POINTER(_vp), C.POINTER(fn_t), _vp]),
    "rsrr_create_fn": (_i, [C.POINTER(_vp), _i, _i, C.POINTER(_i), C.POINTER(_vp), _vp, _vp, _vp]),
    "rsrr_create_bem": (_i, [C.POINTER(_vp), _i, C.POINTER(_d), _d, _vp]),
    "rsrr_destroy": (None, [_vp]),
    "rsrr_sample": (_i, [_vp, C.POINTER(contour_t), C.POINTER(params_t), _vp, _i, _vp, _i,
                         C.POINTER(info_t)]),
    "rsrr_moment_matrix": (_i, [_vp, C.POINTER(contour_t), C.POINTER(params_t), _vp, _i, _vp, _i]),
    "rsrr_orthonormalize": (_i, [_i, _i, _vp, _i, _d, _vp, _i, C.POINTER(_i), _vp]),
    "rsrr_project": (_i, [_vp, C.POINTER(contour_t), C.POINTER(params_t), _vp, _i, _i, _vp,
                          C.POINTER(_i)]),
    "rsrr_solve": (_i, [_vp, C.POINTER(contour_t), C.POINTER(params_t), _vp, C.POINTER(_vp)]),
    "rsrr_workspace_bound": (_i, [_vp, C.POINTER(contour_t), C.POINTER(params_t), C.POINTER(C.c_size_t)]),
    "rsrr_solve_batched": (_i, [_i, C.POINTER(_vp), C.POINTER(contour_t), C.POINTER(params_t), C.POINTER(_vp),
                                C.POINTER(_vp)]),
    "rsrr_server_create": (_i, [C.POINTER(_vp), C.c_size_t, _i]),
    "rsrr_server_submit": (_i, [_vp, _vp, C.POINTER(contour_t), C.POINTER(params_t), _vp,
                                C.POINTER(C.c_uint64)]),
    "rsrr_server_wait": (_i, [_vp, C.c_uint64, _d, C.POINTER(_vp), C.POINTER(_d)]),
    "rsrr_server_pending": (_i, [_vp, C.POINTER(_i), C.POINTER(_i)]),
    "rsrr_server_destroy": (None, [_vp]),
    "rsrr_result_info": (_i, [_vp, C.POINTER(info_t)]),
    "rsrr_result_copy": (_i, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "rsrr_result_free": (None, [_vp]),
    "rsrr_zgemm_batched": (_i, [_i, _i, _i, _i, _i, cplx, _vp, _i, _ll, _vp, _i, _ll, cplx, _vp, _i,
                                _ll, _i, _vp]),
    "rsrr_cgemm_batched": (_i, [_i, _i, _i, _i, _i, cplx, _vp, _i, _ll, _vp, _i, _ll, cplx, _vp, _i,
                                _ll, _i, _i, _vp]),
    "rsrr_gesv_batched": (_i, [_i, _i, _i, _vp, _i, _ll, _vp, _i, _ll, _i, _i, C.POINTER(_i), _vp]),
    "rsrr_gesv_batched_noalloc": (_i, [_i, _i, _i, _vp, _i, _ll, _vp, _i, _ll, _i, _i, C.POINTER(_i), _vp]),
    "rsrr_tune_lu": (_i, [_i, _i, _i, C.POINTER(_i), C.POINTER(_d)]),
    "rsrr_tune_save": (_i, [C.c_char_p]),
    "rsrr_tune_load": (_i, [C.c_char_p]),
    "rsrr_timers_enable": (None, [_i]),
    "rsrr_timers_only": (None, [C.c_char_p]),
    "rsrr_timers_reset": (None, []),
    "rsrr_timers_count": (_i, []),
    "rsrr_timers_get": (_i, [_i, C.c_char_p, _i, C.POINTER(_ll), C.POINTER(_d), C.POINTER(_d),
                             C.POINTER(_d)]),
    "rsrr_last_error": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads librsrr.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1510_07522_amd.build`"
                           " (there is no CPU fallback)")
    # torch first: it brings its own HIP runtime (same soname), and the
    # library must bind to that one, or the process holds two runtimes and
    # torch's device memory and streams are foreign to the library's
    _torch()
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(code: int) -> int:
    if code < 0:
        raise RsrrError(code, load().rsrr_last_error().decode(errors="replace"))
    return code


# ------------------------------------------------------------ memory helpers
def _torch():
    import torch
    return torch


def stream_ptr():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_device(a: np.ndarray, dtype=None):
    """Column-major copy of a 2-D (or 1-D) numpy array on cuda:0.  An n x m
    matrix becomes a tensor of shape (m, n) whose memory is column-major."""
    torch = _torch()
    a = np.asarray(a)
    if dtype is not None:
        a = a.astype(dtype)
    if a.ndim == 1:
        return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda")


def from_device(t, rows: int | None = None) -> np.ndarray:
    """Inverse of to_device: an (m, n) tensor -> n x m numpy array."""
    a = t.detach().cpu().numpy()
    if a.ndim == 1:
        return a
    out = a.T
    return out[:rows] if rows is not None else out


def empty_device(rows: int, cols: int, dtype="complex128"):
    torch = _torch()
    dt = {"complex128": torch.complex128, "complex64": torch.complex64}[dtype]
    return torch.empty((cols, rows), dtype=dt, device="cuda")


def _ptr(t):
    return C.c_void_p(t.data_ptr())


# --------------------------------------------------------------- parameters
def default_params(**kw) -> params_t:
    p = params_t()
    load().rsrr_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"c128": PREC_C128, "c64_ir": PREC_C64_IR}[v]
        if k == "scheme" and isinstance(v, str):
            v = SCHEME[v]
        if k == "interp" and isinstance(v, str):
            v = INTERP[v]
        setattr(p, k, v)
    return p


def contour(center: complex, a: float, b: float, kind: str = "ellipse", n_h: int = 0,
            n_v: int = 0) -> contour_t:
    """Ellipse (semi-axes a, b) or rectangle (half-sides a, b; n_h / n_v
    sampling nodes per horizontal / vertical side, 0 = split by length)."""
    c = contour_t()
    c.center = cplx(float(np.real(center)), float(np.imag(center)))
    c.a, c.b = float(a), float(b)
    c.kind = CONTOUR_KIND[kind]
    c.n_h, c.n_v = int(n_h), int(n_v)
    return c


def _fn(spec) -> fn_t:
    f = fn_t()
    f.kind = FN_KIND[spec[0]]
    f.c = cplx(float(np.real(spec[1])), float(np.imag(spec[1])))
    f.p = int(spec[2])
    f.t = cplx(0.0, 0.0)
    if spec[0] in ("exp", "rat"):
        f.t = cplx(float(np.real(spec[3])), float(np.imag(spec[3])))
    return f


def _scalar_callback(fns):
    """rsrr_scalar_fn calling the Python functions fn_k(z) -> (f, f' or None)
    for the m nodes the library passes; fills f[q*J + k] and df[q*J + k]."""
    J = len(fns)

    def cb(ctx, zp, m, fp, dfp):
        try:
            z = np.ctypeslib.as_array(C.cast(zp, C.POINTER(C.c_double)), shape=(m, 2))
            z = z[:, 0] + 1j * z[:, 1]
            f = np.ctypeslib.as_array(C.cast(fp, C.POINTER(C.c_double)), shape=(m, J, 2))
            df = (np.ctypeslib.as_array(C.cast(dfp, C.POINTER(C.c_double)), shape=(m, J, 2))
                  if dfp else None)
            for k, fn in enumerate(fns):
                v, dv = fn(z)
                v = np.broadcast_to(np.asarray(v, np.complex128), (m,))
                f[:, k, 0], f[:, k, 1] = v.real, v.imag
                if df is not None:
                    if dv is None:
                        return 1                      # no derivatives: no winding count
                    dv = np.broadcast_to(np.asarray(dv, np.complex128), (m,))
                    df[:, k, 0], df[:, k, 1] = dv.real, dv.imag
            return 0
        except Exception:                             # reported as an error by the library
            return -1
    return SCALAR_FN(cb)


# ------------------------------------------------------------------ problems
class Problem:
    """A problem handle: coefficient form (nep_inputs.CoeffProblem) or BEM
    (nep_inputs.BemProblem)."""

    def __init__(self, prob):
        lib = load()
        h = C.c_void_p()
        self.n = prob.n
        self._keep = []
        if hasattr(prob, "xyz"):
            xyz = np.ascontiguousarray(prob.xyz, dtype=np.float64)
            check(lib.rsrr_create_bem(C.byref(h), prob.n, xyz.ctypes.data_as(C.POINTER(C.c_double)),
                                      float(prob.h), stream_ptr()))
            self.bem = True
        else:
            J = prob.J
            kinds = (C.c_int * J)(*[MAT_KIND[k] for k in prob.kinds])
            ptrs = (C.c_void_p * J)()
            for k in range(J):
                kind, A = prob.kinds[k], prob.mats[k]
                if kind == "identity":
                    ptrs[k] = None
                    continue
                if kind == "diag":
                    arr = np.ascontiguousarray(A, dtype=np.complex128)
                elif kind == "real":
                    arr = np.asfortranarray(np.real(A), dtype=np.float64)
                else:
                    arr = np.asfortranarray(A, dtype=np.complex128)
                self._keep.append(arr)
                ptrs[k] = arr.ctypes.data
            if any(sp[0] == "callable" for sp in prob.fspecs):
                # every f_k comes from its Python function through the callback
                assert all(sp[0] == "callable" for sp in prob.fspecs), "mix of callables and menu specs"
                self._cb = _scalar_callback([sp[1] for sp in prob.fspecs])
                check(lib.rsrr_create_fn(C.byref(h), prob.n, J, kinds, ptrs, C.cast(self._cb, C.c_void_p),
                                         None, stream_ptr()))
            else:
                fns = (fn_t * J)(*[_fn(s) for s in prob.fspecs])
                check(lib.rsrr_create(C.byref(h), prob.n, J, kinds, ptrs, fns, stream_ptr()))
            self._keep = []
            self.bem = False
        self.handle = h

    def close(self):
        if self.handle:
            load().rsrr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sample(self, c: contour_t, prm: params_t, U, S=None):
        """S_hat = [T(z_j)^{-1} U] as a column-major device tensor (NL, n)."""
        n, NL = self.n, prm.N * prm.L
        if S is None:
            S = empty_device(n, NL)
        info = info_t()
        st = check(load().rsrr_sample(self.handle, C.byref(c), C.byref(prm), _ptr(U), n, _ptr(S),
                                      n, C.byref(info)))
        return S, info, st

    def moment_matrix(self, c: contour_t, prm: params_t, S, M=None):
        """M_hat = [M_0 ... M_{K'-1}] of the moment scheme from S_hat, as a
        column-major device tensor (K'L, n)."""
        Kp = prm.Kp if prm.Kp > 0 else prm.N
        if M is None:
            M = empty_device(self.n, Kp * prm.L)
        check(load().rsrr_moment_matrix(self.handle, C.byref(c), C.byref(prm), _ptr(S), self.n,
                                        _ptr(M), self.n))
        return M

    def project(self, c: contour_t, prm: params_t, Q, kS: int, J_max: int = 64):
        torch = _torch()
        B = torch.empty((J_max * kS, kS), dtype=torch.complex128, device="cuda")
        J = C.c_int(0)
        check(load().rsrr_project(self.handle, C.byref(c), C.byref(prm), _ptr(Q), self.n, kS,
                                  _ptr(B), C.byref(J)))
        return B[: J.value * kS], J.value

    def solve(self, c: contour_t, prm: params_t, U=None):
        lib = load()
        r = C.c_void_p()
        st = check(lib.rsrr_solve(self.handle, C.byref(c), C.byref(prm),
                                  _ptr(U) if U is not None else None, C.byref(r)))
        return _take_result(r, self.n, prm, st)

    def workspace_bound(self, c: contour_t, prm: params_t) -> int:
        b = C.c_size_t(0)
        check(load().rsrr_workspace_bound(self.handle, C.byref(c), C.byref(prm), C.byref(b)))
        return b.value


def _take_result(r, n: int, prm: params_t, st: int) -> dict:
    """Copies a library result object to host arrays and frees it."""
    lib = load()
    try:
        info = info_t()
        check(lib.rsrr_result_info(r, C.byref(info)))
        ne = info.n_eig
        lam = np.zeros(ne, np.complex128)
        V = np.zeros((ne, n), np.complex128)
        res = np.zeros(ne)
        resp = np.zeros(ne)
        hs = np.zeros(max(1, prm.K * info.k_S))
        check(lib.rsrr_result_copy(r, lam.ctypes.data, V.ctypes.data, res.ctypes.data,
                                   resp.ctypes.data, hs.ctypes.data))
    finally:
        lib.rsrr_result_free(r)
    return dict(lam=lam, V=V.T, res=res, res_paper=resp, hankel_sigma=hs[: prm.K * info.k_S],
                info=info.as_dict(), status=st)


def solve_batched(problems, contours, params, Us=None):
    """rsrr_solve_batched: Alg. 2 for several problems whose sampling LUs are
    factored together; returns one result dict per problem (as
    Problem.solve)."""
    lib = load()
    k = len(problems)
    hs = (C.c_void_p * k)(*[pr.handle for pr in problems])
    cs = (contour_t * k)(*contours)
    ps = (params_t * k)(*params)
    us = None if Us is None else (C.c_void_p * k)(*[None if u is None else u.data_ptr() for u in Us])
    outs = (C.c_void_p * k)()
    st = check(lib.rsrr_solve_batched(k, hs, cs, ps, us, outs))
    res = []
    for i in range(k):
        r = _take_result(C.c_void_p(outs[i]), problems[i].n, params[i], st)
        r["status"] = r["info"]["status"]
        res.append(r)
    return res


class Server:
    """Continuous-batching request loop (rsrr_server_*): submit solves of any
    problems; each runs in one of max_slots concurrent slots once it fits the
    device-memory budget."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int):
        self.handle = C.c_void_p()
        check(load().rsrr_server_create(C.byref(self.handle), int(hbm_budget_bytes), int(max_slots)))
        self._req = {}

    def submit(self, prob: "Problem", c: contour_t, prm: params_t, U: np.ndarray | None = None) -> int:
        t = C.c_uint64(0)
        Uh = None if U is None else np.asfortranarray(U, dtype=np.complex128)
        check(load().rsrr_server_submit(self.handle, prob.handle, C.byref(c), C.byref(prm),
                                        None if Uh is None else Uh.ctypes.data, C.byref(t)))
        self._req[t.value] = (prob.n, prm)
        return t.value

    def wait(self, ticket: int, timeout_s: float = 0.0):
        """(result dict as Problem.solve returns it, latency in seconds);
        timeout_s > 0 bounds the wait (RsrrError with code ETIMEDOUT and the
        server state in its message; the ticket stays valid)."""
        n, prm = self._req[ticket]
        r = C.c_void_p()
        lat = C.c_double(0)
        st = check(load().rsrr_server_wait(self.handle, C.c_uint64(ticket), float(timeout_s), C.byref(r),
                                           C.byref(lat)))
        del self._req[ticket]
        return _take_result(r, n, prm, st), lat.value

    def pending(self):
        q, r = C.c_int(0), C.c_int(0)
        check(load().rsrr_server_pending(self.handle, C.byref(q), C.byref(r)))
        return q.value, r.value

    def close(self):
        if self.handle:
            load().rsrr_server_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def orthonormalize(S, rows: int, cols: int, delta: float = 1e-14):
    """Orthonormal basis of the columns of a device matrix (column-major)."""
    torch = _torch()
    Q = torch.empty((min(rows, cols), rows), dtype=torch.complex128, device="cuda")
    k = C.c_int(0)
    check(load().rsrr_orthonormalize(rows, cols, _ptr(S), rows, float(delta), _ptr(Q), rows,
                                     C.byref(k), stream_ptr()))
    return Q[: k.value], k.value


def timers_enable(on: bool = True):
    load().rsrr_timers_enable(int(on))


def tune_lu(precision: str, n: int, batch: int):
    """(best panel width, its time in ms) from rsrr_tune_lu."""
    nb, ms = C.c_int(0), C.c_double(0)
    check(load().rsrr_tune_lu({"c128": PREC_C128, "c64_ir": PREC_C64_IR}[precision], n, batch, C.byref(nb),
                              C.byref(ms)))
    return nb.value, ms.value


def tune_save(path: str):
    check(load().rsrr_tune_save(path.encode()))


def tune_load(path: str) -> int:
    return check(load().rsrr_tune_load(path.encode()))


def timers_only(sym: str | None):
    """Times only the launches of one kernel function (None: every class)."""
    load().rsrr_timers_only(None if sym is None else sym.encode())


def timers_reset():
    load().rsrr_timers_reset()


def timers_read() -> dict:
    """{kernel class: {launches, ms, flops, bytes}} accumulated since reset."""
    lib = load()
    out = {}
    for i in range(lib.rsrr_timers_count()):
        name = C.create_string_buffer(128)
        la, ms, fl, by = C.c_longlong(), C.c_double(), C.c_double(), C.c_double()
        check(lib.rsrr_timers_get(i, name, 128, C.byref(la), C.byref(ms), C.byref(fl), C.byref(by)))
        out[name.value.decode()] = dict(launches=la.value, ms=ms.value, flops=fl.value,
                                        bytes=by.value)
    return out


OPS = {"N": 0, "T": 1, "C": 2}


def gemm(opA: str, opB: str, A, B, Cm, M: int, N: int, K: int, alpha=1.0, beta=0.0,
         lda=None, ldb=None, ldc=None, batch: int = 1, sA=0, sB=0, sC=0, gauss3m=False):
    """Batched complex GEMM on device tensors (complex128 or complex64)."""
    torch = _torch()
    lib = load()
    lda = lda or (M if opA == "N" else K)
    ldb = ldb or (K if opB == "N" else N)
    ldc = ldc or M
    al = cplx(float(np.real(alpha)), float(np.imag(alpha)))
    be = cplx(float(np.real(beta)), float(np.imag(beta)))
    if Cm.dtype == torch.complex128:
        return check(lib.rsrr_zgemm_batched(OPS[opA], OPS[opB], M, N, K, al, _ptr(A), lda, sA,
                                            _ptr(B), ldb, sB, be, _ptr(Cm), ldc, sC, batch,
                                            stream_ptr()))
    return check(lib.rsrr_cgemm_batched(OPS[opA], OPS[opB], M, N, K, al, _ptr(A), lda, sA,
                                        _ptr(B), ldb, sB, be, _ptr(Cm), ldc, sC, batch,
                                        int(gauss3m), stream_ptr()))


def gesv(A, B, n: int, nrhs: int, batch: int, nb: int = 64, noalloc: bool = False, status: bool = True):
    """Batched LU solve in place (A: batch x n x n, B: batch x n x nrhs,
    column-major); noalloc uses the entry point whose work space is the
    library's fixed device array.  status=False passes no status buffer (the
    allocation-free call then only enqueues its kernels); the returned list is
    then empty."""
    torch = _torch()
    prec = PREC_C128 if A.dtype == torch.complex128 else PREC_C64_IR
    info = (C.c_int * batch)() if status else None
    f = load().rsrr_gesv_batched_noalloc if noalloc else load().rsrr_gesv_batched
    st = f(prec, n, nrhs, _ptr(A), n, n * n, _ptr(B), n, n * nrhs, batch, nb, info, stream_ptr())
    return st, list(info) if status else []
