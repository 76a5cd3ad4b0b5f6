"""ctypes binding of librbws.so (C ABI in include/rbws.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Device buffers are torch tensors on a ROCm device (``tensor.data_ptr()``);
streams are torch streams.  Importing this module imports torch, then loads
the library (so that both use torch's HIP runtime), and raises if it has not
been built (``python -m paper_2311_13862_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbws.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENUMERIC = 0, -1, -2, -3, -4, -5
KIND_BLOCKS, KIND_OCTANTS, KIND_OCTANTS_ANISO = 0, 1, 2
F_ONE, F_GAUSS = 0, 1
INIT_ZERO, INIT_RB, INIT_LEARNED = 0, 1, 2
FP64, FP32_IR = 0, 1
PREC_NONE, PREC_JACOBI, PREC_MG = 0, 1, 2
SOLVE_CONVERGED, SOLVE_MAXITER, SOLVE_BREAKDOWN, SOLVE_NAN = 0, 1, 2, 3
LIFT_EXACT, LIFT_MFMA = 0, 1
IR_RESTART, IR_RELIABLE = 0, 1
FLAG_FORCE_EXACT_DOTS = 1
FLAG_NO_GRAPH = 2
FLAG_EXPLICIT_FALLBACK = 4


class RbwsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rbws error {code}: {msg}")
        self.code = code


class ProblemDesc(C.Structure):
    _fields_ = [("n", C.c_int), ("kind", C.c_int), ("nblocks", C.c_int),
                ("blocks", C.POINTER(C.c_int)), ("f_kind", C.c_int), ("gauss_width", C.c_double)]


class SolveStat(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer_iters", C.c_int), ("extra_spmv", C.c_int),
                ("status", C.c_int), ("init_used", C.c_int), ("vcycles", C.c_int),
                ("init_rr", C.c_double), ("final_rr", C.c_double), ("ff", C.c_double),
                ("t_done_ms", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("precond", C.c_int),
                ("precision", C.c_int), ("init", C.c_int), ("lift", C.c_int),
                ("eta_inner", C.c_double), ("max_outer", C.c_int), ("fallback", C.c_int),
                ("flags", C.c_int), ("check_every", C.c_int), ("ir_mode", C.c_int),
                ("mg_nu", C.c_int), ("mg_omega", C.c_double)]


class MlpDesc(C.Structure):
    _fields_ = [("p", C.c_int), ("nout", C.c_int), ("hidden", C.c_int), ("depth", C.c_int),
                ("log_cols", C.c_int), ("in_m", C.c_double), ("in_s", C.c_double),
                ("lin_lo", C.c_double), ("lin_hi", C.c_double), ("out_pow", C.c_double)]


class MlpTrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_double), ("lr_min", C.c_double),
                ("seed", C.c_ulonglong), ("use_graph", C.c_int)]


_RUNTIMES = ("libamdhip64", "libhsa-runtime64")


def mapped_runtimes() -> dict:
    """Paths of the HIP and HSA runtime libraries mapped into this process, by
    library name (read from /proc/self/maps)."""
    found = {k: set() for k in _RUNTIMES}
    with open("/proc/self/maps") as fh:
        for line in fh:
            parts = line.split()
            if len(parts) < 6:
                continue
            path = parts[-1]
            base = os.path.basename(path)
            for k in _RUNTIMES:
                if base.startswith(k + ".so"):
                    found[k].add(path)
    return found


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_13862_amd.build`")
    # torch provides the device memory and streams the library works on, so the
    # library must bind torch's HIP runtime.  torch ships its own libamdhip64 and
    # libhsa-runtime64 and links them by their unversioned names; loaded first,
    # librbws.so would pull in the system copies under their versioned names,
    # torch would then map its own pair as well, and with two runtimes in one
    # process the library's runtime sees no device.  Importing torch first maps
    # torch's pair, whose sonames then satisfy librbws.so's dependencies.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    # (only the HIP runtime is checked: a profiler that preloads its own HSA
    # runtime maps a second libhsa-runtime64 without harm)
    hip = sorted(mapped_runtimes()["libamdhip64"])
    if len(hip) > 1:
        raise ImportError(f"two copies of the HIP runtime are mapped after loading {LIB_PATH}: {hip}")
    vp, i, d, ll = C.c_void_p, C.c_int, C.c_double, C.c_longlong
    dp = C.POINTER(C.c_double)
    sigs = {
        "rbws_last_error": (C.c_char_p, []),
        "rbws_version": (C.c_char_p, []),
        "rbws_solve_opts_default": (None, [C.POINTER(SolveOpts)]),
        "rbws_problem_create": (i, [C.POINTER(ProblemDesc), i, C.POINTER(vp)]),
        "rbws_problem_destroy": (None, [vp]),
        "rbws_rb_residual_estimate": (i, [vp, dp, i, dp, dp, vp]),
        "rbws_mg_apply": (i, [vp, dp, i, i, d, vp, vp, i, vp]),
        "rbws_problem_info": (i, [vp, C.POINTER(i), C.POINTER(i), C.POINTER(i), C.POINTER(ll)]),
        "rbws_theta": (i, [vp, dp, i, dp]),
        "rbws_spmv": (i, [vp, dp, i, vp, vp, i, vp]),
        "rbws_exact_dots": (i, [vp, vp, ll, i, dp, i, vp]),
        "rbws_exact_dots_noalloc": (i, [vp, vp, ll, i, vp, i, vp]),
        "rbws_stream_copy": (i, [vp, vp, ll, vp]),
        "rbws_solve": (i, [C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), i, C.POINTER(i), dp, i,
                           C.POINTER(SolveOpts), vp, C.POINTER(vp), C.POINTER(SolveStat)]),
    }
    optional = {
        "rbws_rb_build": (i, [vp, dp, i, i, d, i, i, vp, C.POINTER(vp), C.POINTER(i), dp,
                              C.POINTER(i)]),
        "rbws_rb_build_l1roc": (i, [vp, dp, i, i, d, i, i, vp, C.POINTER(vp), C.POINTER(i), dp,
                                    C.POINTER(i)]),
        "rbws_basis_l1roc": (i, [vp, C.POINTER(i), C.POINTER(ll), C.POINTER(i), C.POINTER(ll), C.POINTER(i),
                                 C.POINTER(ll), dp]),
        "rbws_basis_destroy": (None, [vp]),
        "rbws_basis_info": (i, [vp, C.POINTER(i), C.POINTER(i), C.POINTER(ll), dp]),
        "rbws_basis_get": (i, [vp, dp, dp, dp]),
        "rbws_basis_device_v": (i, [vp, C.POINTER(vp)]),
        "rbws_rb_coeffs": (i, [vp, dp, i, dp, vp]),
        "rbws_rb_lift": (i, [vp, vp, i, vp, i, vp]),
        "rbws_basis_save": (i, [vp, C.c_char_p]),
        "rbws_basis_load": (i, [vp, C.c_char_p, C.POINTER(vp)]),
        "rbws_mlp_create": (i, [C.POINTER(MlpDesc), i, C.POINTER(C.c_float), C.c_ulonglong, C.POINTER(vp)]),
        "rbws_mlp_destroy": (None, [vp]),
        "rbws_mlp_param_count": (i, [vp, C.POINTER(ll)]),
        "rbws_mlp_info": (i, [vp, C.POINTER(MlpDesc)]),
        "rbws_mlp_get_params": (i, [vp, C.POINTER(C.c_float)]),
        "rbws_mlp_set_params": (i, [vp, C.POINTER(C.c_float)]),
        "rbws_mlp_set_output_scaling": (i, [vp, dp, dp]),
        "rbws_mlp_get_output_scaling": (i, [vp, dp, dp]),
        "rbws_mlp_fit_output_scaling": (i, [vp, dp, dp, i]),
        "rbws_mlp_predict": (i, [vp, dp, i, dp]),
        "rbws_mlp_forward": (i, [vp, dp, i, C.POINTER(C.c_float)]),
        "rbws_mlp_grad": (i, [vp, dp, dp, i, dp, C.POINTER(C.c_float)]),
        "rbws_mlp_adam_step": (i, [vp, dp, dp, i, d, dp]),
        "rbws_mlp_train": (i, [vp, dp, dp, i, C.POINTER(MlpTrainCfg), dp]),
        "rbws_mlp_save": (i, [vp, C.c_char_p]),
        "rbws_mlp_load": (i, [C.c_char_p, i, C.POINTER(vp)]),
    }
    for name, (res, args) in list(sigs.items()) + list(optional.items()):
        fn = getattr(L, name, None)
        if fn is None:
            if name in sigs:
                raise ImportError(f"{LIB_PATH} does not export {name}")
            continue
        fn.restype = res
        fn.argtypes = args
    return L


_L = _load()


def lib():
    return _L


def _check(code: int):
    if code != OK:
        raise RbwsError(code, _L.rbws_last_error().decode())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def version() -> str:
    return _L.rbws_version().decode()


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    _L.rbws_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Problem:
    """Operator setup (rbws_problem_create) for one grid and parameter family."""

    def __init__(self, spec, device: int = 0):
        self.spec = spec
        blocks = np.ascontiguousarray(np.asarray(spec.blocks, dtype=np.int32).reshape(-1))
        self._blocks = blocks
        bp = blocks.ctypes.data_as(C.POINTER(C.c_int)) if blocks.size else None
        desc = ProblemDesc(spec.n, spec.kind, len(spec.blocks), bp, spec.f_kind, spec.gauss_width)
        h = C.c_void_p()
        _check(_L.rbws_problem_create(C.byref(desc), device, C.byref(h)))
        self.handle = h
        n, p, q, nd = C.c_int(), C.c_int(), C.c_int(), C.c_longlong()
        _check(_L.rbws_problem_info(h, C.byref(n), C.byref(p), C.byref(q), C.byref(nd)))
        self.n, self.p, self.Q, self.ndof = n.value, p.value, q.value, nd.value
        self.device = device

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _L is not None:
            _L.rbws_problem_destroy(h)
            self.handle = None

    def theta(self, mu) -> np.ndarray:
        mu = _f64(mu).reshape(-1, self.p)
        out = np.empty((mu.shape[0], self.Q))
        _check(_L.rbws_theta(self.handle, _dp(mu), mu.shape[0], _dp(out)))
        return out

    def spmv(self, mu, x, y, precision=FP64, stream=None):
        """y[b] = A(mu[b]) x[b]; x, y torch device tensors (nmu, ndof)."""
        mu = _f64(mu).reshape(-1, self.p)
        _check(_L.rbws_spmv(self.handle, _dp(mu), mu.shape[0], C.c_void_p(x.data_ptr()),
                            C.c_void_p(y.data_ptr()), precision, _stream(stream)))

    def mg_apply(self, mu, r, s, nu=1, omega=6.0 / 7.0, precision=FP64, stream=None):
        """s[b] = MG(r[b]), one V-cycle; r, s torch device tensors (nmu, ndof) of
        float64 (FP64) or float32 (FP32_IR)."""
        mu = _f64(mu).reshape(-1, self.p)
        _check(_L.rbws_mg_apply(self.handle, _dp(mu), mu.shape[0], nu, float(omega), C.c_void_p(r.data_ptr()),
                                C.c_void_p(s.data_ptr()), precision, _stream(stream)))


def exact_dots(x, y, flags: int = 0, stream=None) -> np.ndarray:
    """Correctly rounded row-wise dots of two (count, len) float64 device tensors."""
    count, length = x.shape
    out = np.empty(count)
    _check(_L.rbws_exact_dots(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), length, count,
                              _dp(out), flags, _stream(stream)))
    return out


def exact_dots_noalloc(x, y, out, flags: int = 0, stream=None):
    """rbws_exact_dots_noalloc: the same dots as exact_dots, written to the
    float64 device tensor out (count,) on the stream; no allocation, no
    synchronisation (the library's fixed workspace holds the partial sums)."""
    count, length = x.shape
    _check(_L.rbws_exact_dots_noalloc(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), length, count,
                                      C.c_void_p(out.data_ptr()), flags, _stream(stream)))


def stream_copy(src, dst, stream=None):
    """dst = src for two device tensors of the same byte size (a multiple of
    16), with the library's non-temporal streaming copy kernel."""
    nb = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nb
    _check(_L.rbws_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nb, _stream(stream)))


NOALLOC_SCRATCH_BYTES = 4 << 20
NOALLOC_PARTIAL_BYTES = 24  # one double-double partial sum and its error bound


def stats_array(st, n: int) -> np.ndarray:
    """The first n SolveStat records as one numpy structured array: st[b]["iters"]
    for one solve, st["iters"] for the column.  One allocation per batch (a list
    of per-solve dicts would create thousands of Python objects per call)."""
    return np.ctypeslib.as_array(st)[:n].copy()


def solve(problems: Sequence[Problem], mu, opts: SolveOpts, problem_of=None, bases=None,
          mlps=None, u_out=None, stream=None):
    """Batched solve (rbws_solve).  u_out: None or a list of device tensors
    (one per solve).  Returns the per-solve statistics as a numpy structured
    array with SolveStat's fields (stats_array)."""
    problems = list(problems)
    nprob = len(problems)
    p = problems[0].p
    mu = _f64(mu).reshape(-1, p)
    nmu = mu.shape[0]
    ph = (C.c_void_p * nprob)(*[pr.handle for pr in problems])
    bh = (C.c_void_p * nprob)(*[(b.handle if b is not None else None) for b in (bases or [None] * nprob)])
    mh = (C.c_void_p * nprob)(*[(m.handle if m is not None else None) for m in (mlps or [None] * nprob)])
    po = None
    if problem_of is not None:
        po_arr = np.ascontiguousarray(problem_of, dtype=np.int32)
        po = po_arr.ctypes.data_as(C.POINTER(C.c_int))
    uo = None
    if u_out is not None:
        uo = (C.c_void_p * nmu)(*[t.data_ptr() if t is not None else None for t in u_out])
    st = (SolveStat * max(nmu, 1))()
    _check(_L.rbws_solve(ph, bh, mh, nprob, po, _dp(mu), nmu, C.byref(opts), _stream(stream), uo, st))
    return stats_array(st, nmu)


class Basis:
    """Reduced basis handle (rbws_rb_build / rbws_basis_load)."""

    def __init__(self, problem: Problem, handle, selected=None, hist=None):
        self.problem = problem
        self.handle = handle
        N, q, nd, fm = C.c_int(), C.c_int(), C.c_longlong(), C.c_double()
        _check(_L.rbws_basis_info(handle, C.byref(N), C.byref(q), C.byref(nd), C.byref(fm)))
        self.N, self.Q, self.ndof, self.final_max = N.value, q.value, nd.value, fm.value
        self.selected = selected
        self.hist = hist

    @classmethod
    def build(cls, problem: Problem, mu_train, N: int, snap_tol: float, precond=PREC_JACOBI,
              snap_maxit: int = 50000, stream=None, method: str = "galerkin") -> "Basis":
        """Greedy build: method "galerkin" (rbws_rb_build) or "l1roc" (rbws_rb_build_l1roc)."""
        mu = _f64(mu_train).reshape(-1, problem.p)
        nt = mu.shape[0]
        h = C.c_void_p()
        sel = np.full(N, -1, dtype=np.int32)
        hist = np.full((N, nt), np.nan)
        nre = C.c_int()
        fn = {"galerkin": _L.rbws_rb_build, "l1roc": _L.rbws_rb_build_l1roc}[method]
        _check(fn(problem.handle, _dp(mu), nt, N, snap_tol, precond, snap_maxit,
                  _stream(stream), C.byref(h), sel.ctypes.data_as(C.POINTER(C.c_int)),
                  _dp(hist), C.byref(nre)))
        k = nre.value
        return cls(problem, h, sel[:k].copy(), hist[:k].copy())

    @classmethod
    def load(cls, problem: Problem, path: str) -> "Basis":
        h = C.c_void_p()
        _check(_L.rbws_basis_load(problem.handle, path.encode(), C.byref(h)))
        return cls(problem, h)

    def save(self, path: str):
        _check(_L.rbws_basis_save(self.handle, path.encode()))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _L is not None:
            _L.rbws_basis_destroy(h)
            self.handle = None

    def get(self):
        V = np.empty((self.N, self.ndof))
        A = np.empty((self.Q, self.N, self.N))
        f = np.empty(self.N)
        _check(_L.rbws_basis_get(self.handle, _dp(V), _dp(A), _dp(f)))
        return V, A, f

    def coeffs(self, mu, stream=None) -> np.ndarray:
        mu = _f64(mu).reshape(-1, self.problem.p)
        c = np.empty((mu.shape[0], self.N))
        _check(_L.rbws_rb_coeffs(self.handle, _dp(mu), mu.shape[0], _dp(c), _stream(stream)))
        return c

    def l1roc_info(self) -> dict:
        """Collocation points, snapshot and residual DEIM points and T of an L1ROC basis."""
        N = self.N
        npts, nxs, nxr = C.c_int(), C.c_int(), C.c_int()
        pts = np.zeros(2 * N, dtype=np.int64)
        xs = np.zeros(N, dtype=np.int64)
        xr = np.zeros(N, dtype=np.int64)
        T = np.zeros((N, N))
        lp = C.POINTER(C.c_longlong)
        _check(_L.rbws_basis_l1roc(self.handle, C.byref(npts), pts.ctypes.data_as(lp), C.byref(nxs),
                                   xs.ctypes.data_as(lp), C.byref(nxr), xr.ctypes.data_as(lp), _dp(T)))
        return {"pts": pts[:npts.value].copy(), "xs": xs[:nxs.value].copy(), "xr": xr[:nxr.value].copy(), "T": T}

    def residual_estimate(self, mu, c, stream=None) -> np.ndarray:
        """||f - A(mu_b) V c_b|| / ||f|| from the basis's residual decomposition."""
        mu = _f64(mu).reshape(-1, self.problem.p)
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(mu.shape[0], self.N)
        rel = np.empty(mu.shape[0])
        _check(_L.rbws_rb_residual_estimate(self.handle, _dp(mu), mu.shape[0], _dp(c), _dp(rel), _stream(stream)))
        return rel

    def lift(self, c, u, mode=LIFT_EXACT, stream=None):
        """u[b] = V c[b]; c (nmu, N) and u (nmu, ndof) float64 device tensors."""
        _check(_L.rbws_rb_lift(self.handle, C.c_void_p(c.data_ptr()), c.shape[0],
                               C.c_void_p(u.data_ptr()), mode, _stream(stream)))


def _fp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Mlp:
    """Learned start (rbws_mlp_*): a BF16-MFMA multilayer perceptron mu -> c(mu)."""

    def __init__(self, handle):
        self.handle = handle
        desc = MlpDesc()
        _check(_L.rbws_mlp_info(handle, C.byref(desc)))
        self.desc = desc
        n = C.c_longlong()
        _check(_L.rbws_mlp_param_count(handle, C.byref(n)))
        self.nparams = n.value
        self.p, self.nout = desc.p, desc.nout

    @classmethod
    def create(cls, p: int, nout: int, hidden: int = 256, depth: int = 3, log_cols: Optional[int] = None,
               in_m: float = 0.0, in_s: float = 1.0, lin_lo: float = 0.0, lin_hi: float = 1.0,
               out_pow: float = 0.0, params=None, seed: int = 0, device: int = 0) -> "Mlp":
        d = MlpDesc(p, nout, hidden, depth, p if log_cols is None else log_cols, in_m, in_s, lin_lo, lin_hi,
                    out_pow)
        h = C.c_void_p()
        pp = None
        if params is not None:
            params = np.ascontiguousarray(params, dtype=np.float32)
            pp = _fp(params)
        _check(_L.rbws_mlp_create(C.byref(d), device, pp, seed, C.byref(h)))
        return cls(h)

    @classmethod
    def load(cls, path: str, device: int = 0) -> "Mlp":
        h = C.c_void_p()
        _check(_L.rbws_mlp_load(path.encode(), device, C.byref(h)))
        return cls(h)

    def save(self, path: str):
        _check(_L.rbws_mlp_save(self.handle, path.encode()))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _L is not None:
            _L.rbws_mlp_destroy(h)
            self.handle = None

    def get_params(self) -> np.ndarray:
        out = np.empty(self.nparams, dtype=np.float32)
        _check(_L.rbws_mlp_get_params(self.handle, _fp(out)))
        return out

    def set_params(self, params):
        params = np.ascontiguousarray(params, dtype=np.float32)
        assert params.size == self.nparams
        _check(_L.rbws_mlp_set_params(self.handle, _fp(params)))

    def set_output_scaling(self, mean=None, std=None):
        m = None if mean is None else _f64(mean)
        sd = None if std is None else _f64(std)
        _check(_L.rbws_mlp_set_output_scaling(self.handle, None if m is None else _dp(m),
                                              None if sd is None else _dp(sd)))

    def output_scaling(self):
        m = np.empty(self.nout)
        sd = np.empty(self.nout)
        _check(_L.rbws_mlp_get_output_scaling(self.handle, _dp(m), _dp(sd)))
        return m, sd

    def fit_output_scaling(self, mu, c):
        mu = _f64(mu).reshape(-1, self.p)
        c = _f64(c).reshape(-1, self.nout)
        _check(_L.rbws_mlp_fit_output_scaling(self.handle, _dp(mu), _dp(c), mu.shape[0]))

    def predict(self, mu) -> np.ndarray:
        mu = _f64(mu).reshape(-1, self.p)
        c = np.empty((mu.shape[0], self.nout))
        _check(_L.rbws_mlp_predict(self.handle, _dp(mu), mu.shape[0], _dp(c)))
        return c

    def forward(self, mu) -> np.ndarray:
        mu = _f64(mu).reshape(-1, self.p)
        y = np.empty((mu.shape[0], self.nout), dtype=np.float32)
        _check(_L.rbws_mlp_forward(self.handle, _dp(mu), mu.shape[0], _fp(y)))
        return y

    def grad(self, mu, c):
        mu = _f64(mu).reshape(-1, self.p)
        c = _f64(c).reshape(-1, self.nout)
        g = np.empty(self.nparams, dtype=np.float32)
        loss = C.c_double()
        _check(_L.rbws_mlp_grad(self.handle, _dp(mu), _dp(c), mu.shape[0], C.byref(loss), _fp(g)))
        return loss.value, g

    def adam_step(self, mu, c, lr: float) -> float:
        mu = _f64(mu).reshape(-1, self.p)
        c = _f64(c).reshape(-1, self.nout)
        loss = C.c_double()
        _check(_L.rbws_mlp_adam_step(self.handle, _dp(mu), _dp(c), mu.shape[0], lr, C.byref(loss)))
        return loss.value

    def train(self, mu, c, epochs: int = 200, batch: int = 256, lr: float = 1e-3, lr_min: float = 0.0,
              seed: int = 0, use_graph: bool = True) -> np.ndarray:
        mu = _f64(mu).reshape(-1, self.p)
        c = _f64(c).reshape(-1, self.nout)
        cfg = MlpTrainCfg(epochs, batch, lr, lr_min, seed, 1 if use_graph else 0)
        steps = epochs * (mu.shape[0] // batch)
        hist = np.empty(max(steps, 1))
        _check(_L.rbws_mlp_train(self.handle, _dp(mu), _dp(c), mu.shape[0], C.byref(cfg), _dp(hist)))
        return hist[:steps]


def unpack_params(params, p: int, nout: int, hidden: int, depth: int):
    """Split a packed parameter vector into [(W, b), ...] (W of shape (out, in))."""
    out = []
    k = 0
    params = np.asarray(params)
    for layer in range(depth + 1):
        i = p if layer == 0 else hidden
        o = nout if layer == depth else hidden
        W = params[k:k + o * i].reshape(o, i)
        k += o * i
        b = params[k:k + o]
        k += o
        out.append((W, b))
    assert k == params.size
    return out


def pack_params(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([np.asarray(W).ravel(), np.asarray(b).ravel()]) for W, b in layers])


KERNEL_KINDS = ("ap_sweep", "resid_pass", "fin1", "up2_sweep", "fin2", "spmv", "lift_mfma", "rb_coeffs", "mg_vcycle",
                "mg_pre0", "mg_post0", "rb_project")


def profile(enable: bool, reset: bool = True):
    """Kernel times so far (ms, launches per kind), then reset / switch timing."""
    fn = getattr(_L, "rbws_profile")
    fn.restype = C.c_int
    fn.argtypes = [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_longlong), C.c_int]
    ms = (C.c_double * len(KERNEL_KINDS))()
    n = (C.c_longlong * len(KERNEL_KINDS))()
    _check(fn(1 if enable else 0, ms, n, 1 if reset else 0))
    return {k: (ms[i], n[i]) for i, k in enumerate(KERNEL_KINDS)}


def exact_fallbacks(reset: bool = True):
    """Exact-path recomputations since the last reset (solver, basis dots, per-entry, Cholesky)."""
    fn = getattr(_L, "rbws_exact_fallbacks")
    fn.restype = C.c_int
    fn.argtypes = [C.POINTER(C.c_longlong), C.c_int]
    c = (C.c_longlong * 4)()
    _check(fn(c, 1 if reset else 0))
    return {"solver": c[0], "pair_dots": c[1], "entries": c[2], "cholesky": c[3]}


TUNE_SWEEP32 = 0
TUNE_GRID = 1
TUNE_TZ = 2
TUNE_MG_PZ = 3


def set_tuning(key: int, value: int):
    fn = getattr(_L, "rbws_set_tuning")
    fn.restype = C.c_int
    fn.argtypes = [C.c_int, C.c_int]
    _check(fn(key, value))


def autotune(problem: Problem, nsolve: int, precision=FP32_IR, stream=None):
    """Tile-depth autotuner (rbws_autotune): returns (tz, {tz: ms})."""
    fn = getattr(_L, "rbws_autotune")
    fn.restype = C.c_int
    fn.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)]
    tz = C.c_int()
    ms = (C.c_double * 5)()
    _check(fn(problem.handle, nsolve, precision, _stream(stream), C.byref(tz), ms))
    return tz.value, {t: ms[i] for i, t in enumerate((4, 8, 16, 32, 64)) if ms[i] > 0}


def autotune_clear():
    fn = getattr(_L, "rbws_autotune_clear")
    fn.restype = C.c_int
    _check(fn())
