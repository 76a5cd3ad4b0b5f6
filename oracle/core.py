"""ctypes front end of the C oracle (``rbws_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Each function states
the passage of the paper it restates; the arithmetic itself is in the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbws_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

PREC_NONE, PREC_JACOBI = 0, 1
MG_NU, MG_OMEGA = 1, 6.0 / 7.0   # V-cycle defaults: one damped-Jacobi sweep before and after
CONVERGED, MAXITER, BREAKDOWN, NAN = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lquadmath", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int), ("kind", C.c_int), ("nblocks", C.c_int),
                ("blocks", C.POINTER(C.c_int)), ("f_kind", C.c_int),
                ("gauss_width", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("extra_spmv", C.c_int), ("status", C.c_int),
                ("outer", C.c_int), ("init_rr", C.c_double), ("final_rr", C.c_double),
                ("ff", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d, i, l = C.POINTER(C.c_double), C.c_int, C.c_long
        lp = C.POINTER(C.c_long)
        pp = C.POINTER(_Problem)
        sig = {
            "orc_exact_dot": (C.c_double, [d, d, l]),
            "orc_exact_sum": (C.c_double, [d, l]),
            "orc_set_naive_dots": (None, [i]),
            "orc_exp": (C.c_double, [C.c_double]),
            "orc_nq": (i, [pp]),
            "orc_theta": (None, [pp, d, d]),
            "orc_face_coeffs": (None, [pp, d, d, d, d]),
            "orc_apply": (None, [pp, d, d, d]),
            "orc_apply_theta": (None, [pp, d, d, d]),
            "orc_diag": (None, [pp, d, d]),
            "orc_rhs": (None, [pp, d, d]),
            "orc_cg": (i, [pp, d, d, d, i, C.c_double, i, d, C.POINTER(Stats), d]),
            "orc_cg_batch": (None, [pp, d, i, d, d, i, C.c_double, i, d, C.POINTER(Stats), i]),
            "orc_mg_levels": (i, [i, C.POINTER(C.c_int)]),
            "orc_mg_apply": (i, [pp, d, i, C.c_double, d, d]),
            "orc_mg_transfer": (None, [i, i, i, d, d]),
            "orc_mgcg": (i, [pp, d, d, d, i, C.c_double, C.c_double, i, d, C.POINTER(Stats)]),
            "orc_mgcg_batch": (None, [pp, d, i, d, d, i, C.c_double, C.c_double, i, d, C.POINTER(Stats), i]),
            "orc_rb_assemble": (None, [i, i, i, d, d, d]),
            "orc_chol_solve": (i, [i, d, d, d]),
            "orc_lift": (None, [i, l, d, d, d]),
            "orc_rb_coeffs": (i, [pp, i, i, d, d, d, d, d]),
            "orc_indicators": (None, [pp, i, i, d, d, d, d, i, d, i]),
            "orc_greedy": (i, [pp, d, i, i, C.c_double, i, i, d, d, d, C.POINTER(C.c_int), d,
                               C.POINTER(C.c_int), C.POINTER(Stats), i]),
            "orc_ir_solve2": (i, [pp, d, d, d, i, C.c_double, C.c_double, i, i, i, d,
                                  C.POINTER(Stats)]),
            "orc_ir_batch": (None, [pp, d, i, d, d, i, C.c_double, C.c_double, i, i, i, d,
                                    C.POINTER(Stats), i]),
            "orc_l1roc_greedy": (i, [pp, d, i, i, C.c_double, i, i, d, d, lp, C.POINTER(C.c_int), lp, lp,
                                     C.POINTER(C.c_int), C.POINTER(C.c_int), d, C.POINTER(C.c_int), i]),
            "orc_l1roc_coeffs": (i, [pp, i, d, lp, i, d, d]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def nthreads_default() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


class Problem:
    """Problem description (grid, sub-domains, source) held for the C calls."""

    def __init__(self, spec):
        self.spec = spec
        self.n = spec.n
        self.ndof = spec.n ** 3
        self.p = spec.p
        self._blocks = np.ascontiguousarray(np.asarray(spec.blocks, dtype=np.int32).reshape(-1))
        if self._blocks.size == 0:
            self._blocks = np.zeros(6, dtype=np.int32)
        self._c = _Problem(spec.n, spec.kind, len(spec.blocks),
                           self._blocks.ctypes.data_as(C.POINTER(C.c_int)),
                           spec.f_kind, spec.gauss_width)
        self.Q = lib().orc_nq(C.byref(self._c))

    @property
    def ref(self):
        return C.byref(self._c)

    # -- operator (Eq. 1 with the FD discretisation) ---------------------
    def theta(self, mu) -> np.ndarray:
        """theta(mu) of the affine form A(mu) = sum_q theta_q(mu) A_q."""
        mu = _f64(mu)
        out = np.empty(self.Q)
        lib().orc_theta(self.ref, _dp(mu), _dp(out))
        return out

    def face_coeffs(self, theta):
        n = self.n
        m = (n + 1) * n * n
        kx, ky, kz = np.empty(m), np.empty(m), np.empty(m)
        lib().orc_face_coeffs(self.ref, _dp(_f64(theta)), _dp(kx), _dp(ky), _dp(kz))
        return kx, ky, kz

    def apply(self, mu, x) -> np.ndarray:
        """y = A_h(mu) x (unscaled 7-point operator)."""
        x = _f64(x)
        y = np.empty(self.ndof)
        lib().orc_apply(self.ref, _dp(_f64(mu)), _dp(x), _dp(y))
        return y

    def apply_theta(self, theta, x) -> np.ndarray:
        """y = A(theta) x; theta = e_q gives the affine term A_q."""
        y = np.empty(self.ndof)
        lib().orc_apply_theta(self.ref, _dp(_f64(theta)), _dp(_f64(x)), _dp(y))
        return y

    def diag(self, mu) -> np.ndarray:
        d = np.empty(self.ndof)
        lib().orc_diag(self.ref, _dp(_f64(mu)), _dp(d))
        return d

    def rhs(self, mu) -> np.ndarray:
        """f_h(mu) = h^2 f(x_P)."""
        f = np.empty(self.ndof)
        lib().orc_rhs(self.ref, _dp(_f64(mu)), _dp(f))
        return f

    def dense(self, mu) -> np.ndarray:
        """Dense A_h(mu) by applying the operator to unit vectors (tiny n only)."""
        m = self.ndof
        A = np.empty((m, m))
        e = np.zeros(m)
        for i in range(m):
            e[:] = 0.0
            e[i] = 1.0
            A[:, i] = self.apply(mu, e)
        return A

    # -- Alg. 1 ------------------------------------------------------------
    def cg(self, mu, f=None, u0=None, prec=PREC_JACOBI, tol=1e-10, maxit=50000, hist=False):
        """PCG (Alg. 1) from u0 (None = zero); returns (x, stats[, history])."""
        mu = _f64(mu)
        f = self.rhs(mu) if f is None else _f64(f)
        x = np.empty(self.ndof)
        st = Stats()
        h = np.full(maxit + 1, np.nan) if hist else None
        lib().orc_cg(self.ref, _dp(mu), _dp(f), _dp(None if u0 is None else _f64(u0)), prec,
                     tol, maxit, _dp(x), C.byref(st), _dp(h))
        if hist:
            return x, st.as_dict(), h[: st.iters + 1]
        return x, st.as_dict()

    # -- multigrid preconditioner (Alg. 2) and MGCG ----------------------
    def mg_levels(self):
        out = (C.c_int * 16)()
        k = lib().orc_mg_levels(self.n, out)
        return [out[i] for i in range(k)]

    def mg_transfer(self, level: int, x, restrict: bool) -> np.ndarray:
        """Restriction ((n_c+1)/(n_f+1)) P^T x or prolongation P x between levels
        level and level + 1 of the V-cycle (Alg. 2)."""
        ns = self.mg_levels()
        nf, nc = ns[level], ns[level + 1]
        out = np.empty(nc ** 3 if restrict else nf ** 3)
        lib().orc_mg_transfer(nf, nc, 0 if restrict else 1, _dp(_f64(x)), _dp(out))
        return out

    def mg_apply(self, mu, r, nu=MG_NU, omega=MG_OMEGA) -> np.ndarray:
        """s = MG(r): one V-cycle (Alg. 2) with zero initial value."""
        s = np.empty(self.ndof)
        rc = lib().orc_mg_apply(self.ref, _dp(_f64(mu)), nu, omega, _dp(_f64(r)), _dp(s))
        if rc != 0:
            raise ArithmeticError("coarsest operator not positive definite")
        return s

    def mgcg(self, mu, f=None, u0=None, nu=MG_NU, omega=MG_OMEGA, tol=1e-10, maxit=50000):
        """MGCG: Alg. 1 with the V-cycle of Alg. 2 as P; returns (x, stats)."""
        mu = _f64(mu)
        f = self.rhs(mu) if f is None else _f64(f)
        x = np.empty(self.ndof)
        st = Stats()
        lib().orc_mgcg(self.ref, _dp(mu), _dp(f), _dp(None if u0 is None else _f64(u0)), nu, omega, tol, maxit,
                       _dp(x), C.byref(st))
        return x, st.as_dict()

    def mgcg_batch(self, mu, u0=None, nu=MG_NU, omega=MG_OMEGA, tol=1e-10, maxit=50000, nthreads=None):
        mu = _f64(mu)
        B = mu.shape[0]
        f = np.stack([self.rhs(m) for m in mu]) if B else np.zeros((0, self.ndof))
        x = np.empty((B, self.ndof))
        st = (Stats * max(B, 1))()
        lib().orc_mgcg_batch(self.ref, _dp(mu), B, _dp(f), _dp(None if u0 is None else _f64(u0)), nu, omega,
                             tol, maxit, _dp(x), st, nthreads or nthreads_default())
        return x, [st[i].as_dict() for i in range(B)]

    def cg_batch(self, mu, u0=None, prec=PREC_JACOBI, tol=1e-10, maxit=50000, nthreads=None,
                 f=None):
        mu = _f64(mu)
        B = mu.shape[0]
        if f is None:
            f = np.stack([self.rhs(m) for m in mu]) if B else np.zeros((0, self.ndof))
        f = _f64(f)
        x = np.empty((B, self.ndof))
        st = (Stats * max(B, 1))()
        lib().orc_cg_batch(self.ref, _dp(mu), B, _dp(f), _dp(None if u0 is None else _f64(u0)),
                           prec, tol, maxit, _dp(x), st, nthreads or nthreads_default())
        return x, [st[i].as_dict() for i in range(B)]

    # -- FP32-in-FP64 refinement -------------------------------------------
    def ir(self, mu, u0=None, prec=PREC_JACOBI, tol=1e-10, eta=1e-4, kin_max=5000,
           max_outer=40, f=None, reliable=False):
        """FP32-inner / FP64-outer refinement: classic (restart) or reliable updates."""
        mu = _f64(mu)
        f = self.rhs(mu) if f is None else _f64(f)
        u = np.empty(self.ndof)
        st = Stats()
        lib().orc_ir_solve2(self.ref, _dp(mu), _dp(f), _dp(None if u0 is None else _f64(u0)),
                            prec, tol, eta, kin_max, max_outer, 1 if reliable else 0, _dp(u),
                            C.byref(st))
        return u, st.as_dict()

    def ir_batch(self, mu, u0=None, prec=PREC_JACOBI, tol=1e-10, eta=1e-4, kin_max=5000,
                 max_outer=40, nthreads=None, reliable=False):
        mu = _f64(mu)
        B = mu.shape[0]
        f = _f64(np.stack([self.rhs(m) for m in mu]))
        u = np.empty((B, self.ndof))
        st = (Stats * max(B, 1))()
        lib().orc_ir_batch(self.ref, _dp(mu), B, _dp(f), _dp(None if u0 is None else _f64(u0)),
                           prec, tol, eta, kin_max, max_outer, 1 if reliable else 0, _dp(u), st,
                           nthreads or nthreads_default())
        return u, [st[i].as_dict() for i in range(B)]


# -- exact arithmetic ----------------------------------------------------------
def exact_dot(x, y) -> float:
    """Correctly rounded sum_i x_i y_i."""
    x, y = _f64(x), _f64(y)
    assert x.shape == y.shape
    return lib().orc_exact_dot(_dp(x), _dp(y), x.size)


def exp_rn(x: float) -> float:
    """exp(x) rounded to nearest, as the oracle's Gaussian source evaluates it."""
    return lib().orc_exp(float(x))


def set_naive_dots(on: bool) -> None:
    """Process-wide: the solvers' inner products (PCG, refinement) become a
    plain FP64 loop instead of correctly rounded dots.  Only for timing a
    conventional CPU code; every other use keeps the default (off)."""
    lib().orc_set_naive_dots(1 if on else 0)


def exact_sum(x) -> float:
    x = _f64(x)
    return lib().orc_exact_sum(_dp(x), x.size)


# -- reduced basis (Eq. "RB system", Alg. 4, Alg. 5) -----------------------------
@dataclass
class Basis:
    problem: Problem
    V: np.ndarray          # (N, ndof)
    AqN: np.ndarray        # (Q, Nmax, Nmax)
    fN: np.ndarray         # (Nmax,)
    selected: np.ndarray   # (N,)
    hist: np.ndarray       # (Nmax, ntrain)
    snap_stats: list

    @property
    def N(self) -> int:
        return self.V.shape[0]

    def coeffs(self, mu) -> np.ndarray:
        """Galerkin RB coefficients c(mu): A_N(mu) c = b_N(mu), Cholesky."""
        mu = _f64(mu)
        c = np.empty(self.N)
        rc = lib().orc_rb_coeffs(self.problem.ref, self.N, self.AqN.shape[1], _dp(self.AqN),
                                 _dp(self.fN), _dp(self.V), _dp(mu), _dp(c))
        if rc != 0:
            raise FloatingPointError("reduced matrix is not positive definite")
        return c

    def lift(self, c) -> np.ndarray:
        """u0 = V c, each entry a correctly rounded dot."""
        c = _f64(c)
        u = np.empty(self.problem.ndof)
        lib().orc_lift(self.N, self.problem.ndof, _dp(self.V), _dp(c), _dp(u))
        return u

    def indicators(self, mu, nthreads=None) -> np.ndarray:
        mu = _f64(mu)
        out = np.empty(mu.shape[0])
        lib().orc_indicators(self.problem.ref, self.N, self.AqN.shape[1], _dp(self.AqN),
                             _dp(self.fN), _dp(self.V), _dp(mu), mu.shape[0], _dp(out),
                             nthreads or nthreads_default())
        return out


def greedy(problem: Problem, mu_train, N: int, snap_tol: float, prec=PREC_JACOBI,
           snap_maxit=50000, nthreads=None) -> Basis:
    """Greedy RB build (Alg. 4 skeleton): snapshot by Alg. 1, two Gram-Schmidt
    passes, reduced matrices A_q^N = V^T A_q V and f^N = V^T f, residual-norm
    indicator over the training set, argmax with lowest-index tie-break."""
    mu_train = _f64(mu_train)
    nt = mu_train.shape[0]
    m = problem.ndof
    V = np.zeros((N, m))
    AqN = np.zeros((problem.Q, N, N))
    fN = np.zeros(N)
    sel = np.full(N, -1, dtype=np.int32)
    hist = np.full((N, nt), np.nan)
    nre = C.c_int(0)
    st = (Stats * N)()
    rc = lib().orc_greedy(problem.ref, _dp(mu_train), nt, N, snap_tol, prec, snap_maxit,
                          _dp(V), _dp(AqN), _dp(fN), sel.ctypes.data_as(C.POINTER(C.c_int)),
                          _dp(hist), C.byref(nre), st, nthreads or nthreads_default())
    if rc != 0:
        raise FloatingPointError("greedy: reduced matrix breakdown")
    k = nre.value
    return Basis(problem, V[:k].copy(), AqN, fN, sel[:k].copy(), hist[:k].copy(),
                 [st[i].as_dict() for i in range(k)])


class L1rocBasis:
    """An L1ROC basis (Sec. 3.1, Alg. 4): W (N x m, DEIM-normalised), T (W = U T
    with U the snapshots), the collocation points (ascending grid indices), the
    snapshot and residual DEIM points, the selected training indices and the
    L1 indicator history (row k: with k+1 vectors)."""

    def __init__(self, problem, W, T, pts, xs, xr, selected, hist):
        self.problem, self.W, self.T, self.pts = problem, W, T, pts
        self.xs, self.xr, self.selected, self.hist = xs, xr, selected, hist

    @property
    def N(self) -> int:
        return self.W.shape[0]

    def coeffs(self, mu) -> np.ndarray:
        """c = argmin || P (f(mu) - A(mu) W c) || over the collocation points (Householder QR)."""
        mu = _f64(mu)
        c = np.empty(self.N)
        rc = lib().orc_l1roc_coeffs(self.problem.ref, self.N, _dp(self.W),
                                   self.pts.ctypes.data_as(C.POINTER(C.c_long)), len(self.pts), _dp(mu), _dp(c))
        if rc != 0:
            raise FloatingPointError("L1ROC least-squares breakdown")
        return c

    def lift(self, c) -> np.ndarray:
        """u0 = W c, each entry a correctly rounded dot."""
        c = _f64(c)
        u = np.empty(self.problem.ndof)
        lib().orc_lift(self.N, self.problem.ndof, _dp(self.W), _dp(c), _dp(u))
        return u


def l1roc_greedy(problem: Problem, mu_train, N: int, snap_tol: float, prec=PREC_JACOBI,
                 snap_maxit=50000, nthreads=None) -> L1rocBasis:
    """L1ROC offline greedy (Alg. 4): snapshots by Alg. 1, DEIM of each snapshot
    and of the current approximation's residual, L1 indicator over the
    training set, argmax with lowest-index tie-break."""
    mu_train = _f64(mu_train)
    nt = mu_train.shape[0]
    m = problem.ndof
    W = np.zeros((N, m))
    T = np.zeros((N, N))
    pts = np.zeros(2 * N, dtype=np.int64)
    xs = np.zeros(N, dtype=np.int64)
    xr = np.zeros(N, dtype=np.int64)
    npts, nre = C.c_int(0), C.c_int(0)
    nsr = (C.c_int * 2)()
    sel = np.full(N, -1, dtype=np.int32)
    hist = np.full((N, nt), np.nan)
    lp = C.POINTER(C.c_long)
    rc = lib().orc_l1roc_greedy(problem.ref, _dp(mu_train), nt, N, snap_tol, prec, snap_maxit, _dp(W), _dp(T),
                                pts.ctypes.data_as(lp), C.byref(npts), xs.ctypes.data_as(lp),
                                xr.ctypes.data_as(lp), nsr, sel.ctypes.data_as(C.POINTER(C.c_int)), _dp(hist),
                                C.byref(nre), nthreads or nthreads_default())
    if rc != 0:
        raise FloatingPointError("L1ROC greedy: least-squares breakdown")
    k = nre.value
    return L1rocBasis(problem, W[:k].copy(), T[:k, :k].copy(), pts[:npts.value].copy(), xs[:nsr[0]].copy(),
                      xr[:nsr[1]].copy(), sel[:k].copy(), hist[:k].copy())


def rbi_cg(basis: Basis, mu, prec=PREC_JACOBI, tol=1e-10, maxit=50000):
    """Alg. 5: u0 = RB solution, then PCG from it (one continuing run)."""
    u0 = basis.lift(basis.coeffs(mu))
    x, st = basis.problem.cg(mu, u0=u0, prec=prec, tol=tol, maxit=maxit)
    return x, st, u0
