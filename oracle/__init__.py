"""FP64 CPU oracle for group-sparse smooth-dual optimal transport.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference the HIP library is checked against.  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code with ``paper_2303_07597_amd`` and never imports
it.

The arithmetic lives in ``otgs_oracle.c`` (double precision, compiled with
gcc without fast-math); this module marshals numpy arrays into it.  Each
wrapper names the passage of the paper it follows:

  * :func:`dual_grad`   - objective of the smooth relaxed dual (Eq. 4) and its
                          gradient through the closed-form soft threshold of
                          Eq. 5; grad_alpha = a - T 1, grad_beta = b - T^T 1.
  * :func:`plan`        - plan recovery t_j = grad psi(alpha + beta_j 1 - c_j).
  * :func:`primal`      - primal objective of Eqs. 2-3.
  * :func:`group_norms` - z_lj (Def. 1), o_lj and k_lj (Def. 2).
  * :func:`upper_bound` - Eq. 6;  :func:`lower_bound` - Eq. 7.
  * :func:`gradpsi`     - Algorithm 2 with the Theorem 1 counters.
  * :func:`solve`       - Algorithm 1 around L-BFGS (screening on), or the
                          original dense method (screening off).
  * :func:`cost_sqeuclid` - c_ij = ||x_i - y_j||^2 (Sec. 2.1).
  * :func:`rho_form`    - the (gamma, rho) parameterisation of the
                          experiments mapped to (gamma, mu).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "otgs_oracle.c")
_SO = os.path.join(_HERE, "liborc.so")
_lib = None

_dp = ct.POINTER(ct.c_double)
_ip = ct.POINTER(ct.c_int)


class _Problem(ct.Structure):
    _fields_ = [("ns", ct.c_int), ("nt", ct.c_int), ("L", ct.c_int),
                ("C", _dp), ("labels", _ip), ("a", _dp), ("b", _dp),
                ("gamma", ct.c_double), ("mu", ct.c_double)]


class _State(ct.Structure):
    _fields_ = [("alpha_s", _dp), ("beta_s", _dp), ("Zs", _dp), ("Os", _dp), ("Ks", _dp),
                ("inN", ct.POINTER(ct.c_ubyte)),
                ("s_i", ct.c_longlong), ("s_n", ct.c_longlong),
                ("s_u", ct.c_longlong), ("s_r", ct.c_longlong)]


class _Opts(ct.Structure):
    _fields_ = [("max_iter", ct.c_int), ("hist", ct.c_int), ("r", ct.c_int),
                ("use_screen", ct.c_int), ("use_lower", ct.c_int), ("max_ls", ct.c_int),
                ("c1", ct.c_double), ("c2", ct.c_double), ("gtol", ct.c_double), ("nthreads", ct.c_int)]


class _AgdOpts(ct.Structure):
    _fields_ = [("max_iter", ct.c_int), ("r", ct.c_int), ("use_screen", ct.c_int), ("use_lower", ct.c_int),
                ("max_bt", ct.c_int), ("gtol", ct.c_double), ("shrink", ct.c_double), ("momentum", ct.c_int)]


class _Info(ct.Structure):
    _fields_ = [("iters", ct.c_int), ("evals", ct.c_int), ("status", ct.c_int),
                ("obj", ct.c_double), ("gnorm_inf", ct.c_double),
                ("s_i", ct.c_longlong), ("s_n", ct.c_longlong),
                ("s_u", ct.c_longlong), ("s_r", ct.c_longlong)]


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/liborc.so`` (gcc, -O3, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-fno-fast-math", "-fopenmp",
                               "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ct.CDLL(_SO)
        P = ct.POINTER(_Problem)
        _lib.orc_dual_grad.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp]
        _lib.orc_dual_grad_par.argtypes = [P, _dp, _dp, _dp, _dp, _dp, ct.c_int]
        _lib.orc_primal.argtypes = [P, _dp]
        _lib.orc_primal.restype = ct.c_double
        _lib.orc_group_norms.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        _lib.orc_upper_bound.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp]
        _lib.orc_lower_bound.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        _lib.orc_gradpsi.argtypes = [P, ct.POINTER(_State), _dp, _dp, _dp, _dp, _dp]
        _lib.orc_extract.argtypes = [P, ct.POINTER(_State), _dp, _dp]
        _lib.orc_snapshot.argtypes = [P, ct.POINTER(_State), _dp, _dp]
        _lib.orc_solve.argtypes = [P, ct.POINTER(_Opts), _dp, _dp, ct.POINTER(_Info), _dp]
        _lib.orc_agd_solve.argtypes = [P, ct.POINTER(_AgdOpts), _dp, _dp, ct.POINTER(_Info), _dp]
        _lib.orc_cost_sqeuclid.argtypes = [ct.c_int, ct.c_int, ct.c_int, _dp, _dp, _dp]
    return _lib


def _d(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(x):
    return None if x is None else x.ctypes.data_as(_dp)


class Problem:
    """A problem instance in double precision.  ``C`` [n_src, n_tgt]; labels in
    [0, n_groups); marginals default to uniform a = 1/n_src, b = 1/n_tgt."""

    def __init__(self, C, labels, n_groups, gamma, mu, a=None, b=None):
        self.C = _d(C)
        self.ns, self.nt = self.C.shape
        self.labels = np.ascontiguousarray(labels, dtype=np.int32)
        self.L = int(n_groups)
        self.a = _d(np.full(self.ns, 1.0 / self.ns) if a is None else a)
        self.b = _d(np.full(self.nt, 1.0 / self.nt) if b is None else b)
        self.gamma, self.mu = float(gamma), float(mu)
        self._s = _Problem(self.ns, self.nt, self.L, _ptr(self.C),
                           self.labels.ctypes.data_as(_ip), _ptr(self.a), _ptr(self.b),
                           self.gamma, self.mu)

    @property
    def ref(self):
        return ct.byref(self._s)

    def group_sizes(self):
        return np.bincount(self.labels, minlength=self.L)


def dual_grad(P: Problem, alpha, beta, want_plan=False):
    """(grad_alpha, grad_beta, D[, T]) at (alpha, beta)."""
    al, be = _d(alpha), _d(beta)
    ga, gb = np.empty(P.ns), np.empty(P.nt)
    D = ct.c_double()
    T = np.empty((P.ns, P.nt)) if want_plan else None
    rc = lib().orc_dual_grad(P.ref, _ptr(al), _ptr(be), _ptr(ga), _ptr(gb), ct.byref(D), _ptr(T))
    assert rc == 0, rc
    return (ga, gb, D.value, T) if want_plan else (ga, gb, D.value)


def dual_grad_par(P: Problem, alpha, beta, nthreads=0):
    """dual_grad's values (bit for bit) from OpenMP threads over the target
    columns; nthreads 0 = the OpenMP default."""
    al, be = _d(alpha), _d(beta)
    ga, gb = np.empty(P.ns), np.empty(P.nt)
    D = ct.c_double()
    rc = lib().orc_dual_grad_par(P.ref, _ptr(al), _ptr(be), _ptr(ga), _ptr(gb), ct.byref(D), int(nthreads))
    assert rc == 0, rc
    return ga, gb, D.value


def dual_obj(P: Problem, alpha, beta):
    return dual_grad(P, alpha, beta)[2]


def plan(P: Problem, alpha, beta):
    return dual_grad(P, alpha, beta, want_plan=True)[3]


def transport(P: Problem, alpha, beta, X):
    """Barycentric mapping of the source samples X [n_src, d] onto the
    targets with the plan at (alpha, beta): diag(1/b) T^T X, the paper's
    n T^T X_S for uniform b (Sec. 2.1).  T from plan(); a library matmul."""
    T = plan(P, alpha, beta)
    return (T.T @ _d(X)) / P.b[:, None]


def primal(P: Problem, T):
    return lib().orc_primal(P.ref, _ptr(_d(T)))


def group_norms(P: Problem, alpha, beta):
    """(Z, O, K), each [n_groups, n_tgt]: ||[f]_+||, ||[f]_-||, ||f|| per group."""
    Z, O, K = (np.empty((P.L, P.nt)) for _ in range(3))
    rc = lib().orc_group_norms(P.ref, _ptr(_d(alpha)), _ptr(_d(beta)), _ptr(Z), _ptr(O), _ptr(K))
    assert rc == 0
    return Z, O, K


def upper_bound(P: Problem, alpha, beta, alpha_s, beta_s, Zs):
    out = np.empty((P.L, P.nt))
    rc = lib().orc_upper_bound(P.ref, _ptr(_d(alpha)), _ptr(_d(beta)), _ptr(_d(alpha_s)),
                               _ptr(_d(beta_s)), _ptr(_d(Zs)), _ptr(out))
    assert rc == 0
    return out


def lower_bound(P: Problem, alpha, beta, alpha_s, beta_s, Ks, Os):
    out = np.empty((P.L, P.nt))
    rc = lib().orc_lower_bound(P.ref, _ptr(_d(alpha)), _ptr(_d(beta)), _ptr(_d(alpha_s)),
                               _ptr(_d(beta_s)), _ptr(_d(Ks)), _ptr(_d(Os)), _ptr(out))
    assert rc == 0
    return out


class ScreenState:
    """Snapshot (alpha~, beta~, Z~, O~, K~), the set N and the Theorem 1
    counters of Algorithms 1-2."""

    def __init__(self, P: Problem, alpha_s=None, beta_s=None):
        self.P = P
        self.alpha_s = _d(np.zeros(P.ns) if alpha_s is None else alpha_s).copy()
        self.beta_s = _d(np.zeros(P.nt) if beta_s is None else beta_s).copy()
        self.Zs, self.Os, self.Ks = group_norms(P, self.alpha_s, self.beta_s)
        self.inN = np.zeros((P.L, P.nt), dtype=np.uint8)
        self._s = _State(_ptr(self.alpha_s), _ptr(self.beta_s), _ptr(self.Zs), _ptr(self.Os),
                         _ptr(self.Ks), self.inN.ctypes.data_as(ct.POINTER(ct.c_ubyte)), 0, 0, 0, 0)

    @property
    def counters(self):
        return dict(s_i=self._s.s_i, s_n=self._s.s_n, s_u=self._s.s_u, s_r=self._s.s_r)

    def extract(self, alpha, beta):
        assert lib().orc_extract(self.P.ref, ct.byref(self._s), _ptr(_d(alpha)), _ptr(_d(beta))) == 0

    def snapshot(self, alpha, beta):
        assert lib().orc_snapshot(self.P.ref, ct.byref(self._s), _ptr(_d(alpha)), _ptr(_d(beta))) == 0


def gradpsi(P: Problem, S: ScreenState, alpha, beta):
    """Algorithm 2: (grad_alpha, grad_beta, D) using the snapshot in ``S``."""
    ga, gb = np.empty(P.ns), np.empty(P.nt)
    D = ct.c_double()
    rc = lib().orc_gradpsi(P.ref, ct.byref(S._s), _ptr(_d(alpha)), _ptr(_d(beta)),
                           _ptr(ga), _ptr(gb), ct.byref(D))
    assert rc == 0
    return ga, gb, D.value


def solve(P: Problem, max_iter=200, hist=10, r=10, use_screen=False, use_lower=True,
          max_ls=40, c1=1e-4, c2=0.9, gtol=0.0, alpha0=None, beta0=None, nthreads=0):
    """L-BFGS ascent on the dual from (alpha0, beta0) (zeros by default).

    Returns dict(alpha, beta, obj, trace, iters, evals, status, gnorm_inf,
    s_i, s_n, s_u, s_r); ``trace[k]`` is D after k accepted iterations."""
    al = _d(np.zeros(P.ns) if alpha0 is None else alpha0).copy()
    be = _d(np.zeros(P.nt) if beta0 is None else beta0).copy()
    opts = _Opts(int(max_iter), int(hist), int(r), int(bool(use_screen)), int(bool(use_lower)),
                 int(max_ls), float(c1), float(c2), float(gtol), int(nthreads))
    info = _Info()
    trace = np.full(max_iter + 1, np.nan)
    rc = lib().orc_solve(P.ref, ct.byref(opts), _ptr(al), _ptr(be), ct.byref(info), _ptr(trace))
    assert rc == 0
    n = info.iters + 1
    return dict(alpha=al, beta=be, obj=info.obj, trace=trace[:n], iters=info.iters,
                evals=info.evals, status=info.status, gnorm_inf=info.gnorm_inf,
                s_i=info.s_i, s_n=info.s_n, s_u=info.s_u, s_r=info.s_r)


def agd_solve(P: Problem, max_iter=2000, r=10, use_screen=False, use_lower=True, max_bt=60, gtol=0.0,
              shrink=0.8, alpha0=None, beta0=None, momentum=True):
    """Accelerated gradient ascent on the dual (momentum with backtracking
    and function-value restart, in marginal-scaled variables) from (alpha0,
    beta0), zeros by default; with use_screen, Algorithm 1's snapshots and
    set N around it.  Returns the dict of ``solve``; ``trace[k]`` is D after
    k accepted steps."""
    al = _d(np.zeros(P.ns) if alpha0 is None else alpha0).copy()
    be = _d(np.zeros(P.nt) if beta0 is None else beta0).copy()
    opts = _AgdOpts(int(max_iter), int(r), int(bool(use_screen)), int(bool(use_lower)), int(max_bt),
                    float(gtol), float(shrink), int(bool(momentum)))
    info = _Info()
    trace = np.full(max_iter + 1, np.nan)
    rc = lib().orc_agd_solve(P.ref, ct.byref(opts), _ptr(al), _ptr(be), ct.byref(info), _ptr(trace))
    assert rc == 0
    n = info.iters + 1
    return dict(alpha=al, beta=be, obj=info.obj, trace=trace[:n], iters=info.iters,
                evals=info.evals, status=info.status, gnorm_inf=info.gnorm_inf,
                s_i=info.s_i, s_n=info.s_n, s_u=info.s_u, s_r=info.s_r)


def cost_sqeuclid(xs, xt):
    """c_ij = ||x_i - y_j||^2 evaluated term by term in double precision."""
    xs, xt = _d(xs), _d(xt)
    assert xs.shape[1] == xt.shape[1]
    C = np.empty((xs.shape[0], xt.shape[0]))
    lib().orc_cost_sqeuclid(xs.shape[0], xt.shape[0], xs.shape[1], _ptr(xs), _ptr(xt), _ptr(C))
    return C


def cost_normalized(xs, xt):
    """(C / max C, 1 / max C) in double precision."""
    C = cost_sqeuclid(xs, xt)
    s = 1.0 / C.max()
    return C * s, s


def rho_form(gamma, rho):
    """The experiments' regulariser gamma((1-rho)/2 ||t||^2 + rho sum_l ||t_[l]||)
    equals Eq. 3 with gamma' = gamma (1 - rho) and mu' = rho / (1 - rho)."""
    if not (0.0 <= rho < 1.0):
        raise ValueError("rho must lie in [0, 1)")
    return gamma * (1.0 - rho), rho / (1.0 - rho)
