"""ctypes binding of libotgs (include/otgs.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libotgs.so``.  Device arrays are torch tensors on the GPU; the
binding passes their data pointers and the current HIP stream.  Importing
this module on a machine where the library was not built raises
``OSError`` - there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as ct
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libotgs.so")

OT_GS_OK = 0
OT_GS_EINVAL = -1
OT_GS_ESHAPE = -2
OT_GS_EDEVICE = -3
OT_GS_ENUMERIC = -4
OT_GS_ENOMEM = -5
OT_GS_EVERIFY = -6
OT_GS_NOT_CONVERGED = 1
OT_GS_LINESEARCH = 2

OT_GS_DENSE = 0
OT_GS_SCREENED = 1
OT_GS_SNAPSHOT = 2
OT_GS_CHECK = 0x100
OT_GS_VERIFY = 0x200

OT_GS_SOLVER_LBFGS = 0
OT_GS_SOLVER_AGD = 1

OT_GS_COST_GIVEN = 0
OT_GS_COST_MATERIALIZE = 1
OT_GS_COST_ONTHEFLY = 2

KERNEL_GRAD, KERNEL_SCREEN, KERNEL_REDUCE, KERNEL_LBFGS = 0, 1, 2, 3
NBUCKET = 13   # row buckets of the tile lists; tile-configuration bucket NBUCKET = split chunks


class ot_gs_problem(ct.Structure):
    _fields_ = [("n_src", ct.c_int), ("n_tgt", ct.c_int), ("dim", ct.c_int), ("n_groups", ct.c_int),
                ("labels", ct.c_void_p), ("cost_mode", ct.c_int), ("cost", ct.c_void_p),
                ("x_src", ct.c_void_p), ("x_tgt", ct.c_void_p), ("cost_scale", ct.c_float),
                ("a", ct.c_void_p), ("b", ct.c_void_p), ("gamma", ct.c_double), ("mu", ct.c_double)]


class ot_gs_stats(ct.Structure):
    _fields_ = [(n, ct.c_longlong) for n in ("evals", "pairs_total", "pairs_in_N", "pairs_checked",
                                             "pairs_unskipped", "refreshes", "tiles_total",
                                             "tiles_computed")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class ot_gs_options(ct.Structure):
    _fields_ = [("max_iter", ct.c_int), ("hist", ct.c_int), ("refresh", ct.c_int),
                ("use_screen", ct.c_int), ("use_lower", ct.c_int), ("max_ls", ct.c_int),
                ("init_user", ct.c_int), ("c1", ct.c_double), ("c2", ct.c_double),
                ("gtol", ct.c_double), ("obj_trace", ct.c_void_p), ("time_trace", ct.c_void_p),
                ("use_graph", ct.c_int), ("verify", ct.c_int), ("recenter", ct.c_int), ("solver", ct.c_int),
                ("stats_trace", ct.c_void_p), ("gnorm_trace", ct.c_void_p), ("resume", ct.c_int),
                ("recenter_tol", ct.c_double)]


class ot_gs_info(ct.Structure):
    _fields_ = [("iters", ct.c_int), ("evals", ct.c_int), ("status", ct.c_int),
                ("obj", ct.c_double), ("gnorm_inf", ct.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with `python -m paper_2303_07597_amd.build` "
                      "(there is no CPU fallback)")
    lib = ct.CDLL(LIB_PATH)
    vp, i, d = ct.c_void_p, ct.c_int, ct.c_double
    lib.ot_gs_create.argtypes = [ct.POINTER(ot_gs_problem), i, ct.POINTER(vp), vp]
    lib.ot_gs_destroy.argtypes = [vp]
    lib.ot_gs_destroy.restype = None
    lib.ot_gs_dual_grad.argtypes = [vp, vp, vp, vp, vp, vp, i, vp]
    lib.ot_gs_solve.argtypes = [vp, ct.POINTER(ot_gs_options), vp, vp, ct.POINTER(ot_gs_info), vp]
    lib.ot_gs_default_options.argtypes = [ct.POINTER(ot_gs_options)]
    lib.ot_gs_default_options.restype = None
    lib.ot_gs_plan.argtypes = [vp, vp, vp, vp, vp]
    lib.ot_gs_plan_csr.argtypes = [vp, vp, vp, vp, vp, vp, ct.POINTER(ct.c_longlong), vp]
    lib.ot_gs_cost.argtypes = [vp, vp, vp]
    lib.ot_gs_rho_to_mu.argtypes = [d, d, ct.POINTER(d), ct.POINTER(d)]
    lib.ot_gs_get_stats.argtypes = [vp, ct.POINTER(ot_gs_stats), i, vp]
    lib.ot_gs_kernel_timing.argtypes = [vp, i]
    lib.ot_gs_kernel_time.argtypes = [vp, i, ct.POINTER(d), ct.POINTER(ct.c_longlong)]
    lib.ot_gs_profile_tiles.argtypes = [vp, vp, vp, i, ct.POINTER(d), vp]
    lib.ot_gs_layout_info.argtypes = [vp, i, ct.POINTER(i), ct.POINTER(i), ct.POINTER(i)]
    lib.ot_gs_mlp_create.argtypes = [i, i, i, ct.POINTER(vp)]
    lib.ot_gs_mlp_destroy.argtypes = [vp]
    lib.ot_gs_mlp_destroy.restype = None
    lib.ot_gs_mlp_n_params.argtypes = [vp]
    lib.ot_gs_mlp_set_params.argtypes = [vp, vp, vp]
    lib.ot_gs_mlp_get_params.argtypes = [vp, vp, vp]
    lib.ot_gs_mlp_forward.argtypes = [vp, vp, ct.c_longlong, vp, vp]
    lib.ot_gs_mlp_loss_grad.argtypes = [vp, vp, vp, i, vp, vp, vp]
    lib.ot_gs_mlp_train.argtypes = [vp, vp, vp, ct.c_longlong, i, i, ct.c_float, vp, vp]
    lib.ot_gs_features.argtypes = [ct.POINTER(ot_gs_problem), i, ct.POINTER(ct.c_float), vp, vp]
    lib.ot_gs_cost_scale.argtypes = [vp, ct.POINTER(ct.c_float)]
    lib.ot_gs_warm_start.argtypes = [vp, vp, ct.POINTER(ot_gs_problem), vp, vp, vp]
    lib.ot_gs_autotune.argtypes = [vp, i, vp]
    lib.ot_gs_tile_config.argtypes = [vp, i, i, i]
    lib.ot_gs_get_tile_config.argtypes = [vp, i, ct.POINTER(i), ct.POINTER(i), ct.POINTER(i)]
    lib.ot_gs_check.argtypes = [vp, vp]
    lib.ot_gs_workspace_size.argtypes = [ct.POINTER(ot_gs_problem), i, i, ct.POINTER(ct.c_size_t), vp]
    lib.ot_gs_create_ws.argtypes = [ct.POINTER(ot_gs_problem), i, i, vp, ct.c_size_t, ct.POINTER(vp), vp]
    lib.ot_gs_transport.argtypes = [vp, vp, vp, vp, i, vp, vp]
    lib.ot_gs_solver_state_size.argtypes = [vp, ct.POINTER(ct.c_size_t)]
    lib.ot_gs_solver_save.argtypes = [vp, vp, ct.c_size_t, vp]
    lib.ot_gs_solver_load.argtypes = [vp, vp, ct.c_size_t, vp]
    lib.ot_gs_screen_state.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.ot_gs_last_error.restype = ct.c_char_p
    lib.ot_gs_version.restype = ct.c_char_p
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


class OTGSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"otgs error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc < 0:
        raise OTGSError(rc, lib().ot_gs_last_error().decode())
    return rc


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensors only")
    if not t.is_contiguous():
        raise ValueError("contiguous tensors only")
    return ct.c_void_p(t.data_ptr())


def ot_gs_version():
    return lib().ot_gs_version().decode()


def ot_gs_rho_to_mu(gamma, rho):
    g, m = ct.c_double(), ct.c_double()
    _check(lib().ot_gs_rho_to_mu(gamma, rho, ct.byref(g), ct.byref(m)))
    return g.value, m.value


def problem_array(problems):
    """ctypes array of ot_gs_problem for a list of problem dicts (see Handle)."""
    n = len(problems)
    arr = (ot_gs_problem * n)()
    n_src, n_tgt = [], []
    for k, p in enumerate(problems):
        labels = p["labels"]
        mode = p.get("cost_mode", OT_GS_COST_GIVEN if p.get("cost") is not None else OT_GS_COST_MATERIALIZE)
        ns = int(labels.numel())
        nt = int(p["cost"].shape[1]) if p.get("cost") is not None else int(p["x_tgt"].shape[0])
        dim = int(p["x_src"].shape[1]) if p.get("x_src") is not None else 0
        arr[k] = ot_gs_problem(ns, nt, dim, int(p["n_groups"]), _ptr(labels), mode,
                               _ptr(p.get("cost")), _ptr(p.get("x_src")), _ptr(p.get("x_tgt")),
                               float(p.get("cost_scale", 0.0)), _ptr(p.get("a")), _ptr(p.get("b")),
                               float(p["gamma"]), float(p["mu"]))
        n_src.append(ns)
        n_tgt.append(nt)
    return arr, n_src, n_tgt


def workspace_size(problems, max_hist=10, stream=None):
    """Device bytes a handle of these problems needs in a caller workspace."""
    arr, _, _ = problem_array(problems)
    nb = ct.c_size_t()
    _check(lib().ot_gs_workspace_size(arr, len(problems), int(max_hist), ct.byref(nb), _stream(stream)))
    return nb.value


def features(problems, scales, F, stream=None):
    """Warm-start features of the problems into F (float32 cuda
    [sum n_src + sum n_tgt, dim + 8]); scales: per-instance cost scales."""
    arr, _, _ = problem_array(problems)
    sc = (ct.c_float * len(problems))(*[float(x) for x in scales])
    _check(lib().ot_gs_features(arr, len(problems), sc, _ptr(F), _stream(stream)))


class Mlp:
    """Owner of an ``ot_gs_mlp`` (warm-start network)."""

    def __init__(self, d_in, width=256, max_rows=65536):
        m = ct.c_void_p()
        _check(lib().ot_gs_mlp_create(int(d_in), int(width), int(max_rows), ct.byref(m)))
        self.m = m
        self.d_in, self.width, self.max_rows = d_in, width, max_rows
        self.n_params = lib().ot_gs_mlp_n_params(m)

    def close(self):
        if getattr(self, "m", None):
            lib().ot_gs_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p, stream=None):
        _check(lib().ot_gs_mlp_set_params(self.m, _ptr(p), _stream(stream)))

    def get_params(self, stream=None):
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(lib().ot_gs_mlp_get_params(self.m, _ptr(p), _stream(stream)))
        return p

    def forward(self, F, out=None, stream=None):
        if out is None:
            out = torch.empty(F.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().ot_gs_mlp_forward(self.m, _ptr(F), int(F.shape[0]), _ptr(out), _stream(stream)))
        return out

    def loss_grad(self, F, y, stream=None):
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(lib().ot_gs_mlp_loss_grad(self.m, _ptr(F), _ptr(y), int(F.shape[0]), _ptr(loss), _ptr(g),
                                         _stream(stream)))
        return loss, g

    def train(self, F, y, batch, epochs, lr, loss_trace=None, stream=None):
        _check(lib().ot_gs_mlp_train(self.m, _ptr(F), _ptr(y), int(F.shape[0]), int(batch), int(epochs),
                                     float(lr), _ptr(loss_trace), _stream(stream)))


class Handle:
    """Owner of an ``ot_gs_handle``.  ``problems`` is a list of dicts with keys
    labels (int32 cuda), n_groups, gamma, mu and either cost (float32 cuda
    [n_src, n_tgt]) or x_src / x_tgt (float32 cuda) with cost_mode; optional
    a, b, cost_scale.  Tensors are referenced only during creation."""

    def __init__(self, problems, stream=None, workspace=None, max_hist=10):
        """workspace: None (the library allocates), or a cuda uint8 tensor of
        at least workspace_size(problems, max_hist) bytes that the handle
        keeps its device memory in (the tensor must outlive the handle)."""
        if isinstance(problems, dict):
            problems = [problems]
        arr, self.n_src, self.n_tgt = problem_array(problems)
        n = len(problems)
        h = ct.c_void_p()
        if workspace is None:
            _check(lib().ot_gs_create(arr, n, ct.byref(h), _stream(stream)))
        else:
            _check(lib().ot_gs_create_ws(arr, n, int(max_hist), _ptr(workspace), workspace.numel(), ct.byref(h),
                                         _stream(stream)))
        self.workspace = workspace
        self.h = h
        self.count = n

    def close(self):
        if getattr(self, "h", None):
            lib().ot_gs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- calls
    def dual_grad(self, alpha, beta, grad_alpha=None, grad_beta=None, obj=None,
                  mode=OT_GS_DENSE, stream=None):
        _check(lib().ot_gs_dual_grad(self.h, _ptr(alpha), _ptr(beta), _ptr(grad_alpha),
                                     _ptr(grad_beta), _ptr(obj), int(mode), _stream(stream)))

    def solve(self, alpha=None, beta=None, stream=None, obj_trace=None, time_trace=None, stats_trace=None,
              gnorm_trace=None, **opts):
        o = ot_gs_options()
        lib().ot_gs_default_options(ct.byref(o))
        for k, v in opts.items():
            setattr(o, k, v)
        if obj_trace is not None:
            o.obj_trace = _ptr(obj_trace).value
        if time_trace is not None:
            o.time_trace = _ptr(time_trace).value
        if stats_trace is not None:
            o.stats_trace = _ptr(stats_trace).value
        if gnorm_trace is not None:
            o.gnorm_trace = _ptr(gnorm_trace).value
        dev = torch.device("cuda")
        if alpha is None:
            alpha = torch.zeros(sum(self.n_src), dtype=torch.float32, device=dev)
        if beta is None:
            beta = torch.zeros(sum(self.n_tgt), dtype=torch.float32, device=dev)
        info = (ot_gs_info * self.count)()
        rc = _check(lib().ot_gs_solve(self.h, ct.byref(o), _ptr(alpha), _ptr(beta), info, _stream(stream)))
        return alpha, beta, [x.as_dict() for x in info], rc

    def prepare_dual_grad(self, alpha, beta, grad_alpha=None, grad_beta=None, obj=None,
                          mode=OT_GS_DENSE, stream=None):
        """The same call as dual_grad with its arguments marshalled once:
        returns a function of no arguments that enqueues one evaluation
        (for loops that evaluate at buffers whose contents change in place)."""
        f = lib().ot_gs_dual_grad
        args = (self.h, _ptr(alpha), _ptr(beta), _ptr(grad_alpha), _ptr(grad_beta), _ptr(obj),
                int(mode), _stream(stream))
        keep = (alpha, beta, grad_alpha, grad_beta, obj)

        def call():
            rc = f(*args)
            if rc < 0:
                _check(rc)
            return keep
        return call

    def plan(self, alpha, beta, T, stream=None):
        _check(lib().ot_gs_plan(self.h, _ptr(alpha), _ptr(beta), _ptr(T), _stream(stream)))

    def plan_csr(self, alpha, beta, stream=None):
        """The plan in CSR form: (row_ptr int64 [sum n_src + 1], col_idx int32
        [nnz], val float32 [nnz]) on the device (ot_gs_plan_csr's two calls)."""
        dev = alpha.device
        row_ptr = torch.empty(sum(self.n_src) + 1, dtype=torch.int64, device=dev)
        nnz = ct.c_longlong()
        _check(lib().ot_gs_plan_csr(self.h, _ptr(alpha), _ptr(beta), _ptr(row_ptr), None, None, ct.byref(nnz),
                                    _stream(stream)))
        col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(nnz.value, 1), dtype=torch.float32, device=dev)
        _check(lib().ot_gs_plan_csr(self.h, _ptr(alpha), _ptr(beta), _ptr(row_ptr), _ptr(col), _ptr(val), None,
                                    _stream(stream)))
        return row_ptr, col[:nnz.value], val[:nnz.value]

    def check(self, stream=None):
        _check(lib().ot_gs_check(self.h, _stream(stream)))

    def screen_state(self, n_groups, stream=None):
        """(alpha_s, beta_s, z_snap, o_snap, in_N): the snapshot point in the
        caller's order and per-(label, target) snapshot norms and set-N flags,
        instance blocks of n_groups[k] x n_tgt[k] concatenated."""
        dev = torch.device("cuda")
        npairs = sum(L * m for L, m in zip(n_groups, self.n_tgt))
        a = torch.empty(sum(self.n_src), dtype=torch.float32, device=dev)
        b = torch.empty(sum(self.n_tgt), dtype=torch.float32, device=dev)
        z = torch.empty(max(npairs, 1), dtype=torch.float32, device=dev)
        o = torch.empty_like(z)
        n = torch.empty(max(npairs, 1), dtype=torch.uint8, device=dev)
        _check(lib().ot_gs_screen_state(self.h, _ptr(a), _ptr(b), _ptr(z), _ptr(o), _ptr(n), _stream(stream)))
        return a, b, z[:npairs], o[:npairs], n[:npairs]

    def transport(self, alpha, beta, x_src, stream=None):
        """Barycentric mapping y_j = (1/b_j) sum_i T_ij x_i of the source
        features x_src (cuda [sum n_src, dim]) onto the targets."""
        y = torch.empty((sum(self.n_tgt), x_src.shape[1]), dtype=torch.float32, device=x_src.device)
        _check(lib().ot_gs_transport(self.h, _ptr(alpha), _ptr(beta), _ptr(x_src), int(x_src.shape[1]), _ptr(y),
                                     _stream(stream)))
        return y

    def solver_state(self, stream=None):
        """The handle's L-BFGS solver state as bytes (ot_gs_solver_save)."""
        n = ct.c_size_t()
        _check(lib().ot_gs_solver_state_size(self.h, ct.byref(n)))
        buf = ct.create_string_buffer(n.value)
        _check(lib().ot_gs_solver_save(self.h, buf, n.value, _stream(stream)))
        return buf.raw

    def load_solver_state(self, data, stream=None):
        """Restore a state from solver_state() (ot_gs_solver_load)."""
        buf = ct.create_string_buffer(bytes(data), len(data))
        _check(lib().ot_gs_solver_load(self.h, buf, len(data), _stream(stream)))

    def cost(self, C_out, stream=None):
        _check(lib().ot_gs_cost(self.h, _ptr(C_out), _stream(stream)))

    def stats(self, reset=False, stream=None):
        st = ot_gs_stats()
        _check(lib().ot_gs_get_stats(self.h, ct.byref(st), int(reset), _stream(stream)))
        return st.as_dict()

    def kernel_timing(self, enable=True):
        _check(lib().ot_gs_kernel_timing(self.h, int(enable)))

    def kernel_time(self, which):
        ms, n = ct.c_double(), ct.c_longlong()
        _check(lib().ot_gs_kernel_time(self.h, int(which), ct.byref(ms), ct.byref(n)))
        return ms.value, n.value

    def profile_tiles(self, repeats=100, alpha=None, beta=None, stream=None):
        us = ct.c_double()
        _check(lib().ot_gs_profile_tiles(self.h, _ptr(alpha) if alpha is not None else None,
                                         _ptr(beta) if beta is not None else None, int(repeats), ct.byref(us),
                                         _stream(stream)))
        return us.value

    def cost_scale(self):
        sc = (ct.c_float * self.count)()
        _check(lib().ot_gs_cost_scale(self.h, sc))
        return [float(x) for x in sc]

    def warm_start(self, mlp, problems, stream=None):
        """Predicted starting point (alpha, beta) of every instance."""
        arr, _, _ = problem_array(problems)
        alpha = torch.empty(sum(self.n_src), dtype=torch.float32, device="cuda")
        beta = torch.empty(sum(self.n_tgt), dtype=torch.float32, device="cuda")
        _check(lib().ot_gs_warm_start(self.h, mlp.m, arr, _ptr(alpha), _ptr(beta), _stream(stream)))
        return alpha, beta

    def autotune(self, repeats=10, stream=None):
        _check(lib().ot_gs_autotune(self.h, int(repeats), _stream(stream)))

    def tile_config(self, bucket, variant, grid_mult):
        _check(lib().ot_gs_tile_config(self.h, int(bucket), int(variant), int(grid_mult)))

    def get_tile_config(self, bucket):
        v, g, n = ct.c_int(), ct.c_int(), ct.c_int()
        _check(lib().ot_gs_get_tile_config(self.h, int(bucket), ct.byref(v), ct.byref(g), ct.byref(n)))
        return dict(variant=v.value, grid_mult=g.value, n_tiles=n.value)

    def layout_info(self, k=0):
        g, tp, nt = ct.c_int(), ct.c_int(), ct.c_int()
        _check(lib().ot_gs_layout_info(self.h, k, ct.byref(g), ct.byref(tp), ct.byref(nt)))
        return dict(n_groups_nonempty=g.value, n_tgt_padded=tp.value, n_tiles=nt.value)


EXPORTED = [
    "ot_gs_create", "ot_gs_destroy", "ot_gs_dual_grad", "ot_gs_solve", "ot_gs_default_options",
    "ot_gs_plan", "ot_gs_cost", "ot_gs_rho_to_mu", "ot_gs_get_stats", "ot_gs_kernel_timing", "ot_gs_kernel_time",
    "ot_gs_layout_info", "ot_gs_last_error", "ot_gs_version", "ot_gs_profile_tiles",
    "ot_gs_mlp_create", "ot_gs_mlp_destroy", "ot_gs_mlp_n_params", "ot_gs_mlp_set_params",
    "ot_gs_mlp_get_params", "ot_gs_mlp_forward", "ot_gs_mlp_loss_grad", "ot_gs_mlp_train",
    "ot_gs_features", "ot_gs_cost_scale", "ot_gs_warm_start",
    "ot_gs_autotune", "ot_gs_tile_config", "ot_gs_get_tile_config", "ot_gs_check", "ot_gs_screen_state",
    "ot_gs_transport", "ot_gs_workspace_size", "ot_gs_create_ws",
    "ot_gs_solver_state_size", "ot_gs_solver_save", "ot_gs_solver_load",
    "ot_gs_plan_csr",
]
