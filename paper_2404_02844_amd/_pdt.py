"""ctypes binding of libpdt (include/pdt.h): argument marshalling only.

Every computation runs in the HIP library.  Device arrays are torch tensors on the
GPU, passed by ``data_ptr()``; streams are torch's current HIP stream.  If the shared
library is missing the binding raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdt.so")

PDT_OK = 0
PDT_ERR_INVALID_ARG = 1
PDT_ERR_OUT_OF_MEMORY = 2
PDT_ERR_DEVICE = 3
PDT_ERR_NOT_CONVERGED = 4
PDT_ERR_NUMERIC = 5

PDT_FP64 = 0
PDT_FP32 = 1
PDT_MIXED = 2

PDT_TAIL_TRUNCATE = 0
PDT_TAIL_LUMP = 1

PDT_INIT_UNIFORM = 0
PDT_INIT_USER = 1
PDT_INIT_LEARNED = 2

PDT_STEP_UNIFORM = 0
PDT_STEP_DIAG = 1

PDT_RESTART_FUNCTION = 0
PDT_RESTART_GRADIENT = 1

STATUS_NAMES = {0: "PDT_OK", 1: "PDT_ERR_INVALID_ARG", 2: "PDT_ERR_OUT_OF_MEMORY", 3: "PDT_ERR_DEVICE",
                4: "PDT_ERR_NOT_CONVERGED", 5: "PDT_ERR_NUMERIC"}


class PdtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class pdt_problem_desc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("D", ctypes.c_int64),
                ("mu", ctypes.POINTER(ctypes.c_double)), ("P", ctypes.c_void_p),
                ("P_on_device", ctypes.c_int), ("gamma", ctypes.c_double),
                ("pmf_threshold", ctypes.c_double), ("tail_mode", ctypes.c_int)]


class pdt_solve_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("init", ctypes.c_int), ("max_iters", ctypes.c_int64),
                ("rel_obj_tol", ctypes.c_double), ("f_star", ctypes.c_double), ("step_L", ctypes.c_double),
                ("history", ctypes.c_void_p), ("model", ctypes.c_void_p), ("scaling", ctypes.c_int),
                ("kkt_tol", ctypes.c_double), ("skip_refine", ctypes.c_int), ("history_stride", ctypes.c_int64),
                ("restart", ctypes.c_int)]


class pdt_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("rejects", ctypes.c_int64), ("objective", ctypes.c_double),
                ("kkt", ctypes.c_double), ("L_used", ctypes.c_double), ("seconds", ctypes.c_double),
                ("converged", ctypes.c_int), ("refine_iters", ctypes.c_int64), ("fell_back_to_cold", ctypes.c_int),
                ("fw_gap", ctypes.c_double), ("status", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class pdt_newton_opts(ctypes.Structure):
    _fields_ = [("max_newton", ctypes.c_int64), ("eps_kkt", ctypes.c_double), ("stage_switch", ctypes.c_double),
                ("cg_rtol", ctypes.c_double), ("cg_max", ctypes.c_int32), ("init", ctypes.c_int32),
                ("stage2_only", ctypes.c_int32), ("history", ctypes.c_void_p), ("f_star", ctypes.c_double),
                ("rel_obj_tol", ctypes.c_double), ("eps_cap", ctypes.c_double)]


class pdt_newton_info(ctypes.Structure):
    _fields_ = [("stage1_iters", ctypes.c_int64), ("stage2_iters", ctypes.c_int64), ("cg_iters", ctypes.c_int64),
                ("line_trials", ctypes.c_int64), ("objective", ctypes.c_double), ("kkt", ctypes.c_double),
                ("seconds", ctypes.c_double), ("converged", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2404_02844_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        L.pdt_make_problem.argtypes = [ctypes.POINTER(pdt_problem_desc), i64, vp, ctypes.POINTER(vp)]
        L.pdt_destroy_problem.argtypes = [vp]
        L.pdt_destroy_problem.restype = None
        L.pdt_solve.argtypes = [vp, vp, ctypes.POINTER(pdt_solve_opts), ctypes.POINTER(pdt_solve_info)]
        L.pdt_objective.argtypes = [vp, vp, dp, vp]
        L.pdt_kkt.argtypes = [vp, vp, dp]
        L.pdt_project_simplex.argtypes = [vp, vp, i64, i64, vp]
        L.pdt_project_simplex_f32.argtypes = [vp, vp, i64, i64, vp]
        L.pdt_problem_bands.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), dp, dp,
                                        ctypes.POINTER(ctypes.c_int64)]
        L.pdt_problem_scaling.argtypes = [vp, dp, dp]
        L.pdt_problem_set_tiles.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.pdt_problem_tiles.argtypes = [vp, i64, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.pdt_replay_kernel.argtypes = [vp, ctypes.c_int, ctypes.c_int, i64]
        L.pdt_problem_set_fx_split.argtypes = [vp, i64, ctypes.c_int]
        L.pdt_problem_fx_split.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_int)]
        L.pdt_problem_set_fx_split.restype = ctypes.c_int
        L.pdt_problem_fx_split.restype = ctypes.c_int
        L.pdt_problem_set_ftr_split.argtypes = [vp, i64, ctypes.c_int]
        L.pdt_problem_ftr_split.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_int)]
        L.pdt_problem_set_ftr_split.restype = ctypes.c_int
        L.pdt_problem_ftr_split.restype = ctypes.c_int
        L.pdt_replay_kernel.restype = ctypes.c_int
        L.pdt_model_create.argtypes = [i64, i64, i64, vp, vp, ctypes.POINTER(vp)]
        L.pdt_model_destroy.argtypes = [vp]
        L.pdt_model_destroy.restype = None
        L.pdt_model_num_params.argtypes = [vp]
        L.pdt_model_num_params.restype = ctypes.c_int64
        L.pdt_model_get_params.argtypes = [vp, vp]
        L.pdt_model_forward.argtypes = [vp, vp, vp, i64]
        L.pdt_model_gradients.argtypes = [vp, vp, vp, i64, vp]
        L.pdt_model_train_step.argtypes = [vp, vp, vp, i64, ctypes.c_float, dp]
        L.pdt_warmstart_features.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64)]
        for name in ("pdt_model_create", "pdt_model_get_params", "pdt_model_forward", "pdt_model_gradients",
                     "pdt_model_train_step", "pdt_warmstart_features"):
            getattr(L, name).restype = ctypes.c_int
        L.pdt_solve_batch.argtypes = [vp, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(pdt_solve_opts), dp,
                                      ctypes.POINTER(pdt_solve_info)]
        L.pdt_solve_batch.restype = ctypes.c_int
        L.pdt_newton_solve.argtypes = [vp, vp, ctypes.POINTER(pdt_newton_opts), ctypes.POINTER(pdt_newton_info)]
        L.pdt_hessian_apply.argtypes = [vp, vp, vp]
        L.pdt_newton_direction.argtypes = [vp, ctypes.c_int, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                           vp, vp, ctypes.POINTER(ctypes.c_int64), dp]
        L.pdt_smooth_rows.argtypes = [vp, vp, i64, i64, ctypes.c_int32, i64, vp]
        L.pdt_smooth_rows_noalloc.argtypes = [vp, vp, i64, i64, ctypes.c_int32, i64, vp]
        for name in ("pdt_newton_solve", "pdt_hessian_apply", "pdt_newton_direction", "pdt_smooth_rows",
                     "pdt_smooth_rows_noalloc"):
            getattr(L, name).restype = ctypes.c_int
        L.pdt_last_error.argtypes = []
        L.pdt_last_error.restype = ctypes.c_char_p
        for name in ("pdt_make_problem", "pdt_solve", "pdt_objective", "pdt_kkt", "pdt_project_simplex",
                     "pdt_project_simplex_f32", "pdt_problem_bands", "pdt_problem_scaling",
                     "pdt_problem_set_tiles", "pdt_problem_tiles"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def pdt_last_error() -> str:
    return lib().pdt_last_error().decode()


def _check(status: int, allow=()) -> int:
    if status != PDT_OK and status not in allow:
        raise PdtError(status, pdt_last_error())
    return status


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


def _f64_host(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.float64)


def pdt_make_problem(mu, P, M: int, gamma: float, pmf_threshold: float, tail_mode: int, stream=None):
    """Create a problem from probe means ``mu`` [D] (host) and outcomes ``P`` [D, N]
    (numpy array on the host, or a float64 torch tensor on the GPU)."""
    mu_h = _f64_host(mu)
    desc = pdt_problem_desc()
    desc.M = int(M)
    desc.D = int(mu_h.shape[0])
    keep = [mu_h]
    if hasattr(P, "data_ptr") and getattr(P, "is_cuda", False):
        if str(P.dtype) != "torch.float64" or not P.is_contiguous():
            raise ValueError("device P must be a contiguous float64 tensor")
        desc.N = int(P.shape[1])
        desc.P = ctypes.c_void_p(P.data_ptr())
        desc.P_on_device = 1
    else:
        P_h = _f64_host(P)
        keep.append(P_h)
        desc.N = int(P_h.shape[1])
        desc.P = P_h.ctypes.data_as(ctypes.c_void_p)
        desc.P_on_device = 0
    desc.mu = mu_h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    desc.gamma = float(gamma)
    desc.pmf_threshold = float(pmf_threshold)
    desc.tail_mode = int(tail_mode)
    out = ctypes.c_void_p()
    stream_arg = ctypes.c_void_p(0) if stream == 0 else _stream_ptr(stream)
    _check(lib().pdt_make_problem(ctypes.byref(desc), 1, stream_arg, ctypes.byref(out)))
    return out


def pdt_destroy_problem(handle) -> None:
    if handle:
        lib().pdt_destroy_problem(handle)


def pdt_solve(handle, Pi, *, precision=PDT_FP64, init=PDT_INIT_UNIFORM, max_iters=1000, rel_obj_tol=0.0,
              f_star=0.0, step_L=0.0, history=None, model=None, scaling=PDT_STEP_UNIFORM, kkt_tol=0.0,
              skip_refine=False, history_stride=1, restart=PDT_RESTART_FUNCTION, allow_not_converged=True) -> dict:
    """Solve in place: ``Pi`` is a contiguous float64 [M, N] GPU tensor."""
    if model is not None and init == PDT_INIT_UNIFORM:
        init = PDT_INIT_LEARNED
    o = pdt_solve_opts(precision=precision, init=init, max_iters=int(max_iters), rel_obj_tol=float(rel_obj_tol),
                       f_star=float(f_star), step_L=float(step_L),
                       history=ctypes.c_void_p(history.data_ptr()) if history is not None else None,
                       model=(model.handle if isinstance(model, Model) else model), scaling=int(scaling),
                       kkt_tol=float(kkt_tol), skip_refine=int(bool(skip_refine)),
                       history_stride=int(history_stride), restart=int(restart))
    info = pdt_solve_info()
    st = _check(lib().pdt_solve(handle, ctypes.c_void_p(Pi.data_ptr()), ctypes.byref(o), ctypes.byref(info)),
                allow=(PDT_ERR_NOT_CONVERGED,) if allow_not_converged else ())
    d = info.as_dict()
    d["status"] = st
    return d


def pdt_objective(handle, Pi, grad=None) -> float:
    f = ctypes.c_double()
    _check(lib().pdt_objective(handle, ctypes.c_void_p(Pi.data_ptr()), ctypes.byref(f),
                               ctypes.c_void_p(grad.data_ptr()) if grad is not None else None))
    return f.value


def pdt_kkt(handle, Pi) -> float:
    k = ctypes.c_double()
    _check(lib().pdt_kkt(handle, ctypes.c_void_p(Pi.data_ptr()), ctypes.byref(k)))
    return k.value


def pdt_newton_solve(handle, Pi, *, max_newton=200, eps_kkt=1e-10, stage_switch=1e-4, cg_rtol=1e-4, cg_max=50,
                     init=PDT_INIT_UNIFORM, stage2_only=False, history=None, f_star=0.0, rel_obj_tol=0.0,
                     eps_cap=1e-9, allow_not_converged=True) -> dict:
    """Two-stage Newton solve in place: ``Pi`` is a contiguous float64 [M, N] GPU tensor.
    ``history``: optional float64 numpy array of at least max_newton + 1 entries."""
    import numpy as np
    if history is not None and (history.dtype != np.float64 or history.size < max_newton + 1
                                or not history.flags["C_CONTIGUOUS"]):
        raise ValueError("history must be a contiguous float64 array of max_newton + 1 entries")
    o = pdt_newton_opts(max_newton=int(max_newton), eps_kkt=float(eps_kkt), stage_switch=float(stage_switch),
                        cg_rtol=float(cg_rtol), cg_max=int(cg_max), init=int(init), stage2_only=int(bool(stage2_only)),
                        history=history.ctypes.data_as(ctypes.c_void_p) if history is not None else None,
                        f_star=float(f_star), rel_obj_tol=float(rel_obj_tol), eps_cap=float(eps_cap))
    info = pdt_newton_info()
    st = _check(lib().pdt_newton_solve(handle, ctypes.c_void_p(Pi.data_ptr()), ctypes.byref(o), ctypes.byref(info)),
                allow=(PDT_ERR_NOT_CONVERGED,) if allow_not_converged else ())
    d = info.as_dict()
    d["status"] = st
    return d


def pdt_hessian_apply(handle, V, HV) -> None:
    """HV = H V for contiguous float64 [M, N] GPU tensors."""
    _check(lib().pdt_hessian_apply(handle, ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(HV.data_ptr())))


def pdt_newton_direction(handle, stage: int, Pi, eps: float, cg_rtol: float, cg_max: int, Dir, row_max=None) -> dict:
    """One Newton direction at ``Pi`` into ``Dir`` (float64 [M, N] GPU tensors); ``row_max``:
    optional int32 [M] GPU tensor for the stage-2 row maxima."""
    it = ctypes.c_int64()
    sl = ctypes.c_double()
    _check(lib().pdt_newton_direction(handle, int(stage), ctypes.c_void_p(Pi.data_ptr()), float(eps),
                                      float(cg_rtol), int(cg_max), ctypes.c_void_p(Dir.data_ptr()),
                                      ctypes.c_void_p(row_max.data_ptr()) if row_max is not None else None,
                                      ctypes.byref(it), ctypes.byref(sl)))
    return {"cg_iters": it.value, "slope": sl.value}


def pdt_smooth_rows(Pi, out=None, divisor: int = 50, skip: int = 100, stream=None):
    """Long-range smoothing of a contiguous float64 [M, N] GPU tensor (Eq. smoothing)."""
    if out is None:
        out = Pi.new_empty(Pi.shape)
    _check(lib().pdt_smooth_rows(ctypes.c_void_p(Pi.data_ptr()), ctypes.c_void_p(out.data_ptr()), int(Pi.shape[0]),
                                 int(Pi.shape[1]), int(divisor), int(skip), _stream_ptr(stream)))
    return out


# doubles of the fixed device array behind pdt_smooth_rows_noalloc (include/pdt.h)
SMOOTH_NOALLOC_MAX_DOUBLES = 8 << 20


def pdt_smooth_rows_noalloc(Pi, out, divisor: int = 50, skip: int = 100, stream=None):
    """pdt_smooth_rows on the library's fixed device array: allocates nothing, so `out`
    (a contiguous float64 [M, N] GPU tensor, may be Pi) must be given."""
    _check(lib().pdt_smooth_rows_noalloc(ctypes.c_void_p(Pi.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         int(Pi.shape[0]), int(Pi.shape[1]), int(divisor), int(skip),
                                         _stream_ptr(stream)))
    return out


def pdt_project_simplex(X, Y=None, stream=None):
    """Row-wise simplex projection of a 2-D float64 or float32 GPU tensor."""
    if Y is None:
        Y = X.new_empty(X.shape)
    rows, cols = int(X.shape[0]), int(X.shape[1])
    fn = lib().pdt_project_simplex if str(X.dtype) == "torch.float64" else lib().pdt_project_simplex_f32
    _check(fn(ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()), rows, cols, _stream_ptr(stream)))
    return Y


def pdt_replay_kernel(handle, kernel: int, precision: int, reps: int) -> None:
    _check(lib().pdt_replay_kernel(handle, int(kernel), int(precision), int(reps)))


def pdt_problem_bands(handle, D: int) -> dict:
    import numpy as np
    lo = np.zeros(D, dtype=np.int32)
    hi = np.zeros(D, dtype=np.int32)
    tail = np.zeros(D, dtype=np.float64)
    L = ctypes.c_double()
    nnz = ctypes.c_int64()
    _check(lib().pdt_problem_bands(handle, lo.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   hi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   tail.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(L),
                                   ctypes.byref(nnz)))
    return {"lo": lo, "hi": hi, "tail": tail, "lipschitz": L.value, "nnz": nnz.value}


def pdt_problem_scaling(handle, M: int) -> dict:
    import numpy as np
    h = np.zeros(M, dtype=np.float64)
    Lw = ctypes.c_double()
    _check(lib().pdt_problem_scaling(handle, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(Lw)))
    return {"hdiag": h, "lipschitz_scaled": Lw.value}


def pdt_problem_set_tiles(handle, instance: int, precision: int, ks_fx: int, ks_ftr: int) -> None:
    _check(lib().pdt_problem_set_tiles(handle, int(instance), int(precision), int(ks_fx), int(ks_ftr)))


def pdt_problem_tiles(handle, instance: int, precision: int) -> tuple:
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(lib().pdt_problem_tiles(handle, int(instance), int(precision), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


class Problem:
    """Owns a problem handle; thin convenience over the pdt_* calls."""

    def __init__(self, mu, P, M, gamma, pmf_threshold, tail_mode, stream=None):
        self.M = int(M)
        self.D = int(len(mu))
        self.N = int(P.shape[1])
        self.handle = pdt_make_problem(mu, P, M, gamma, pmf_threshold, tail_mode, stream)

    @classmethod
    def from_instance(cls, inst, stream=None):
        return cls(inst.mu, inst.P, inst.M, inst.gamma, inst.threshold, inst.tail_mode, stream)

    def solve(self, Pi, **kw):
        return pdt_solve(self.handle, Pi, **kw)

    def objective(self, Pi, grad=None):
        return pdt_objective(self.handle, Pi, grad)

    def kkt(self, Pi):
        return pdt_kkt(self.handle, Pi)

    def bands(self):
        return pdt_problem_bands(self.handle, self.D)

    def newton(self, Pi, **kw):
        return pdt_newton_solve(self.handle, Pi, **kw)

    def hessian(self, V, HV):
        pdt_hessian_apply(self.handle, V, HV)

    def newton_direction(self, stage, Pi, eps, cg_rtol, cg_max, Dir, row_max=None):
        return pdt_newton_direction(self.handle, stage, Pi, eps, cg_rtol, cg_max, Dir, row_max)

    def scaling(self):
        return pdt_problem_scaling(self.handle, self.M)

    def set_tiles(self, precision, ks_fx, ks_ftr):
        pdt_problem_set_tiles(self.handle, 0, precision, ks_fx, ks_ftr)

    def tiles(self, precision):
        return pdt_problem_tiles(self.handle, 0, precision)

    def set_fx_split(self, split):
        _check(lib().pdt_problem_set_fx_split(self.handle, 0, int(split)))

    def fx_split(self):
        v = ctypes.c_int()
        _check(lib().pdt_problem_fx_split(self.handle, 0, ctypes.byref(v)))
        return v.value

    def set_ftr_split(self, split):
        _check(lib().pdt_problem_set_ftr_split(self.handle, 0, int(split)))

    def ftr_split(self):
        v = ctypes.c_int()
        _check(lib().pdt_problem_ftr_split(self.handle, 0, ctypes.byref(v)))
        return v.value

    def close(self):
        if self.handle:
            pdt_destroy_problem(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- warm-start network ------------------------------------------------------------------

def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Model:
    """Owns a warm-start network handle (pdt_model_*)."""

    def __init__(self, n_in: int, hidden: int, n_out: int, params=None, stream=None):
        import numpy as np
        self.n_in, self.hidden, self.n_out = int(n_in), int(hidden), int(n_out)
        out = ctypes.c_void_p()
        p = None
        if params is not None:
            self._p = np.ascontiguousarray(params, dtype=np.float32)
            p = self._p.ctypes.data_as(ctypes.c_void_p)
        _check(lib().pdt_model_create(self.n_in, self.hidden, self.n_out, p, _stream_ptr(stream), ctypes.byref(out)))
        self.handle = out

    @property
    def num_params(self) -> int:
        return int(lib().pdt_model_num_params(self.handle))

    def params(self):
        import numpy as np
        out = np.empty(self.num_params, dtype=np.float32)
        _check(lib().pdt_model_get_params(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def forward(self, X, Y=None):
        if Y is None:
            Y = X.new_empty((X.shape[0], self.n_out))
        _check(lib().pdt_model_forward(self.handle, _dptr(X), _dptr(Y), int(X.shape[0])))
        return Y

    def gradients(self, X, dY, grads=None):
        import torch
        if grads is None:
            grads = torch.empty(self.num_params, dtype=torch.float32, device=X.device)
        _check(lib().pdt_model_gradients(self.handle, _dptr(X), _dptr(dY), int(X.shape[0]), _dptr(grads)))
        return grads

    def train_step(self, X, T, lr: float) -> float:
        loss = ctypes.c_double()
        _check(lib().pdt_model_train_step(self.handle, _dptr(X), _dptr(T), int(X.shape[0]), float(lr),
                                          ctypes.byref(loss)))
        return loss.value

    def close(self):
        if getattr(self, "handle", None):
            lib().pdt_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack_params(layers) -> "np.ndarray":
    """[(W, b), ...] -> the flat FP32 parameter vector W1, b1, W2, b2, ..."""
    import numpy as np
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers]).astype(np.float32)


def unpack_params(vec, sizes) -> list:
    import numpy as np
    out, off = [], 0
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        W = np.asarray(vec[off:off + fin * fout], dtype=np.float64).reshape(fout, fin)
        off += fin * fout
        b = np.asarray(vec[off:off + fout], dtype=np.float64)
        off += fout
        out.append((W, b))
    return out


def pdt_warmstart_features(handle, X) -> int:
    """Features of the problem's real outcomes into the float32 GPU tensor X [bins+1, 258]."""
    bins = ctypes.c_int64()
    _check(lib().pdt_warmstart_features(handle, _dptr(X), ctypes.byref(bins)))
    return bins.value


# ---- batches -------------------------------------------------------------------------------

class BatchProblem:
    """Several independent instances (uneven M, N, D) solved together by pdt_solve_batch."""

    def __init__(self, instances, stream=None):
        import numpy as np
        self.instances = list(instances)
        n = len(self.instances)
        descs = (pdt_problem_desc * n)()
        self._keep = []
        for k, inst in enumerate(self.instances):
            mu = np.ascontiguousarray(inst.mu, dtype=np.float64)
            P = np.ascontiguousarray(inst.P, dtype=np.float64)
            self._keep += [mu, P]
            d = descs[k]
            d.M, d.N, d.D = int(inst.M), int(P.shape[1]), int(mu.shape[0])
            d.mu = mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.P = P.ctypes.data_as(ctypes.c_void_p)
            d.P_on_device = 0
            d.gamma = float(inst.gamma)
            d.pmf_threshold = float(inst.threshold)
            d.tail_mode = int(inst.tail_mode)
        out = ctypes.c_void_p()
        _check(lib().pdt_make_problem(descs, n, _stream_ptr(stream), ctypes.byref(out)))
        self.handle = out

    def solve(self, Pis, *, precision=PDT_FP64, init=PDT_INIT_UNIFORM, max_iters=1000, rel_obj_tol=0.0,
              f_star=None, step_L=0.0, scaling=PDT_STEP_UNIFORM, skip_refine=False, restart=PDT_RESTART_FUNCTION):
        """Every instance's dict carries its own "status"; the call's own is "batch_status"."""
        import numpy as np
        n = len(self.instances)
        ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in Pis])
        o = pdt_solve_opts(precision=precision, init=init, max_iters=int(max_iters), rel_obj_tol=float(rel_obj_tol),
                           f_star=0.0, step_L=float(step_L), history=None, model=None, scaling=int(scaling),
                           skip_refine=int(bool(skip_refine)), restart=int(restart))
        fs = None
        if f_star is not None:
            self._fs = np.ascontiguousarray(f_star, dtype=np.float64)
            fs = self._fs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        infos = (pdt_solve_info * n)()
        st = _check(lib().pdt_solve_batch(self.handle, ptrs, ctypes.byref(o), fs, infos),
                    allow=(PDT_ERR_NOT_CONVERGED,))
        out = [i.as_dict() for i in infos]
        for d in out:
            d["batch_status"] = st
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().pdt_destroy_problem(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
