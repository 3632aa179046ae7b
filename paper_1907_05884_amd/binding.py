"""Python binding of libfst (randomized functional sparse Tucker on MI355X / gfx950).

Argument marshalling only: every step runs in the C-ABI library (host C++ for the host
steps of Algorithm 1, HIP kernels for the GPU path).  Functions carry the names of the C
entry points declared in include/fst.h.  Device arrays are torch tensors on a ROCm device;
torch provides memory and the current stream, nothing else.  Host arrays are numpy arrays.

The library must be built first (``python -m paper_1907_05884_amd.build``); importing this
module without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfst.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1907_05884_amd.build`")
_lib = C.CDLL(LIB_PATH)

FST_OK = 0
FST_E_INVAL, FST_E_NOMEM, FST_E_DEVICE, FST_E_NOT_SPD, FST_E_UNSUPPORTED, FST_E_FORMAT = -1, -2, -3, -4, -5, -6
FST_F64, FST_F32 = 0, 1
FST_GRAM_F64, FST_GRAM_F32, FST_GRAM_BF16, FST_GRAM_F16 = 0, 1, 2, 3
FST_GRAM_F16X2, FST_GRAM_BF16X3, FST_GRAM_BF16X2 = 4, 5, 6
FST_STREAM_INTERP, FST_STREAM_LS = 1, 2
FST_SOLVER_OMP, FST_SOLVER_LARS = 0, 1

_STATUS_NAMES = {-1: "FST_E_INVAL", -2: "FST_E_NOMEM", -3: "FST_E_DEVICE", -4: "FST_E_NOT_SPD",
                 -5: "FST_E_UNSUPPORTED", -6: "FST_E_FORMAT"}


class FstError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class fst_fit_params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("dtype", C.c_int32),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("grid", C.c_int32 * 3), ("rank", C.c_int32 * 3), ("degree", C.c_int32 * 3),
                ("interp_fraction", C.c_double), ("idw_k", C.c_int32), ("idw_power", C.c_double),
                ("n_samples", C.c_int64), ("seed", C.c_uint64), ("gram_prec", C.c_int32),
                ("refine_steps", C.c_int32), ("n_threads", C.c_int32), ("eps", C.c_double),
                ("sparse_solver", C.c_int32), ("wavelet_level", C.c_int32), ("wavelet_degree", C.c_int32)]


class fst_fit_params_d(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("dtype", C.c_int32), ("d", C.c_int32),
                ("lo", C.c_double * 4), ("hi", C.c_double * 4),
                ("grid", C.c_int32 * 4), ("rank", C.c_int32 * 4), ("degree", C.c_int32 * 4),
                ("interp_fraction", C.c_double), ("idw_k", C.c_int32), ("idw_power", C.c_double),
                ("n_samples", C.c_int64), ("seed", C.c_uint64), ("n_threads", C.c_int32), ("eps", C.c_double),
                ("sparse_solver", C.c_int32), ("wavelet_level", C.c_int32), ("wavelet_degree", C.c_int32)]


_vp, _i64, _i32, _dp = C.c_void_p, C.c_int64, C.c_int32, C.POINTER(C.c_double)


def _proto(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


class fst_train_params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("steps", C.c_int32), ("batch", C.c_int32),
                ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("seed", C.c_uint64), ("init_params", C.c_void_p)]


_P = C.POINTER(fst_fit_params)
_TP = C.POINTER(fst_train_params)
_lib_fns = dict(
    fst_last_error=(C.c_char_p,),
    fst_version=(C.c_char_p,),
    fst_fit_params_default=(None, _P),
    fst_fit_workspace_bytes=(C.c_size_t, _P, _i64),
    fst_fit=(_i32, _P, _i64, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp, C.POINTER(_vp)),
    fst_compress_host=(_i32, _P, _i64, _vp, _vp, _vp, _vp, C.POINTER(_vp)),
    fst_refit_workspace_bytes=(C.c_size_t, _vp, _i32, _i64, _i32),
    fst_refit_core=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _i64, C.c_uint64, _i32, _i32, _vp,
                    C.c_size_t, _vp, C.POINTER(_vp)),
    fst_eval=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp),
    fst_factor_eval=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp),
    fst_eval_error_workspace_bytes=(C.c_size_t, _i32, _i64),
    fst_eval_grid_workspace_bytes=(C.c_size_t, _vp, _i32, _i64, _i64, _i64),
    fst_refit_core_mixed_workspace_bytes=(C.c_size_t, _vp, _i32, _i64, _i64),
    fst_refit_core_mixed=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _i64, C.c_uint64, _vp, C.c_size_t, _vp,
                          C.POINTER(_vp)),
    fst_eval_grid=(_i32, _vp, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, C.c_size_t, _vp),
    fst_eval_error=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp, C.c_size_t, _vp, _vp),
    fst_gram_workspace_bytes=(C.c_size_t, _vp, _i64),
    fst_gram=(_i32, _vp, _i32, _i64, _vp, _vp, _i32, _vp, _vp, _vp, C.c_size_t, _vp),
    fst_cholesky_workspace_bytes=(C.c_size_t, _i64),
    fst_cholesky=(_i32, _i64, _vp, C.c_double, C.POINTER(_i64), _vp, C.c_size_t, _vp),
    fst_cholesky_noalloc=(_i32, _i64, _vp, C.c_double, C.POINTER(_i64), _vp),
    fst_solve_core_workspace_bytes=(C.c_size_t, _vp, _i64, _i32),
    fst_solve_core=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _i32, _i32, _vp, _vp, _vp,
                    C.POINTER(_i32), C.POINTER(_i64), C.POINTER(_i32), C.POINTER(C.c_double), _vp, C.c_size_t, _vp),
    fst_model_factor=(_i32, _vp, _i32, _vp, _vp, _vp, C.POINTER(_i64)),
    fst_mixed_rows=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _i64, C.c_uint64, _vp, _vp, _vp, C.c_size_t, _vp),
    fst_leverage=(_i32, _i64, _i64, _i64, _vp, _vp, _vp, _vp),
    fst_cholesky_solve=(_i32, _i64, _vp, _vp, _vp, _vp),
    fst_residual_workspace_bytes=(C.c_size_t, _vp, _i64),
    fst_residual=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, C.c_size_t, _vp),
    fst_refine_workspace_bytes=(C.c_size_t, _vp, _i64),
    fst_refine_step=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, C.c_size_t, _vp),
    fst_sample_indices=(_i32, C.c_uint64, _i32, _i64, _i64, _vp),
    fst_idw_grid=(_i32, _vp, _vp, _i64, _vp, _i32, C.c_double, _i32, _vp),
    fst_sthosvd=(_i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp),
    fst_sthosvd_eps=(_i32, _vp, _vp, C.c_double, _vp, _i32, _vp, _vp, _vp, _vp),
    fst_sparse_fit=(_i32, _vp, _i32, _i32, _i32, _vp),
    fst_sparse_fit_lars=(_i32, _vp, _i32, _i32, _i32, _vp),
    fst_gram_dense_workspace_bytes=(C.c_size_t, _vp, _i32, _i64),
    fst_gram_split_workspace_bytes=(C.c_size_t, _vp, _i32, _i64),
    fst_design_rows=(_i32, _vp, _i32, _i64, _vp, _vp, _i64, _vp, _vp, _vp),
    fst_gram_rows=(_i32, _i32, _i64, _i64, _vp, _vp, _vp, _vp, _i32, _vp),
    fst_sparse_fit_choice=(_i32, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp),
    fst_model_from_parts_wavelet=(_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_vp)),
    fst_model_wavelets=(_i32, _vp, _vp, _vp),
    fst_model_from_parts=(_i32, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_vp)),
    fst_model_from_parts_d=(_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_vp)),
    fst_model_info_d=(_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp),
    fst_eval_d=(_i32, _vp, _i32, _i64, _vp, _vp, _vp),
    fst_refit_core_d_workspace_bytes=(C.c_size_t, _vp, _i32, _i64),
    fst_refit_core_d=(_i32, _vp, _i32, _i64, _vp, _vp, _i64, C.c_uint64, _vp, C.c_size_t, _vp, C.POINTER(_vp)),
    fst_fit_params_d_default=(None, C.POINTER(fst_fit_params_d), _i32),
    fst_fit_d_workspace_bytes=(C.c_size_t, C.POINTER(fst_fit_params_d), _i64),
    fst_fit_d=(_i32, C.POINTER(fst_fit_params_d), _i64, _vp, _vp, _vp, C.c_size_t, _vp, C.POINTER(_vp)),
    fst_compress_host_d=(_i32, C.POINTER(fst_fit_params_d), _i64, _vp, _vp, C.POINTER(_vp)),
    fst_model_free=(None, _vp),
    fst_model_info=(_i32, _vp, _vp, _vp, _vp, _vp, _vp),
    fst_model_core=(_i32, _vp, _vp),
    fst_model_coefs=(_i32, _vp, _i32, _vp),
    fst_model_paper_bytes=(_i64, _vp),
    fst_model_fit_info=(_i32, _vp, C.POINTER(_i32), C.POINTER(_i64), C.POINTER(_i32), C.POINTER(C.c_double)),
    fst_model_save=(_i32, _vp, _vp, C.POINTER(C.c_size_t)),
    fst_model_load=(_i32, _vp, C.c_size_t, C.POINTER(_vp)),
    fst_fit_batched=(_i32, _P, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp),
    fst_eval_batched=(_i32, _vp, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp),
    fst_eval_graph_create=(_i32, _vp, _i32, _i32, _i64, _vp, _vp, _vp, _vp, C.POINTER(_vp)),
    fst_graph_launch=(_i32, _vp, _vp),
    fst_graph_free=(None, _vp),
    fst_train_params_default=(None, _TP),
    fst_corrector_workspace_bytes=(C.c_size_t, _TP, _i64),
    fst_corrector_train=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _TP, _vp, C.c_size_t, _vp, C.POINTER(_vp)),
    fst_corrector_from_params=(_i32, _vp, _vp, _vp, C.c_float, C.POINTER(_vp)),
    fst_corrector_params=(_i32, _vp, _vp, _vp),
    fst_corrector_losses=(_i32, _vp, _vp, C.POINTER(_i32)),
    fst_corrector_free=(None, _vp),
    fst_corrector_stored_bytes=(_i64, _vp),
    fst_corrector_apply=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp),
    fst_eval_corrected=(_i32, _vp, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp),
    fst_mlp_grad_workspace_bytes=(C.c_size_t, _i32),
    fst_mlp_grad=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, C.c_size_t, _vp),
    fst_mlp_grad_fp32=(_i32, _vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, C.c_size_t, _vp),
)
_fn = {name: _proto(name, spec[0], *spec[1:]) for name, spec in _lib_fns.items()}
EXPORTED_SYMBOLS = tuple(_lib_fns)


def _check(status: int):
    if status != FST_OK:
        raise FstError(status, _fn["fst_last_error"]().decode(errors="replace"))


def fst_version() -> str:
    return _fn["fst_version"]().decode()


def fst_last_error() -> str:
    return _fn["fst_last_error"]().decode(errors="replace")


# ------------------------------------------------------------------------------ helpers
def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _torch():
    import torch
    return torch


def _dev_ptr(t):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on a GPU device")
    if not t.is_contiguous():
        raise ValueError("device arrays must be contiguous")
    return C.c_void_p(t.data_ptr())


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return FST_F64
    if t.dtype == torch.float32:
        return FST_F32
    raise TypeError("points and values must be float32 or float64")


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def make_params(dtype=FST_F64, lo=(-1.0,) * 3, hi=(1.0,) * 3, grid=(32,) * 3, rank=(8,) * 3,
                degree=(15,) * 3, interp_fraction=0.10, idw_k=8, idw_power=2.0, n_samples=2000,
                seed=1, gram_prec=None, refine_steps=0, n_threads=0, eps=0.0,
                sparse_solver=FST_SOLVER_OMP, wavelet=None) -> fst_fit_params:
    p = fst_fit_params()
    _fn["fst_fit_params_default"](C.byref(p))
    p.dtype = dtype
    for k in range(3):
        p.lo[k], p.hi[k] = float(lo[k]), float(hi[k])
        p.grid[k], p.rank[k], p.degree[k] = int(grid[k]), int(rank[k]), int(degree[k])
    p.interp_fraction = float(interp_fraction)
    p.idw_k = int(idw_k)
    p.idw_power = float(idw_power)
    p.n_samples = int(n_samples)
    p.seed = int(seed)
    if gram_prec is None:
        gram_prec = FST_GRAM_F64 if dtype == FST_F64 else FST_GRAM_F32
    p.gram_prec = int(gram_prec)
    p.refine_steps = int(refine_steps)
    p.n_threads = int(n_threads)
    p.eps = float(eps)
    p.sparse_solver = int(sparse_solver)
    if wavelet is not None:
        p.wavelet_level, p.wavelet_degree = int(wavelet[0]), int(wavelet[1])
    return p


def make_params_d(d=4, dtype=FST_F64, lo=None, hi=None, grid=None, rank=None, degree=None,
                  interp_fraction=0.10, idw_k=8, idw_power=2.0, n_samples=2000, seed=1, n_threads=0,
                  eps=0.0, sparse_solver=FST_SOLVER_OMP, wavelet=None) -> fst_fit_params_d:
    p = fst_fit_params_d()
    _fn["fst_fit_params_d_default"](C.byref(p), int(d))
    p.dtype = dtype
    for k in range(d):
        if lo is not None:
            p.lo[k], p.hi[k] = float(lo[k]), float(hi[k])
        if grid is not None:
            p.grid[k] = int(grid[k])
        if rank is not None:
            p.rank[k] = int(rank[k])
        if degree is not None:
            p.degree[k] = int(degree[k])
    p.interp_fraction = float(interp_fraction)
    p.idw_k = int(idw_k)
    p.idw_power = float(idw_power)
    p.n_samples = int(n_samples)
    p.seed = int(seed)
    p.n_threads = int(n_threads)
    p.eps = float(eps)
    p.sparse_solver = int(sparse_solver)
    if wavelet is not None:
        p.wavelet_level, p.wavelet_degree = int(wavelet[0]), int(wavelet[1])
    return p


def _detail_count(s, q):
    return (q + 1) * ((1 << s) - 1) if s > 0 else 0


# ------------------------------------------------------------------------------ model
class Model:
    """Owns an fst_model handle."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _fn is not None:
            _fn["fst_model_free"](h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self):
        lo, hi = (C.c_double * 4)(), (C.c_double * 4)()
        rank, degree = (C.c_int32 * 4)(), (C.c_int32 * 4)()
        d, nnz = C.c_int32(), C.c_int64()
        _check(_fn["fst_model_info_d"](self._h, C.byref(d), lo, hi, rank, degree, C.byref(nnz)))
        k = d.value
        return dict(d=k, lo=tuple(lo[:k]), hi=tuple(hi[:k]), rank=tuple(rank[:k]), degree=tuple(degree[:k]),
                    nnz=nnz.value)

    @property
    def d(self) -> int:
        return self.info()["d"]

    @property
    def rank(self):
        return self.info()["rank"]

    @property
    def degree(self):
        return self.info()["degree"]

    @property
    def R(self) -> int:
        return int(np.prod(self.rank))

    @property
    def core(self) -> np.ndarray:
        out = np.empty(self.rank, dtype=np.float64)
        _check(_fn["fst_model_core"](self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def wavelets(self):
        """((s_k, q_k) per mode): the wavelet space held beside P_p (0, 0: Legendre only)."""
        d = self.d
        wl, wd = (C.c_int32 * 4)(), (C.c_int32 * 4)()
        _check(_fn["fst_model_wavelets"](self._h, wl, wd))
        return tuple((wl[k], wd[k]) for k in range(d))

    def coefs(self, k: int) -> np.ndarray:
        inf = self.info()
        s_k, q_k = self.wavelets()[k]
        out = np.empty((inf["degree"][k] + 1 + _detail_count(s_k, q_k), inf["rank"][k]), dtype=np.float64)
        _check(_fn["fst_model_coefs"](self._h, int(k), out.ctypes.data_as(C.c_void_p)))
        return out

    def fit_info(self):
        """(Gram precision the core was solved with, core entries dropped as dependent)."""
        d = self.solve_info()
        return d["gram_prec"], d["dropped"]

    def solve_info(self) -> dict:
        prec, dropped, steps, res = _i32(), _i64(), _i32(), C.c_double()
        _check(_fn["fst_model_fit_info"](self._h, C.byref(prec), C.byref(dropped), C.byref(steps), C.byref(res)))
        return dict(gram_prec=prec.value, dropped=dropped.value, refine_steps=steps.value, rel_residual=res.value)

    def paper_bytes(self) -> int:
        return int(_fn["fst_model_paper_bytes"](self._h))


def fst_model_from_parts(lo, hi, rank, degree, core, coefs, wavelet=None) -> Model:
    """A model of d = len(rank) modes (3: fst_model_from_parts, 4: fst_model_from_parts_d);
    wavelet: per-mode (s_k, q_k) of a wavelet space beside P_p (fst_model_from_parts_wavelet)."""
    d = len(rank)
    if not (len(lo) == len(hi) == len(degree) == len(coefs) == d):
        raise ValueError("lo, hi, rank, degree and coefs need one entry per mode")
    lo_a, lo_p = _host(lo, np.float64)
    hi_a, hi_p = _host(hi, np.float64)
    r_a, r_p = _host(rank, np.int32)
    d_a, d_p = _host(degree, np.int32)
    c_a, c_p = _host(core, np.float64)
    cs = [np.ascontiguousarray(c, dtype=np.float64) for c in coefs]
    wav = tuple(wavelet) if wavelet else ((0, 0),) * d
    for k in range(d):
        if cs[k].shape != (int(degree[k]) + 1 + _detail_count(*wav[k]), int(rank[k])):
            raise ValueError("coefficient matrix k must have shape (rows of mode k's basis, rank[k])")
    if c_a.size != int(np.prod(rank)):
        raise ValueError("core must have r1 .. rd entries")
    arr = (C.c_void_p * d)(*[c.ctypes.data_as(C.c_void_p) for c in cs])
    h = C.c_void_p()
    if wavelet:
        wl_a, wl_p = _host([w[0] for w in wav], np.int32)
        wd_a, wd_p = _host([w[1] for w in wav], np.int32)
        _check(_fn["fst_model_from_parts_wavelet"](d, lo_p, hi_p, r_p, d_p, wl_p, wd_p, c_p, arr, C.byref(h)))
    elif d == 3:
        _check(_fn["fst_model_from_parts"](lo_p, hi_p, r_p, d_p, c_p, arr, C.byref(h)))
    else:
        _check(_fn["fst_model_from_parts_d"](d, lo_p, hi_p, r_p, d_p, c_p, arr, C.byref(h)))
    return Model(h)


def fst_model_save(m: Model) -> bytes:
    n = C.c_size_t(0)
    _check(_fn["fst_model_save"](m.handle, None, C.byref(n)))
    buf = (C.c_ubyte * n.value)()
    _check(_fn["fst_model_save"](m.handle, buf, C.byref(n)))
    return bytes(buf[: n.value])


def fst_model_load(data: bytes) -> Model:
    buf = (C.c_ubyte * len(data)).from_buffer_copy(data)
    h = C.c_void_p()
    _check(_fn["fst_model_load"](buf, len(data), C.byref(h)))
    return Model(h)


# ------------------------------------------------------------------------------ whole method
def fst_fit_workspace_bytes(p: fst_fit_params, n: int) -> int:
    b = _fn["fst_fit_workspace_bytes"](C.byref(p), int(n))
    if b == 0:
        raise FstError(FST_E_INVAL, fst_last_error())
    return int(b)


def fst_fit(p: fst_fit_params, x, y, z, v, ws=None, stream=None) -> Model:
    """Algorithm 1 + Algorithm 2 on device arrays x, y, z, v (torch, same dtype).  With ws
    None the library allocates its workspace (with room for the dense Gram route when the
    device has it free)."""
    n = x.numel()
    h = C.c_void_p()
    _check(_fn["fst_fit"](C.byref(p), n, _dev_ptr(x), _dev_ptr(y), _dev_ptr(z), _dev_ptr(v),
                          _dev_ptr(ws), ws.numel() if ws is not None else 0, _stream(stream), C.byref(h)))
    return Model(h)


def fst_compress_host(p: fst_fit_params, x, y, z, v) -> Model:
    """Algorithm 1 on host numpy arrays (dtype given by p.dtype)."""
    dt = np.float64 if p.dtype == FST_F64 else np.float32
    xs = [_host(a, dt) for a in (x, y, z, v)]
    h = C.c_void_p()
    _check(_fn["fst_compress_host"](C.byref(p), xs[0][0].size, *[t[1] for t in xs], C.byref(h)))
    return Model(h)


def fst_refit_workspace_bytes(m: Model, dtype: int, n_samples: int, refine_steps: int = 0) -> int:
    b = _fn["fst_refit_workspace_bytes"](m.handle, int(dtype), int(n_samples), int(refine_steps))
    if b == 0:
        raise FstError(FST_E_INVAL, fst_last_error())
    return int(b)


def fst_refit_core(m: Model, x, y, z, v, n_samples: int, seed: int, gram_prec=None,
                   refine_steps: int = 0, ws=None, stream=None) -> Model:
    """Algorithm 2: re-estimates the core of m from n_samples uniformly sampled rows.  With
    ws None the library allocates its workspace itself (with room for the dense Gram route
    when the device has it free)."""
    dt = _dtype_code(x)
    if gram_prec is None:
        gram_prec = FST_GRAM_F64 if dt == FST_F64 else FST_GRAM_F32
    n = x.numel()
    h = C.c_void_p()
    _check(_fn["fst_refit_core"](m.handle, dt, n, _dev_ptr(x), _dev_ptr(y), _dev_ptr(z), _dev_ptr(v),
                                 int(n_samples), int(seed), int(gram_prec), int(refine_steps),
                                 _dev_ptr(ws), ws.numel() if ws is not None else 0, _stream(stream),
                                 C.byref(h)))
    return Model(h)


def fst_refit_core_mixed(m: Model, x, y, z, v, n_samples: int, seed: int, ws=None, stream=None) -> Model:
    """Algorithm 2 with its randomised mixing (sign flips, Walsh-Hadamard transform, uniform
    row sampling): re-estimates the core of m from n_samples mixed rows."""
    dt = _dtype_code(x)
    n = x.numel()
    if ws is None:
        ws = _workspace(int(_fn["fst_refit_core_mixed_workspace_bytes"](m.handle, dt, n, int(n_samples))), x.device)
    h = C.c_void_p()
    _check(_fn["fst_refit_core_mixed"](m.handle, dt, n, _dev_ptr(x), _dev_ptr(y), _dev_ptr(z), _dev_ptr(v),
                                       int(n_samples), int(seed), _dev_ptr(ws), ws.numel(), _stream(stream),
                                       C.byref(h)))
    return Model(h)


def fst_solve_core(m: Model, x, y, z, v, idx, U, vs, G, h, gram_prec=None, refine_steps: int = 3, ws=None,
                   stream=None):
    """Algorithm 2 step 5 from the caller's normal equations (G overwritten by its Cholesky
    factor): returns (alpha device FP64 tensor, info dict as Model.solve_info)."""
    torch = _torch()
    dt = _dtype_code(x)
    if gram_prec is None:
        gram_prec = FST_GRAM_F64 if dt == FST_F64 else FST_GRAM_F32
    mrows = idx.numel()
    if ws is None:
        ws = _workspace(int(_fn["fst_solve_core_workspace_bytes"](m.handle, int(mrows), int(gram_prec))), x.device)
    alpha = torch.empty(m.R, dtype=torch.float64, device=x.device)
    prec, dropped, steps, res = _i32(), _i64(), _i32(), C.c_double()
    _check(_fn["fst_solve_core"](m.handle, dt, x.numel(), _dev_ptr(x), _dev_ptr(y), _dev_ptr(z), _dev_ptr(v),
                                 _dev_ptr(idx), int(mrows), _dev_ptr(U), _dev_ptr(vs), int(gram_prec),
                                 int(refine_steps), _dev_ptr(G), _dev_ptr(h), _dev_ptr(alpha), C.byref(prec),
                                 C.byref(dropped), C.byref(steps), C.byref(res), _dev_ptr(ws), ws.numel(),
                                 _stream(stream)))
    return alpha, dict(gram_prec=prec.value, dropped=dropped.value, refine_steps=steps.value,
                       rel_residual=res.value)


def fst_model_factor(m: Model, k: int):
    """Factor k as compressed columns: (colptr int32[r_k + 1], rowidx int32[nnz], vals float64[nnz])."""
    nnz = _i64()
    _check(_fn["fst_model_factor"](m.handle, int(k), None, None, None, C.byref(nnz)))
    r = m.info()["rank"][k]
    colptr = np.empty(r + 1, np.int32)
    rowidx = np.empty(max(nnz.value, 1), np.int32)
    vals = np.empty(max(nnz.value, 1), np.float64)
    _check(_fn["fst_model_factor"](m.handle, int(k), colptr.ctypes.data_as(C.c_void_p),
                                   rowidx.ctypes.data_as(C.c_void_p), vals.ctypes.data_as(C.c_void_p),
                                   C.byref(nnz)))
    return colptr, rowidx[:nnz.value], vals[:nnz.value]


def fst_mixed_rows(m: Model, x, y, z, v, n_samples: int, seed: int, ws=None, stream=None):
    """The sampled mixed rows of Algorithm 2 (sign flips, Walsh-Hadamard transform, uniform
    sample): (At (R x Sp), b (Sp)) device tensors of the points' dtype, zero past n_samples."""
    torch = _torch()
    dt = _dtype_code(x)
    n = x.numel()
    Sp = (int(n_samples) + 63) // 64 * 64
    At = torch.empty((m.R, Sp), dtype=x.dtype, device=x.device)
    b = torch.empty(Sp, dtype=x.dtype, device=x.device)
    if ws is None:
        ws = _workspace(int(_fn["fst_refit_core_mixed_workspace_bytes"](m.handle, dt, n, int(n_samples))), x.device)
    _check(_fn["fst_mixed_rows"](m.handle, dt, n, _dev_ptr(x), _dev_ptr(y), _dev_ptr(z), _dev_ptr(v), int(n_samples),
                                 int(seed), _dev_ptr(At), _dev_ptr(b), _dev_ptr(ws), ws.numel(), _stream(stream)))
    return At, b


def fst_leverage(At, L, mrows=None, out=None, stream=None):
    """Leverage of the rows of At (FP64 R x Sp) given L from fst_cholesky of At At^T."""
    torch = _torch()
    R, Sp = At.shape
    mrows = Sp if mrows is None else int(mrows)
    if out is None:
        out = torch.empty(mrows, dtype=torch.float64, device=At.device)
    _check(_fn["fst_leverage"](int(R), int(Sp), mrows, _dev_ptr(At), _dev_ptr(L), _dev_ptr(out), _stream(stream)))
    return out


def fst_eval(m: Model, x, y, z, out=None, stream=None):
    """Reconstruction u~ at device points; returns `out` (allocated if None)."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(x)
    _check(_fn["fst_eval"](m.handle, _dtype_code(x), x.numel(), _dev_ptr(x), _dev_ptr(y), _dev_ptr(z),
                           _dev_ptr(out), _stream(stream)))
    return out


# ------------------------------------------------------------------------------ d-way calls
def _coord_list(coords):
    if any(c.dtype != coords[0].dtype or c.numel() != coords[0].numel() for c in coords):
        raise ValueError("coordinate arrays must share dtype and length")
    return (C.c_void_p * len(coords))(*[_dev_ptr(c) for c in coords])


def fst_eval_d(m: Model, coords, out=None, stream=None):
    """Reconstruction of a d-way model at device points given as one array per mode."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(coords[0])
    _check(_fn["fst_eval_d"](m.handle, _dtype_code(coords[0]), coords[0].numel(), _coord_list(coords),
                             _dev_ptr(out), _stream(stream)))
    return out


def fst_refit_core_d_workspace_bytes(m: Model, dtype: int, n_samples: int) -> int:
    b = _fn["fst_refit_core_d_workspace_bytes"](m.handle, int(dtype), int(n_samples))
    if b == 0:
        raise FstError(FST_E_INVAL, fst_last_error())
    return int(b)


def fst_refit_core_d(m: Model, coords, v, n_samples: int, seed: int, ws=None, stream=None) -> Model:
    """Algorithm 2 for a d-way model from materialised design-row chunks and the dense MFMA Gram."""
    dt = _dtype_code(coords[0])
    n = coords[0].numel()
    if ws is None:
        ws = _workspace(fst_refit_core_d_workspace_bytes(m, dt, n_samples), coords[0].device)
    h = C.c_void_p()
    _check(_fn["fst_refit_core_d"](m.handle, dt, n, _coord_list(coords), _dev_ptr(v), int(n_samples), int(seed),
                                   _dev_ptr(ws), ws.numel(), _stream(stream), C.byref(h)))
    return Model(h)


def fst_fit_d_workspace_bytes(p: fst_fit_params_d, n: int) -> int:
    b = _fn["fst_fit_d_workspace_bytes"](C.byref(p), int(n))
    if b == 0:
        raise FstError(FST_E_INVAL, fst_last_error())
    return int(b)


def fst_fit_d(p: fst_fit_params_d, coords, v, stream=None) -> Model:
    """Algorithm 1 + Algorithm 2 for a d-way dataset given as device arrays (one per mode)."""
    n = coords[0].numel()
    ws = _workspace(fst_fit_d_workspace_bytes(p, n), coords[0].device)
    h = C.c_void_p()
    _check(_fn["fst_fit_d"](C.byref(p), n, _coord_list(coords), _dev_ptr(v), _dev_ptr(ws), ws.numel(),
                            _stream(stream), C.byref(h)))
    return Model(h)


def fst_compress_host_d(p: fst_fit_params_d, coords, v) -> Model:
    """Algorithm 1 for a d-way dataset on host numpy arrays (dtype given by p.dtype)."""
    dt = np.float64 if p.dtype == FST_F64 else np.float32
    hs = [_host(a, dt) for a in list(coords) + [v]]
    arr = (C.c_void_p * len(coords))(*[t[1] for t in hs[:-1]])
    h = C.c_void_p()
    _check(_fn["fst_compress_host_d"](C.byref(p), hs[0][0].size, arr, hs[-1][1], C.byref(h)))
    return Model(h)


# ------------------------------------------------------------------------------ batched form
def fst_fit_batched(p: fst_fit_params, ranks, degrees, x, y, z, values, stream=None):
    """Fits len(values) variables sharing the points x, y, z.  ranks, degrees: (V, 3) ints.
    Returns (models, timings, gram_prec_used) with timings = host steps, row generation,
    batched Gram, A^T v, solves with refinement (seconds) and the Gram precision each
    variable was solved with."""
    V = len(values)
    r, rp = _host(np.asarray(ranks).reshape(V, 3), np.int32)
    d, dp = _host(np.broadcast_to(np.asarray(degrees).reshape(V, -1), (V, 3)), np.int32)
    vptr = (_vp * V)(*[_dev_ptr(v) for v in values])
    outs = (_vp * V)()
    t = np.zeros(5)
    used = np.zeros(V, np.int32)
    _check(_fn["fst_fit_batched"](C.byref(p), V, rp, dp, x.numel(), _dev_ptr(x), _dev_ptr(y), _dev_ptr(z),
                                  vptr, _stream(stream), outs, used.ctypes.data_as(C.c_void_p),
                                  t.ctypes.data_as(C.c_void_p)))
    return [Model(C.c_void_p(h)) for h in outs], t, used


def fst_eval_batched(models, x, y, z, outs=None, stream=None):
    """Reconstruction of every model at the same device points; returns the list of outputs."""
    torch = _torch()
    V = len(models)
    if outs is None:
        outs = [torch.empty_like(x) for _ in range(V)]
    mp = (_vp * V)(*[m.handle for m in models])
    op = (_vp * V)(*[_dev_ptr(o) for o in outs])
    _check(_fn["fst_eval_batched"](mp, V, _dtype_code(x), x.numel(), _dev_ptr(x), _dev_ptr(y), _dev_ptr(z),
                                   op, _stream(stream)))
    return outs


class EvalGraph:
    """The batched reconstruction captured as a HIP graph.  Holds references to the models and
    tensors it was captured with, which therefore stay alive and in place."""

    def __init__(self, models, x, y, z, outs):
        V = len(models)
        self._keep = (list(models), x, y, z, list(outs))
        mp = (_vp * V)(*[m.handle for m in models])
        op = (_vp * V)(*[_dev_ptr(o) for o in outs])
        h = C.c_void_p()
        _check(_fn["fst_eval_graph_create"](mp, V, _dtype_code(x), x.numel(), _dev_ptr(x), _dev_ptr(y),
                                            _dev_ptr(z), op, C.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(_fn["fst_graph_launch"](self._h, _stream(stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _fn["fst_graph_free"](h)
            self._h = None


def fst_eval_graph_create(models, x, y, z, outs) -> EvalGraph:
    return EvalGraph(models, x, y, z, outs)


def fst_graph_launch(g: EvalGraph, stream=None):
    g.launch(stream)


def fst_graph_free(g: EvalGraph):
    g.__del__()


def fst_eval_error(m: Model, x, y, z, v, ws=None, stream=None):
    """(sum (v - f)^2, sum v^2) of the reconstruction at device points, FP64."""
    dt = _dtype_code(x)
    n = x.numel()
    if ws is None:
        ws = _workspace(int(_fn["fst_eval_error_workspace_bytes"](dt, n)), x.device)
    out = np.zeros(2)
    _check(_fn["fst_eval_error"](m.handle, dt, n, _dev_ptr(x), _dev_ptr(y), _dev_ptr(z), _dev_ptr(v),
                                 _dev_ptr(ws), ws.numel(), _stream(stream), out.ctypes.data_as(C.c_void_p)))
    return float(out[0]), float(out[1])


def fst_eval_grid(m: Model, gx, gy, gz, out=None, ws=None, stream=None):
    """Model on the tensor grid gx x gy x gz (device coordinate tensors of one dtype):
    returns out (n1, n2, n3), C order."""
    torch = _torch()
    dt = _dtype_code(gx)
    n1, n2, n3 = gx.numel(), gy.numel(), gz.numel()
    if out is None:
        out = torch.empty((n1, n2, n3), dtype=gx.dtype, device=gx.device)
    if ws is None:
        ws = _workspace(int(_fn["fst_eval_grid_workspace_bytes"](m.handle, dt, n1, n2, n3)), gx.device)
    _check(_fn["fst_eval_grid"](m.handle, dt, _dev_ptr(gx), n1, _dev_ptr(gy), n2, _dev_ptr(gz), n3,
                                _dev_ptr(out), _dev_ptr(ws), ws.numel(), _stream(stream)))
    return out


# ------------------------------------------------------------------------------ per-step GPU
def fst_factor_eval(m: Model, x, y, z, v=None, idx=None, mrows=None, U=None, vs=None, stream=None):
    """Factor values at rows idx (int32 device tensor or None): returns (U [sum r, m], vs)."""
    torch = _torch()
    n = x.numel()
    if mrows is None:
        mrows = idx.numel() if idx is not None else n
    sr = sum(m.rank)
    if U is None:
        U = torch.empty((sr, mrows), dtype=x.dtype, device=x.device)
    if vs is None and v is not None:
        vs = torch.empty(mrows, dtype=x.dtype, device=x.device)
    _check(_fn["fst_factor_eval"](m.handle, _dtype_code(x), n, _dev_ptr(x), _dev_ptr(y), _dev_ptr(z),
                                  _dev_ptr(v), _dev_ptr(idx), int(mrows), _dev_ptr(U), _dev_ptr(vs),
                                  _stream(stream)))
    return U, vs


def fst_gram_dense_workspace_bytes(m: Model, dtype: int, mrows: int) -> int:
    return int(_fn["fst_gram_dense_workspace_bytes"](m.handle, int(dtype), int(mrows)))


def fst_gram_split_workspace_bytes(m: Model, gram_prec: int, mrows: int) -> int:
    return int(_fn["fst_gram_split_workspace_bytes"](m.handle, int(gram_prec), int(mrows)))


def fst_gram_workspace_bytes(m: Model, mrows: int) -> int:
    return int(_fn["fst_gram_workspace_bytes"](m.handle, int(mrows)))


def fst_gram(m: Model, U, vs=None, gram_prec=None, G=None, h=None, ws=None, stream=None, want_G=True):
    """G = A^T A (lower triangle) and h = A^T vs, FP64 device tensors (want_G=False: h only).
    A workspace of fst_gram_dense_workspace_bytes bytes selects the dense route (design rows
    materialised in it, then a dense MFMA Gram; for BF16/FP16 Grams the rows are 16-bit and G
    equals the other route's bit for bit).  The split precisions (FST_GRAM_F16X2,
    FST_GRAM_BF16X3) need fst_gram_split_workspace_bytes and get it when ws is None."""
    torch = _torch()
    dt = _dtype_code(U)
    if gram_prec is None:
        gram_prec = FST_GRAM_F64 if dt == FST_F64 else FST_GRAM_F32
    R = m.R
    mrows = U.shape[1]
    if G is None and want_G:
        G = torch.zeros((R, R), dtype=torch.float64, device=U.device)
    if h is None and vs is not None:
        h = torch.empty(R, dtype=torch.float64, device=U.device)
    if ws is None:
        need = fst_gram_split_workspace_bytes(m, gram_prec, mrows) or fst_gram_workspace_bytes(m, mrows)
        ws = _workspace(need, U.device)
    _check(_fn["fst_gram"](m.handle, dt, int(mrows), _dev_ptr(U), _dev_ptr(vs), int(gram_prec),
                           _dev_ptr(G) if want_G else None, _dev_ptr(h), _dev_ptr(ws), ws.numel(),
                           _stream(stream)))
    return G, h


def fst_design_rows(m: Model, U, vs=None, Sp=None, At=None, b=None, stream=None):
    """A^T (R x Sp, rows past U.shape[1] zero) and b of the rows whose factor values U holds."""
    torch = _torch()
    mrows = U.shape[1]
    if Sp is None:
        Sp = (mrows + 63) // 64 * 64
    if At is None:
        At = torch.empty((m.R, Sp), dtype=U.dtype, device=U.device)
    if b is None and vs is not None:
        b = torch.empty(Sp, dtype=U.dtype, device=U.device)
    _check(_fn["fst_design_rows"](m.handle, _dtype_code(U), int(mrows), _dev_ptr(U), _dev_ptr(vs), int(Sp),
                                  _dev_ptr(At), _dev_ptr(b), _stream(stream)))
    return At, b


def fst_gram_rows(At, b=None, G=None, h=None, want_G=True, accumulate=False, stream=None):
    """G = At At^T (lower triangle) and h = At b, FP64, from materialised rows."""
    torch = _torch()
    R, Sp = At.shape
    if G is None and want_G:
        G = torch.zeros((R, R), dtype=torch.float64, device=At.device)
    if h is None and b is not None:
        h = torch.empty(R, dtype=torch.float64, device=At.device)
    _check(_fn["fst_gram_rows"](_dtype_code(At), int(R), int(Sp), _dev_ptr(At), _dev_ptr(b),
                                _dev_ptr(G) if want_G else None, _dev_ptr(h), 1 if accumulate else 0,
                                _stream(stream)))
    return G, h


def fst_cholesky(G, stream=None, shift: float = 0.0) -> int:
    """In-place FP64 Cholesky of G + shift diag(G) (device (R, R) tensor); raises
    FstError(FST_E_NOT_SPD)."""
    R = G.shape[0]
    ws = _workspace(int(_fn["fst_cholesky_workspace_bytes"](R)), G.device)
    info = C.c_int64(0)
    st = _fn["fst_cholesky"](R, _dev_ptr(G), float(shift), C.byref(info), _dev_ptr(ws), ws.numel(),
                             _stream(stream))
    if st != FST_OK:
        raise FstError(st, fst_last_error() + f" (info={info.value})")
    return info.value


FST_CHOLESKY_NOALLOC_MAX_R = 65536


def fst_cholesky_noalloc(G, stream=None, shift: float = 0.0) -> int:
    """fst_cholesky with the library's own device scratch (no workspace, no allocation);
    R <= FST_CHOLESKY_NOALLOC_MAX_R.  Calls that overlap on one GPU race."""
    R = G.shape[0]
    info = C.c_int64(0)
    st = _fn["fst_cholesky_noalloc"](R, _dev_ptr(G), float(shift), C.byref(info), _stream(stream))
    if st != FST_OK:
        raise FstError(st, fst_last_error() + f" (info={info.value})")
    return info.value


def fst_cholesky_solve(L, b, x=None, stream=None):
    torch = _torch()
    if x is None:
        x = torch.empty_like(b)
    _check(_fn["fst_cholesky_solve"](L.shape[0], _dev_ptr(L), _dev_ptr(b), _dev_ptr(x), _stream(stream)))
    return x


def fst_residual(m: Model, x, y, z, v, idx, alpha, r=None, stream=None):
    """FP64 A^T (v_S - A alpha) at rows idx, rows regenerated in FP64 from the points."""
    torch = _torch()
    mrows = idx.numel()
    if r is None:
        r = torch.empty(m.R, dtype=torch.float64, device=x.device)
    ws = _workspace(int(_fn["fst_residual_workspace_bytes"](m.handle, mrows)), x.device)
    _check(_fn["fst_residual"](m.handle, _dtype_code(x), x.numel(), _dev_ptr(x), _dev_ptr(y), _dev_ptr(z),
                               _dev_ptr(v), _dev_ptr(idx), mrows, _dev_ptr(alpha), _dev_ptr(r),
                               _dev_ptr(ws), ws.numel(), _stream(stream)))
    return r


def fst_refine_step(m: Model, x, y, z, v, idx, L, alpha, r_out=None, ws=None, stream=None):
    """One FP64-residual refinement step of the core (alpha updated in place)."""
    mrows = idx.numel()
    if ws is None:
        ws = _workspace(int(_fn["fst_refine_workspace_bytes"](m.handle, mrows)), x.device)
    _check(_fn["fst_refine_step"](m.handle, _dtype_code(x), x.numel(), _dev_ptr(x), _dev_ptr(y), _dev_ptr(z),
                                  _dev_ptr(v), _dev_ptr(idx), mrows, _dev_ptr(L), _dev_ptr(alpha),
                                  _dev_ptr(r_out), _dev_ptr(ws), ws.numel(), _stream(stream)))
    return alpha


def fst_refine_workspace_bytes(m: Model, mrows: int) -> int:
    return int(_fn["fst_refine_workspace_bytes"](m.handle, int(mrows)))


# ------------------------------------------------------------------------------ host steps
def fst_sample_indices(seed: int, stream: int, n: int, m: int) -> np.ndarray:
    out = np.empty(int(m), dtype=np.int64)
    _check(_fn["fst_sample_indices"](int(seed), int(stream), int(n), int(m), out.ctypes.data_as(C.c_void_p)))
    return out


def fst_idw_grid(xi, v, grid, k=8, power=2.0, n_threads=0) -> np.ndarray:
    xi_a, xi_p = _host(xi, np.float64)
    v_a, v_p = _host(v, np.float64)
    g_a, g_p = _host(grid, np.int32)
    out = np.empty(tuple(int(g) for g in grid), dtype=np.float64)
    _check(_fn["fst_idw_grid"](xi_p, v_p, v_a.size, g_p, int(k), float(power), int(n_threads),
                               out.ctypes.data_as(C.c_void_p)))
    return out


def fst_sthosvd(T, rank, n_threads=0):
    """Returns (core, [W1, W2, W3], [sigma1, sigma2, sigma3])."""
    T_a, T_p = _host(T, np.float64)
    dims = np.asarray(T_a.shape, dtype=np.int32)
    r_a, r_p = _host(rank, np.int32)
    core = np.empty(tuple(int(r) for r in rank), dtype=np.float64)
    W = [np.empty((int(dims[k]), int(rank[k])), dtype=np.float64) for k in range(3)]
    S = [np.empty(int(dims[k]), dtype=np.float64) for k in range(3)]
    Wp = (C.c_void_p * 3)(*[w.ctypes.data_as(C.c_void_p) for w in W])
    Sp = (C.c_void_p * 3)(*[s.ctypes.data_as(C.c_void_p) for s in S])
    _check(_fn["fst_sthosvd"](T_p, dims.ctypes.data_as(C.c_void_p), r_p, int(n_threads),
                              core.ctypes.data_as(C.c_void_p), Wp, Sp))
    return core, W, S


def fst_sthosvd_eps(T, eps: float, max_rank, n_threads=0):
    """ST-HOSVD with ranks from the precision eps (capped at max_rank): returns
    (ranks, core, [W1, W2, W3], [sigma1, sigma2, sigma3])."""
    T_a, T_p = _host(T, np.float64)
    dims = np.asarray(T_a.shape, dtype=np.int32)
    mr = np.asarray(max_rank, dtype=np.int32)
    core = np.empty(int(np.prod(mr)), dtype=np.float64)
    W = [np.empty(int(dims[k]) * int(mr[k]), dtype=np.float64) for k in range(3)]
    S = [np.empty(int(dims[k]), dtype=np.float64) for k in range(3)]
    ranks = np.zeros(3, dtype=np.int32)
    Wp = (C.c_void_p * 3)(*[w.ctypes.data_as(C.c_void_p) for w in W])
    Sp = (C.c_void_p * 3)(*[s.ctypes.data_as(C.c_void_p) for s in S])
    _check(_fn["fst_sthosvd_eps"](T_p, dims.ctypes.data_as(C.c_void_p), float(eps), mr.ctypes.data_as(C.c_void_p),
                                  int(n_threads), ranks.ctypes.data_as(C.c_void_p),
                                  core.ctypes.data_as(C.c_void_p), Wp, Sp))
    r = tuple(int(v) for v in ranks)
    core = core[:r[0] * r[1] * r[2]].reshape(r)
    W = [W[k][:int(dims[k]) * r[k]].reshape(int(dims[k]), r[k]) for k in range(3)]
    return r, core, W, S


def fst_sparse_fit_choice(W, p: int, s: int, q: int, solver: int = FST_SOLVER_OMP) -> np.ndarray:
    W_a, W_p = _host(W, np.float64)
    I, r = W_a.shape
    out = np.empty((int(p) + 1 + _detail_count(int(s), int(q)), r), dtype=np.float64)
    _check(_fn["fst_sparse_fit_choice"](W_p, int(I), int(r), int(p), int(s), int(q), int(solver),
                                        out.ctypes.data_as(C.c_void_p)))
    return out


def fst_sparse_fit(W, p: int, solver: int = FST_SOLVER_OMP) -> np.ndarray:
    W_a, W_p = _host(W, np.float64)
    I, r = W_a.shape
    out = np.empty((int(p) + 1, r), dtype=np.float64)
    name = "fst_sparse_fit_lars" if solver == FST_SOLVER_LARS else "fst_sparse_fit"
    _check(_fn[name](W_p, int(I), int(r), int(p), out.ctypes.data_as(C.c_void_p)))
    return out


# ------------------------------------------------------------------------------ corrector
MLP_PARAMS = 4481


class Corrector:
    """Owns an fst_corrector handle."""

    def __init__(self, handle):
        self._h = handle

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _fn is not None:
            _fn["fst_corrector_free"](h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def params(self):
        p = np.empty(MLP_PARAMS, dtype=np.float32)
        sc = C.c_float()
        _check(_fn["fst_corrector_params"](self._h, p.ctypes.data_as(C.c_void_p), C.byref(sc)))
        return p, sc.value

    def losses(self):
        cnt = C.c_int32(0)
        _check(_fn["fst_corrector_losses"](self._h, None, C.byref(cnt)))
        out = np.empty(max(cnt.value, 1), dtype=np.float32)
        _check(_fn["fst_corrector_losses"](self._h, out.ctypes.data_as(C.c_void_p), C.byref(cnt)))
        return out[: cnt.value]

    def stored_bytes(self) -> int:
        return int(_fn["fst_corrector_stored_bytes"](self._h))


def make_train_params(steps=2000, batch=8192, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=1,
                      init_params=None):
    tp = fst_train_params()
    _fn["fst_train_params_default"](C.byref(tp))
    tp.steps, tp.batch, tp.lr, tp.beta1, tp.beta2, tp.eps, tp.seed = int(steps), int(batch), float(lr), \
        float(beta1), float(beta2), float(eps), int(seed)
    if init_params is not None:
        arr = np.ascontiguousarray(init_params, dtype=np.float32)
        if arr.size != MLP_PARAMS:
            raise ValueError("need 4481 initial parameters")
        tp._init_keepalive = arr
        tp.init_params = arr.ctypes.data_as(C.c_void_p)
    return tp


def fst_corrector_train(m: Model, x, y, z, v, tp=None, stream=None) -> Corrector:
    if tp is None:
        tp = make_train_params()
    n = x.numel()
    nb = int(_fn["fst_corrector_workspace_bytes"](C.byref(tp), n))
    if nb == 0:
        raise FstError(FST_E_INVAL, fst_last_error())
    ws = _workspace(nb, x.device)
    h = C.c_void_p()
    _check(_fn["fst_corrector_train"](m.handle, _dtype_code(x), n, _dev_ptr(x), _dev_ptr(y), _dev_ptr(z),
                                      _dev_ptr(v), C.byref(tp), _dev_ptr(ws), ws.numel(), _stream(stream),
                                      C.byref(h)))
    return Corrector(h)


def fst_corrector_from_params(lo, hi, params, out_scale=1.0) -> Corrector:
    lo_a, lo_p = _host(lo, np.float64)
    hi_a, hi_p = _host(hi, np.float64)
    p_a, p_p = _host(params, np.float32)
    if p_a.size != MLP_PARAMS:
        raise ValueError("need 4481 parameters")
    h = C.c_void_p()
    _check(_fn["fst_corrector_from_params"](lo_p, hi_p, p_p, float(out_scale), C.byref(h)))
    return Corrector(h)


def fst_corrector_apply(c: Corrector, x, y, z, out, stream=None):
    _check(_fn["fst_corrector_apply"](c.handle, _dtype_code(x), x.numel(), _dev_ptr(x), _dev_ptr(y), _dev_ptr(z),
                                      _dev_ptr(out), _stream(stream)))
    return out


def fst_eval_corrected(m: Model, c, x, y, z, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty_like(x)
    _check(_fn["fst_eval_corrected"](m.handle, None if c is None else c.handle, _dtype_code(x), x.numel(),
                                     _dev_ptr(x), _dev_ptr(y), _dev_ptr(z), _dev_ptr(out), _stream(stream)))
    return out


def fst_mlp_grad(c: Corrector, x, y, z, target, idx, stream=None, fp32=False):
    """Gradients (4481) and the batch's sum of squared errors, as a device float tensor
    (fp32: the reference mode with the 64 x 64 layer in FP32, fst_mlp_grad_fp32)."""
    torch = _torch()
    batch = idx.numel()
    ws = _workspace(int(_fn["fst_mlp_grad_workspace_bytes"](batch)), x.device)
    g = torch.empty(MLP_PARAMS + 1, dtype=torch.float32, device=x.device)
    _check(_fn["fst_mlp_grad_fp32" if fp32 else "fst_mlp_grad"](c.handle, _dtype_code(x), x.numel(), _dev_ptr(x), _dev_ptr(y), _dev_ptr(z),
                               _dev_ptr(target), _dev_ptr(idx), batch, _dev_ptr(g), _dev_ptr(ws), ws.numel(),
                               _stream(stream)))
    return g
