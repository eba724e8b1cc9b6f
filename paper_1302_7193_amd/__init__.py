"""Python binding of libpcg (include/pcg.h): argument marshalling only.

Every entry point of the C ABI is exposed under the same name; device
vectors are passed as torch tensors (their data pointers) and streams as
torch streams (default: the current stream).  Torch supplies device memory
and streams only -- every step of the solver runs in the HIP kernels of
libpcg.so.  Importing this package fails loudly when libpcg.so has not been
built; there is no fallback path.

The binding checks tensor sizes, dtypes and devices before a pointer crosses
the ABI, because the library itself only sees raw pointers.
"""
from __future__ import annotations

import ctypes
import os
import sys

import torch  # loads the HIP runtime libpcg.so links against

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcg.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libpcg.so is not built (%s); run `python -c 'import __graft_entry__ as g; g.build()'`"
        % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------- constants --
PCG_OK, PCG_E_INVALID, PCG_E_NOMEM, PCG_E_DEVICE = 0, -1, -2, -3
PCG_E_NOCONV, PCG_E_BREAKDOWN, PCG_E_AGAIN, PCG_E_CANCELLED = -4, -5, -6, -7
PCG_BC_DIRICHLET, PCG_BC_PERIODIC = 0, 1
PCG_F64, PCG_F32 = 0, 1
PCG_PREC_FP64, PCG_PREC_MIXED = 0, 1
PCG_PRECOND_LINE, PCG_PRECOND_MG, PCG_PRECOND_RBGS, PCG_PRECOND_AUTO = 0, 1, 2, 3
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_NOCONV",
                -5: "E_BREAKDOWN", -6: "E_AGAIN", -7: "E_CANCELLED"}


class pcg_problem_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("height", ctypes.c_double),
                ("grading", ctypes.c_double), ("k_h", ctypes.c_double), ("k_v", ctypes.c_double),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32)]


class pcg_solve_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("inner_rtol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("fused", ctypes.c_int32), ("graph_chunk", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("true_residual", ctypes.c_int32),
                ("x0_zero", ctypes.c_int32), ("preconditioner", ctypes.c_int32),
                ("mg_levels", ctypes.c_int32)]


class pcg_tuning(ctypes.Structure):
    _fields_ = [("lanes_per_column", ctypes.c_int32), ("block_cap", ctypes.c_int32),
                ("reduction", ctypes.c_int32), ("lanes_per_column_prec", ctypes.c_int32),
                ("block_cap_prec", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class pcg_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("batched", ctypes.c_int32)]


class pcg_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("cancelled", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("queued", ctypes.c_int32), ("active", ctypes.c_int32),
                ("bytes_in_use", ctypes.c_size_t), ("peak_bytes_in_use", ctypes.c_size_t),
                ("peak_active", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class pcg_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("outer_iterations", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("rel_res_recursive", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("r0_norm", ctypes.c_double), ("elapsed_ms", ctypes.c_double),
                ("ms_apply_kernel", ctypes.c_double), ("ms_precond_kernel", ctypes.c_double),
                ("n_apply_kernel", ctypes.c_int32), ("n_precond_kernel", ctypes.c_int32),
                ("preconditioner", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_S = ctypes.c_int
_sig = {
    "pcg_default_opts": (None, [ctypes.POINTER(pcg_solve_opts)]),
    "pcg_desc_from_ratio": (_S, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_int32,
                                 ctypes.POINTER(pcg_problem_desc)]),
    "pcg_problem_create": (_S, [ctypes.POINTER(pcg_problem_desc), ctypes.POINTER(_P)]),
    "pcg_problem_create_stretched": (_S, [ctypes.POINTER(pcg_problem_desc),
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_P)]),
    "pcg_problem_destroy": (None, [_P]),
    "pcg_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(pcg_solve_opts), ctypes.c_int32]),
    "pcg_apply": (_S, [_P, ctypes.c_int32, _P, _P, _P]),
    "pcg_precond": (_S, [_P, ctypes.c_int32, _P, _P, _P]),
    "pcg_mg_levels": (ctypes.c_int32, [_P]),
    "pcg_rbgs_precond": (_S, [_P, ctypes.c_int32, _P, _P, _P]),
    "pcg_mg_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32, ctypes.c_int32]),
    "pcg_mg_precond": (_S, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, _P, ctypes.c_size_t, _P]),
    "pcg_solve": (_S, [_P, _P, _P, _P, ctypes.c_size_t, ctypes.POINTER(pcg_solve_opts),
                       ctypes.POINTER(pcg_result), _P]),
    "pcg_solve_noalloc": (_S, [_P, _P, _P, ctypes.POINTER(pcg_solve_opts),
                               ctypes.POINTER(pcg_result), _P]),
    "pcg_solve_batched": (_S, [_P, ctypes.c_int32, _P, _P, _P, ctypes.c_size_t,
                               ctypes.POINTER(pcg_solve_opts), ctypes.POINTER(pcg_result), _P]),
    "pcg_csr_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32]),
    "pcg_csr_build": (_S, [_P, ctypes.c_int32, _P, ctypes.c_size_t, _P]),
    "pcg_csr_apply": (_S, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "pcg_last_error": (ctypes.c_size_t, [ctypes.c_char_p, ctypes.c_size_t]),
    "pcg_stream_probe": (_S, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                              ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, _P]),
    "pcg_get_tuning": (_S, [_P, ctypes.c_int32, ctypes.POINTER(pcg_tuning)]),
    "pcg_set_tuning": (_S, [_P, ctypes.c_int32, ctypes.POINTER(pcg_tuning)]),
    "pcg_autotune": (_S, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(pcg_tuning)]),
    "pcg_tuning_cache_load": (_S, [ctypes.c_char_p]),
    "pcg_tuning_cache_save": (_S, [ctypes.c_char_p]),
    "pcg_request_bytes": (ctypes.c_size_t, [ctypes.POINTER(pcg_problem_desc),
                                            ctypes.POINTER(pcg_solve_opts)]),
    "pcg_server_create": (_S, [ctypes.POINTER(pcg_server_opts), _P, ctypes.c_size_t,
                               ctypes.POINTER(_P)]),
    "pcg_submit": (_S, [_P, ctypes.POINTER(pcg_problem_desc), ctypes.POINTER(pcg_solve_opts),
                        _P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "pcg_submit_device": (_S, [_P, ctypes.POINTER(pcg_problem_desc),
                               ctypes.POINTER(pcg_solve_opts), _P, _P, _P,
                               ctypes.POINTER(ctypes.c_uint64)]),
    "pcg_poll": (_S, [_P, ctypes.c_uint64, ctypes.POINTER(pcg_result)]),
    "pcg_wait": (_S, [_P, ctypes.c_uint64, ctypes.POINTER(pcg_result)]),
    "pcg_cancel": (_S, [_P, ctypes.c_uint64]),
    "pcg_server_query": (_S, [_P, ctypes.POINTER(pcg_server_stats)]),
    "pcg_server_destroy": (None, [_P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class PCGError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s: %s" % (where, STATUS_NAMES.get(status, status), pcg_last_error()))


def _check(status: int, where: str) -> int:
    if status not in (PCG_OK, PCG_E_NOCONV, PCG_E_BREAKDOWN, PCG_E_AGAIN):
        raise PCGError(status, where)
    return status


_TORCH_DTYPE = {PCG_F64: torch.float64, PCG_F32: torch.float32}


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def _vec(t, n: int, dtype, what: str) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % what)
    if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype or t.numel() < n:
        raise ValueError("%s must be a contiguous %s CUDA tensor with >= %d elements (got %s %s %s)"
                         % (what, dtype, n, t.dtype, tuple(t.shape), t.device))
    return t.data_ptr()


def _buf(t, nbytes: int, what: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous CUDA tensor" % what)
    if t.numel() * t.element_size() < nbytes:
        raise ValueError("%s holds %d bytes, %d needed" % (what, t.numel() * t.element_size(), nbytes))
    return t.data_ptr()


# ----------------------------------------------------------- entry points --

def pcg_last_error() -> str:
    n = _lib.pcg_last_error(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    _lib.pcg_last_error(buf, n + 1)
    return buf.value.decode(errors="replace")


def pcg_default_opts(**overrides) -> pcg_solve_opts:
    o = pcg_solve_opts()
    _lib.pcg_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def pcg_desc_from_ratio(nx, ny, nz, grading, gamma2, bc=PCG_BC_DIRICHLET) -> pcg_problem_desc:
    d = pcg_problem_desc()
    _check(_lib.pcg_desc_from_ratio(nx, ny, nz, grading, gamma2, bc, ctypes.byref(d)),
           "pcg_desc_from_ratio")
    return d


class Problem:
    """Owning handle of a pcg_problem (destroyed with the object).  With
    ``x_widths`` / ``y_widths`` (n_x and n_y cell widths) the horizontal grid
    is stretched (pcg_problem_create_stretched)."""

    def __init__(self, desc: pcg_problem_desc, x_widths=None, y_widths=None):
        self.desc = desc
        self.n = desc.nx * desc.ny * desc.nz
        h = _P()
        if x_widths is None and y_widths is None:
            _check(_lib.pcg_problem_create(ctypes.byref(desc), ctypes.byref(h)),
                   "pcg_problem_create")
        else:
            import numpy as np
            xw = np.ascontiguousarray(np.full(desc.nx, desc.dx) if x_widths is None else x_widths,
                                      dtype=np.float64)
            yw = np.ascontiguousarray(np.full(desc.ny, desc.dy) if y_widths is None else y_widths,
                                      dtype=np.float64)
            if xw.shape != (desc.nx,) or yw.shape != (desc.ny,):
                raise ValueError("x_widths / y_widths must hold n_x / n_y values")
            dp = ctypes.POINTER(ctypes.c_double)
            _check(_lib.pcg_problem_create_stretched(ctypes.byref(desc), xw.ctypes.data_as(dp),
                                                     yw.ctypes.data_as(dp), ctypes.byref(h)),
                   "pcg_problem_create_stretched")
        self.handle = h

    def __del__(self, _sys=sys):
        # at interpreter exit the module's globals may already be gone and
        # the process releases the device memory anyway
        h = getattr(self, "handle", None)
        if h and not _sys.is_finalizing():
            _lib.pcg_problem_destroy(h)
            self.handle = None


def pcg_problem_create(desc: pcg_problem_desc) -> Problem:
    return Problem(desc)


def pcg_problem_create_stretched(desc: pcg_problem_desc, x_widths, y_widths) -> Problem:
    return Problem(desc, x_widths, y_widths)


def pcg_problem_destroy(p: Problem) -> None:
    if p.handle:
        _lib.pcg_problem_destroy(p.handle)
        p.handle = None


def pcg_workspace_bytes(p: Problem, opts: pcg_solve_opts | None = None, nrhs: int = 1) -> int:
    return _lib.pcg_workspace_bytes(p.handle, ctypes.byref(opts) if opts else None, nrhs)


def workspace(p: Problem, opts: pcg_solve_opts | None = None, nrhs: int = 1,
              device="cuda") -> torch.Tensor:
    """Allocate a workspace tensor of pcg_workspace_bytes() bytes."""
    return torch.empty(pcg_workspace_bytes(p, opts, nrhs), dtype=torch.uint8, device=device)


def pcg_apply(p: Problem, dtype: int, x, y, stream=None) -> int:
    td = _TORCH_DTYPE[dtype]
    return _check(_lib.pcg_apply(p.handle, dtype, _vec(x, p.n, td, "x"), _vec(y, p.n, td, "y"),
                                 _stream(stream)), "pcg_apply")


def pcg_precond(p: Problem, dtype: int, r, z, stream=None) -> int:
    td = _TORCH_DTYPE[dtype]
    return _check(_lib.pcg_precond(p.handle, dtype, _vec(r, p.n, td, "r"), _vec(z, p.n, td, "z"),
                                   _stream(stream)), "pcg_precond")


def pcg_rbgs_precond(p: Problem, dtype: int, r, z, stream=None) -> int:
    td = _TORCH_DTYPE[dtype]
    return _check(_lib.pcg_rbgs_precond(p.handle, dtype, _vec(r, p.n, td, "r"),
                                        _vec(z, p.n, td, "z"), _stream(stream)),
                  "pcg_rbgs_precond")


def pcg_mg_levels(p: Problem) -> int:
    return _lib.pcg_mg_levels(p.handle)


def pcg_mg_bytes(p: Problem, dtype: int, mg_levels: int = 0) -> int:
    return _lib.pcg_mg_bytes(p.handle, dtype, mg_levels)


def pcg_mg_precond(p: Problem, dtype: int, r, z, ws, mg_levels: int = 0, stream=None) -> int:
    td = _TORCH_DTYPE[dtype]
    need = pcg_mg_bytes(p, dtype, mg_levels)
    return _check(_lib.pcg_mg_precond(p.handle, dtype, _vec(r, p.n, td, "r"), _vec(z, p.n, td, "z"),
                                      mg_levels, _buf(ws, need, "workspace"),
                                      ws.numel() * ws.element_size(), _stream(stream)),
                  "pcg_mg_precond")


def _check_ws(status: int, where: str) -> int:
    """_check, with a workspace the library found too small (it checks the
    size itself, so the binding does not query it per call) as ValueError."""
    if status == PCG_E_NOMEM and "workspace" in pcg_last_error():
        raise ValueError("%s: %s" % (where, pcg_last_error()))
    return _check(status, where)


def pcg_solve(p: Problem, b, x, ws, opts: pcg_solve_opts | None = None, stream=None):
    """Returns (status, result dict)."""
    opts = opts or pcg_default_opts()
    res = pcg_result()
    st = _check_ws(_lib.pcg_solve(p.handle, _vec(b, p.n, torch.float64, "b"),
                                  _vec(x, p.n, torch.float64, "x"), _buf(ws, 0, "workspace"),
                                  ws.numel() * ws.element_size(), ctypes.byref(opts),
                                  ctypes.byref(res), _stream(stream)), "pcg_solve")
    return st, res.as_dict()


def pcg_solve_noalloc(p: Problem, b, x, opts: pcg_solve_opts | None = None, stream=None):
    """pcg_solve with the library's fixed device scratch as its workspace
    (no allocation in the call).  Returns (status, result dict)."""
    opts = opts or pcg_default_opts()
    res = pcg_result()
    st = _check(_lib.pcg_solve_noalloc(p.handle, _vec(b, p.n, torch.float64, "b"),
                                       _vec(x, p.n, torch.float64, "x"), ctypes.byref(opts),
                                       ctypes.byref(res), _stream(stream)), "pcg_solve_noalloc")
    return st, res.as_dict()


def pcg_solve_batched(p: Problem, nrhs: int, b, x, ws, opts: pcg_solve_opts | None = None,
                      stream=None):
    """Returns (status, [result dict per right-hand side])."""
    opts = opts or pcg_default_opts()
    res = (pcg_result * nrhs)()
    st = _check_ws(_lib.pcg_solve_batched(p.handle, nrhs,
                                          _vec(b, nrhs * p.n, torch.float64, "b"),
                                          _vec(x, nrhs * p.n, torch.float64, "x"),
                                          _buf(ws, 0, "workspace"), ws.numel() * ws.element_size(),
                                          ctypes.byref(opts), res, _stream(stream)),
                   "pcg_solve_batched")
    return st, [r.as_dict() for r in res]


def pcg_csr_bytes(p: Problem, dtype: int) -> int:
    return _lib.pcg_csr_bytes(p.handle, dtype)


def pcg_csr_build(p: Problem, dtype: int, buf, stream=None) -> int:
    need = pcg_csr_bytes(p, dtype)
    return _check(_lib.pcg_csr_build(p.handle, dtype, _buf(buf, need, "csr buffer"),
                                     buf.numel() * buf.element_size(), _stream(stream)),
                  "pcg_csr_build")


def pcg_stream_probe(reads, writes, nontemporal: int = 1, blocks: int = 0, stream=None) -> int:
    """HBM probe: stream the CUDA tensors `reads` in and `writes` out (all of
    one byte size); written tensor k receives sum_i reads[i] * 2^-(i+k)
    (as FP64 pairs).  nontemporal: 0 none, 1 every access, 2 all but the
    first vector's reads, 3 all but the last vector's writes (a bool is 0 or
    1).  Asynchronous on `stream`."""
    vecs = list(reads) + list(writes)
    if not vecs:
        raise ValueError("no vectors")
    nbytes = vecs[0].numel() * vecs[0].element_size()
    for t in vecs:
        if _buf(t, nbytes, "probe vector") and t.numel() * t.element_size() != nbytes:
            raise ValueError("probe vectors must have one byte size")
    arr = (ctypes.c_void_p * len(vecs))(*[t.data_ptr() for t in vecs])
    return _check(_lib.pcg_stream_probe(len(reads), len(writes), arr, nbytes, int(nontemporal),
                                        blocks, _stream(stream)), "pcg_stream_probe")


def pcg_csr_apply(p: Problem, dtype: int, buf, x, y, stream=None) -> int:
    td = _TORCH_DTYPE[dtype]
    need = pcg_csr_bytes(p, dtype)
    return _check(_lib.pcg_csr_apply(p.handle, dtype, _buf(buf, need, "csr buffer"),
                                     _vec(x, p.n, td, "x"), _vec(y, p.n, td, "y"),
                                     _stream(stream)), "pcg_csr_apply")


def pcg_get_tuning(p: Problem, dtype: int) -> pcg_tuning:
    t = pcg_tuning()
    _check(_lib.pcg_get_tuning(p.handle, dtype, ctypes.byref(t)), "pcg_get_tuning")
    return t


def pcg_set_tuning(p: Problem, dtype: int, t: pcg_tuning | None = None, **fields) -> None:
    """Set launch parameters; fields not given keep their current values.  A
    lanes_per_column or block_cap given without its _prec counterpart sets
    both (one launch shape for every kernel)."""
    t = t or pcg_get_tuning(p, dtype)
    for k in ("lanes_per_column", "block_cap"):
        if k in fields and k + "_prec" not in fields:
            fields[k + "_prec"] = fields[k]
    for k, v in fields.items():
        setattr(t, k, v)
    _check(_lib.pcg_set_tuning(p.handle, dtype, ctypes.byref(t)), "pcg_set_tuning")


def pcg_autotune(p: Problem, dtype: int, nrhs: int = 1, stream=None) -> pcg_tuning:
    t = pcg_tuning()
    _check(_lib.pcg_autotune(p.handle, dtype, nrhs, _stream(stream), ctypes.byref(t)),
           "pcg_autotune")
    return t


def pcg_tuning_cache_load(path: str | None = None) -> None:
    _check(_lib.pcg_tuning_cache_load(path.encode() if path else None), "pcg_tuning_cache_load")


def pcg_tuning_cache_save(path: str | None = None) -> None:
    _check(_lib.pcg_tuning_cache_save(path.encode() if path else None), "pcg_tuning_cache_save")


def solve(desc: pcg_problem_desc, b: torch.Tensor, x0: torch.Tensor | None = None, **opts):
    """Convenience: create the problem, allocate the workspace, solve once.
    Returns (x, status, result dict)."""
    p = Problem(desc)
    o = pcg_default_opts(**opts)
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    ws = workspace(p, o)
    st, res = pcg_solve(p, b, x, ws, o)
    torch.cuda.synchronize()
    return x, st, res


# ---------------------------------------------------------------- serving --

def pcg_request_bytes(desc: pcg_problem_desc, opts: pcg_solve_opts | None = None) -> int:
    return _lib.pcg_request_bytes(ctypes.byref(desc), ctypes.byref(opts) if opts else None)


def _host_vec(a, n: int, what: str) -> int:
    """Host FP64 array (numpy or CPU torch tensor) of at least n values."""
    if isinstance(a, torch.Tensor):
        if a.is_cuda or a.dtype != torch.float64 or not a.is_contiguous() or a.numel() < n:
            raise ValueError("%s must be a contiguous CPU float64 tensor with >= %d values" % (what, n))
        return a.data_ptr()
    import numpy as np
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous \
            or a.size < n:
        raise ValueError("%s must be a contiguous float64 array with >= %d values" % (what, n))
    return a.ctypes.data


class Server:
    """Owning handle of a pcg_server.  Keeps every submitted request's host
    arrays alive until the request is collected."""

    def __init__(self, arena: torch.Tensor, hbm_budget_bytes: int, max_active: int = 4,
                 batched: bool = False):
        self.arena = arena
        o = pcg_server_opts(hbm_budget_bytes=hbm_budget_bytes, max_active=max_active,
                            batched=int(bool(batched)))
        h = _P()
        nbytes = arena.numel() * arena.element_size()
        _check(_lib.pcg_server_create(ctypes.byref(o), _buf(arena, nbytes, "arena"), nbytes,
                                      ctypes.byref(h)), "pcg_server_create")
        self.handle = h
        self._keep = {}

    def close(self):
        if getattr(self, "handle", None):
            _lib.pcg_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        self.close()


def pcg_server_create(arena: torch.Tensor, hbm_budget_bytes: int, max_active: int = 4,
                      batched: bool = False) -> Server:
    return Server(arena, hbm_budget_bytes, max_active, batched)


def pcg_server_destroy(s: Server) -> None:
    s.close()


def pcg_submit(s: Server, desc: pcg_problem_desc, b_host, x_host,
               opts: pcg_solve_opts | None = None) -> int:
    n = desc.nx * desc.ny * desc.nz
    t = ctypes.c_uint64()
    _check(_lib.pcg_submit(s.handle, ctypes.byref(desc), ctypes.byref(opts) if opts else None,
                           _host_vec(b_host, n, "b_host"), _host_vec(x_host, n, "x_host"),
                           ctypes.byref(t)), "pcg_submit")
    s._keep[t.value] = (b_host, x_host)
    return t.value


def pcg_submit_device(s: Server, desc: pcg_problem_desc, b: torch.Tensor, x: torch.Tensor,
                      opts: pcg_solve_opts | None = None, stream=None) -> int:
    """Device-resident request; ordered after the work queued so far on
    `stream` (default: the current torch stream, which produced b)."""
    n = desc.nx * desc.ny * desc.nz
    t = ctypes.c_uint64()
    _check(_lib.pcg_submit_device(s.handle, ctypes.byref(desc),
                                  ctypes.byref(opts) if opts else None,
                                  _vec(b, n, torch.float64, "b"), _vec(x, n, torch.float64, "x"),
                                  _stream(stream), ctypes.byref(t)), "pcg_submit_device")
    s._keep[t.value] = (b, x)
    return t.value


def pcg_poll(s: Server, ticket: int):
    """Returns (status, result dict or None); status PCG_E_AGAIN while pending."""
    r = pcg_result()
    st = _lib.pcg_poll(s.handle, ticket, ctypes.byref(r))
    if st == PCG_E_AGAIN:
        return st, None
    s._keep.pop(ticket, None)
    if st == PCG_E_CANCELLED:
        return st, None
    _check(st, "pcg_poll")
    return st, r.as_dict()


def pcg_wait(s: Server, ticket: int):
    r = pcg_result()
    st = _lib.pcg_wait(s.handle, ticket, ctypes.byref(r))
    s._keep.pop(ticket, None)
    if st == PCG_E_CANCELLED:
        return st, None
    _check(st, "pcg_wait")
    return st, r.as_dict()


def pcg_cancel(s: Server, ticket: int) -> int:
    st = _lib.pcg_cancel(s.handle, ticket)
    if st == PCG_OK:
        s._keep.pop(ticket, None)
    return st


def pcg_server_query(s: Server) -> dict:
    st = pcg_server_stats()
    _check(_lib.pcg_server_query(s.handle, ctypes.byref(st)), "pcg_server_query")
    return st.as_dict()
