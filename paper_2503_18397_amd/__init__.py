"""Python binding of libvf.so, the gfx950 library for epsilon-cost sharded
static functions (VFunc) and static filters (VFilter), after S. Vigna,
"epsilon-Cost Sharding: Scaling Hypergraph-Based Static Functions and
Filters to Trillions of Keys" (arXiv 2503.18397).

The functions below carry the names of the C ABI in ``include/vf.h`` and only
marshal arguments: torch tensors provide device memory and the HIP stream,
every step of construction and query runs in the library's kernels.  There is
no CPU fallback: importing this module fails if the library is not built.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# VF_LIBRARY selects another build of the library (the stage-clock build
# for profiling); the default is the in-tree libvf.so.
LIB_PATH = os.environ.get("VF_LIBRARY") or os.path.join(_HERE, "libvf.so")

VF_OK, VF_EINVAL, VF_ENOSPC, VF_EFAIL, VF_EHIP, VF_ECAPACITY, VF_ENOMEM = (
    0, -1, -2, -3, -4, -5, -6)
_ERR = {VF_EINVAL: "VF_EINVAL", VF_ENOSPC: "VF_ENOSPC", VF_EFAIL: "VF_EFAIL",
        VF_EHIP: "VF_EHIP", VF_ECAPACITY: "VF_ECAPACITY", VF_ENOMEM: "VF_ENOMEM"}


class VFError(RuntimeError):
    def __init__(self, code: int, where: str):
        detail = ""
        if code == VF_EHIP:
            detail = " (" + (_lib.vf_last_error() or b"").decode(errors="replace") + ")"
        super().__init__(f"{where}: {_ERR.get(code, code)}{detail}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("h", C.c_int32), ("sigma", C.c_int32), ("c_num", C.c_uint32),
                ("c_den", C.c_uint32), ("tmax", C.c_uint32), ("alpha", C.c_double),
                ("mwhc", C.c_int32), ("max_window", C.c_uint32), ("packed", C.c_uint32),
                ("small", C.c_int32), ("ring_cols", C.c_uint32)]


class Sizes(C.Structure):
    _fields_ = [("structure_bytes", C.c_uint64), ("workspace_bytes", C.c_uint64),
                ("h", C.c_int32), ("shard_cap", C.c_uint32)]


class Info(C.Structure):
    _fields_ = [("is_filter", C.c_int32), ("b", C.c_int32), ("h", C.c_int32),
                ("S", C.c_uint32), ("M", C.c_uint32), ("c_num", C.c_uint32),
                ("c_den", C.c_uint32), ("sigma", C.c_int32), ("l", C.c_uint32),
                ("V", C.c_uint64), ("n", C.c_uint64), ("seed", C.c_uint64),
                ("cell_bytes", C.c_uint32), ("failed_shards", C.c_uint32),
                ("n_failures", C.c_uint32), ("space_bits", C.c_uint64),
                ("cells", C.c_void_p), ("local_seeds", C.c_void_p),
                ("ms_count", C.c_float), ("ms_scatter", C.c_float), ("ms_build", C.c_float),
                ("relaunched_shards", C.c_uint32), ("mwhc", C.c_int32), ("packed", C.c_uint32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchItem(C.Structure):
    _fields_ = [("n", C.c_uint64), ("b", C.c_int32), ("c_num", C.c_uint32),
                ("c_den", C.c_uint32), ("sigma", C.c_int32), ("l", C.c_uint32),
                ("V", C.c_uint64), ("cell_bytes", C.c_uint32), ("local_seed", C.c_uint32),
                ("cells", C.c_void_p), ("packed", C.c_uint32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tuning(C.Structure):
    _fields_ = [("tuned", C.c_int32), ("max_keys", C.c_uint32 * 4), ("use_small", C.c_int32 * 4),
                ("ms_small", C.c_float * 4), ("ms_band", C.c_float * 4),
                ("sampled", C.c_uint32 * 4), ("small_groups_per_cu", C.c_uint32)]

    def as_dict(self) -> dict:
        return {f: (list(getattr(self, f)) if hasattr(getattr(self, f), "__len__")
                    else getattr(self, f)) for f, _ in self._fields_}


class Failure(C.Structure):
    _fields_ = [("shard", C.c_uint32), ("attempt", C.c_uint32), ("kind", C.c_uint32),
                ("core_edges", C.c_uint32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2503_18397_amd.build` "
        "(there is no CPU fallback)")

_lib = C.CDLL(LIB_PATH)
_vp, _u64, _i32, _dbl = C.c_void_p, C.c_uint64, C.c_int32, C.c_double
_lib.vf_default_opts.argtypes = [C.POINTER(Opts)]
_lib.vf_default_opts.restype = None
_lib.vf_plan.argtypes = [_u64, _i32, _dbl, _i32, C.POINTER(Opts), C.POINTER(Sizes)]
_lib.vf_build.argtypes = [_vp, _vp, _u64, _i32, _dbl, _u64, C.POINTER(Opts), _vp, _u64, _vp,
                          _u64, _vp, C.POINTER(_vp)]
_lib.vfilter_build.argtypes = [_vp, _u64, _i32, _dbl, _u64, C.POINTER(Opts), _vp, _u64, _vp,
                               _u64, _vp, C.POINTER(_vp)]
_lib.vfilter_build_host.argtypes = [_vp, _u64, _i32, _dbl, _u64, C.POINTER(Opts), _u64, _vp,
                                    _u64, _vp, _u64, _vp, C.POINTER(_vp)]
_lib.vf_query.argtypes = [_vp, _vp, _u64, _vp, _vp]
_lib.vfilter_contains.argtypes = [_vp, _vp, _u64, _vp, _vp]
_lib.vf_query_grouped_bytes.argtypes = [_vp, _u64, C.POINTER(_u64)]
_lib.vf_query_grouped.argtypes = [_vp, _vp, _u64, _vp, _vp, _u64, _vp]
_lib.vfilter_contains_grouped.argtypes = [_vp, _vp, _u64, _vp, _vp, _u64, _vp]
_lib.vfilter_contains_grouped_noalloc.argtypes = [_vp, _vp, _u64, _vp, _vp]
_lib.vf_info.argtypes = [_vp, C.POINTER(Info)]
_lib.vf_failures.argtypes = [_vp, C.POINTER(Failure), C.c_uint32, C.POINTER(C.c_uint32)]
_lib.vf_free.argtypes = [_vp]
_lib.vf_free.restype = None
_lib.vf_batch_plan.argtypes = [_u64, _vp, _vp, C.POINTER(Opts), C.POINTER(Sizes)]
_lib.vf_batch_build.argtypes = [_vp, _vp, _u64, _vp, _vp, _u64, C.POINTER(Opts), _vp, _u64,
                                _vp, _u64, _vp, C.POINTER(_vp)]
_lib.vf_batch_prepare.argtypes = [_u64, _vp, _vp, _u64, C.POINTER(Opts), _vp, _u64, _vp, _u64,
                                  _vp, C.POINTER(_vp)]
_lib.vf_batch_launch.argtypes = [_vp, _vp, _vp, _vp]
_lib.vf_batch_finish.argtypes = [_vp, _vp]
_lib.vf_query_multi.argtypes = [_vp, C.c_uint32, _vp]
_lib.vf_build_prepare.argtypes = [_u64, C.c_uint32, _i32, _dbl, _i32, _u64, C.POINTER(Opts), _vp,
                                  _u64, _vp, _u64, C.POINTER(_vp)]
_lib.vf_build_launch.argtypes = [_vp, _vp, _vp, _vp]
_lib.vf_build_finish.argtypes = [_vp, _vp]
_lib.vf_batch_query.argtypes = [_vp, _vp, _vp, _u64, _vp, _vp]
_lib.vf_batch_item.argtypes = [_vp, _u64, C.POINTER(BatchItem)]
_lib.vf_batch_tuning.argtypes = [C.POINTER(Tuning)]
_lib.vf_stage_clocks.argtypes = [_vp, _u64, _i32]
_lib.vf_stage_clocks.restype = C.c_int
_lib.vf_last_error.argtypes = []
_lib.vf_last_error.restype = C.c_char_p
for _f in ("vf_plan", "vf_build", "vfilter_build", "vf_query", "vfilter_contains", "vf_info",
           "vf_failures", "vf_batch_plan", "vf_batch_build", "vf_batch_query", "vf_batch_item",
           "vfilter_build_host", "vf_query_grouped_bytes", "vf_query_grouped",
           "vfilter_contains_grouped", "vfilter_contains_grouped_noalloc", "vf_batch_tuning",
           "vf_batch_prepare", "vf_batch_launch", "vf_batch_finish", "vf_query_multi",
           "vf_stage_clocks", "vf_build_prepare", "vf_build_launch", "vf_build_finish"):
    getattr(_lib, _f).restype = C.c_int

EXPORTS = ("vf_default_opts", "vf_plan", "vf_build", "vf_query", "vfilter_build",
           "vfilter_contains", "vf_info", "vf_failures", "vf_free", "vf_batch_plan",
           "vf_batch_build", "vf_batch_query", "vf_batch_item", "vfilter_build_host",
           "vf_query_grouped_bytes", "vf_query_grouped", "vfilter_contains_grouped",
           "vfilter_contains_grouped_noalloc", "vf_batch_tuning", "vf_last_error",
           "vf_batch_prepare", "vf_batch_launch", "vf_batch_finish", "vf_query_multi",
           "vf_stage_clocks", "vf_build_prepare", "vf_build_launch", "vf_build_finish")


def _check(rc: int, where: str) -> None:
    if rc != VF_OK:
        raise VFError(rc, where)


def _on(stream):
    """Context in which tensors are allocated on `stream` (a torch stream or
    None for the current one)."""
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _used_on(stream, *tensors) -> None:
    """Marks tensors as used by work enqueued on `stream` (no-op for the
    current stream)."""
    if stream is not None:
        for t in tensors:
            if t is not None and t.is_cuda:
                t.record_stream(stream)


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_ptr(t: torch.Tensor, name: str) -> int:
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")
    return t.data_ptr()


def vf_default_opts(**overrides) -> Opts:
    o = Opts()
    _lib.vf_default_opts(C.byref(o))
    for k, v in overrides.items():
        if v is not None:
            setattr(o, k, v)
    return o


def vf_plan(n: int, b: int, eps: float, is_filter: bool, opts: Opts | None = None) -> Sizes:
    s = Sizes()
    _check(_lib.vf_plan(n, b, eps, int(is_filter), C.byref(opts) if opts else None,
                        C.byref(s)), "vf_plan")
    return s


def vf_build(keys, values, b, eps, seed, opts, workspace, structure, stream=None):
    """Returns (rc, handle); rc is VF_OK or VF_EFAIL (the handle is valid for
    the failure record); other codes raise."""
    h = C.c_void_p()
    rc = _lib.vf_build(_dev_ptr(keys, "keys"), _dev_ptr(values, "values"), keys.numel(), b,
                       eps, seed, C.byref(opts) if opts else None,
                       _dev_ptr(workspace, "workspace"), workspace.numel(),
                       _dev_ptr(structure, "structure"), structure.numel(), _stream(stream),
                       C.byref(h))
    if rc not in (VF_OK, VF_EFAIL):
        raise VFError(rc, "vf_build")
    return rc, h


def vfilter_build(keys, b, eps, seed, opts, workspace, structure, stream=None):
    h = C.c_void_p()
    rc = _lib.vfilter_build(_dev_ptr(keys, "keys"), keys.numel(), b, eps, seed,
                            C.byref(opts) if opts else None, _dev_ptr(workspace, "workspace"),
                            workspace.numel(), _dev_ptr(structure, "structure"),
                            structure.numel(), _stream(stream), C.byref(h))
    if rc not in (VF_OK, VF_EFAIL):
        raise VFError(rc, "vfilter_build")
    return rc, h


def vfilter_build_host(keys, b, eps, seed, opts, workspace, structure, chunk=1 << 28,
                       stream=None):
    """keys: a contiguous int64 CPU tensor (pinned for the full PCIe rate);
    workspace: vf_plan().workspace_bytes + 8 n rounded up to 256 bytes."""
    if keys.is_cuda or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous host tensor")
    h = C.c_void_p()
    rc = _lib.vfilter_build_host(keys.data_ptr(), keys.numel(), b, eps, seed,
                                 C.byref(opts) if opts else None, chunk,
                                 _dev_ptr(workspace, "workspace"), workspace.numel(),
                                 _dev_ptr(structure, "structure"), structure.numel(),
                                 _stream(stream), C.byref(h))
    if rc not in (VF_OK, VF_EFAIL):
        raise VFError(rc, "vfilter_build_host")
    return rc, h


def vf_query(handle, keys, out, stream=None) -> None:
    _check(_lib.vf_query(handle, _dev_ptr(keys, "keys"), keys.numel(), _dev_ptr(out, "out"),
                         _stream(stream)), "vf_query")


def vfilter_contains(handle, keys, out, stream=None) -> None:
    _check(_lib.vfilter_contains(handle, _dev_ptr(keys, "keys"), keys.numel(),
                                 _dev_ptr(out, "out"), _stream(stream)), "vfilter_contains")


class QueryReq(C.Structure):
    _fields_ = [("h", C.c_void_p), ("keys", C.c_void_p), ("n", C.c_uint64), ("out", C.c_void_p)]


VF_QUERY_MULTI_MAX = 16


def vf_query_multi(reqs, stream=None) -> None:
    """reqs: (handle, keys, out) triples; one launch per 16 requests."""
    arr = (QueryReq * max(1, len(reqs)))()
    for i, (h, keys, out) in enumerate(reqs):
        arr[i].h = h.value if isinstance(h, C.c_void_p) else h
        arr[i].keys = _dev_ptr(keys, "keys")
        arr[i].n = keys.numel()
        arr[i].out = _dev_ptr(out, "out")
    _check(_lib.vf_query_multi(arr, len(reqs), _stream(stream)), "vf_query_multi")


def query_many(pairs, stream=None) -> list:
    """Answers [(structure, keys), ...] with combined launches (vf_query_multi);
    returns the answer tensors, typed as Structure.query returns them."""
    outs, reqs = [], []
    with _on(stream):
        for st, keys in pairs:
            dt = torch.uint8 if st.is_filter else _CELL_DTYPE[st.info["cell_bytes"]]
            out = torch.empty(keys.numel(), dtype=dt, device=keys.device)
            outs.append(out)
            reqs.append((st.handle, keys, out))
        vf_query_multi(reqs, stream)
    for (st, keys), out in zip(pairs, outs):
        _used_on(stream, keys, out)
    return outs


def vf_query_grouped_bytes(handle, n: int) -> int:
    b = C.c_uint64(0)
    _check(_lib.vf_query_grouped_bytes(handle, n, C.byref(b)), "vf_query_grouped_bytes")
    return b.value


def vf_query_grouped(handle, keys, out, workspace, stream=None) -> None:
    _check(_lib.vf_query_grouped(handle, _dev_ptr(keys, "keys"), keys.numel(),
                                 _dev_ptr(out, "out"), _dev_ptr(workspace, "workspace"),
                                 workspace.numel() * workspace.element_size(), _stream(stream)),
           "vf_query_grouped")


def vfilter_contains_grouped(handle, keys, out, workspace, stream=None) -> None:
    _check(_lib.vfilter_contains_grouped(handle, _dev_ptr(keys, "keys"), keys.numel(),
                                         _dev_ptr(out, "out"), _dev_ptr(workspace, "workspace"),
                                         workspace.numel() * workspace.element_size(),
                                         _stream(stream)),
           "vfilter_contains_grouped")


def vfilter_contains_grouped_noalloc(handle, keys, out, stream=None) -> None:
    _check(_lib.vfilter_contains_grouped_noalloc(handle, _dev_ptr(keys, "keys"), keys.numel(),
                                                 _dev_ptr(out, "out"), _stream(stream)),
           "vfilter_contains_grouped_noalloc")


def vf_info(handle) -> dict:
    i = Info()
    _check(_lib.vf_info(handle, C.byref(i)), "vf_info")
    return i.as_dict()


def vf_failures(handle) -> list:
    cnt = C.c_uint32(0)
    _check(_lib.vf_failures(handle, None, 0, C.byref(cnt)), "vf_failures")
    buf = (Failure * max(cnt.value, 1))()
    _check(_lib.vf_failures(handle, buf, cnt.value, C.byref(cnt)), "vf_failures")
    return [(f.shard, f.attempt, f.kind, f.core_edges) for f in buf[: cnt.value]]


def vf_free(handle) -> None:
    _lib.vf_free(handle)


def _host_arrays(n, b):
    import numpy as np
    n = np.ascontiguousarray(np.asarray(n, dtype=np.uint64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.int32))
    if n.shape != b.shape or n.ndim != 1:
        raise ValueError("n and b must be 1-d arrays of the same length")
    return n, b


def vf_batch_plan(n, b, opts: Opts | None = None) -> Sizes:
    n, b = _host_arrays(n, b)
    s = Sizes()
    _check(_lib.vf_batch_plan(n.size, n.ctypes.data, b.ctypes.data,
                              C.byref(opts) if opts else None, C.byref(s)), "vf_batch_plan")
    return s


def vf_batch_build(keys, values, n, b, seed, opts, workspace, structure, stream=None):
    """Returns (rc, handle) like vf_build; n and b are host arrays."""
    n, b = _host_arrays(n, b)
    h = C.c_void_p()
    rc = _lib.vf_batch_build(_dev_ptr(keys, "keys"), _dev_ptr(values, "values"), n.size,
                             n.ctypes.data, b.ctypes.data, seed,
                             C.byref(opts) if opts else None, _dev_ptr(workspace, "workspace"),
                             workspace.numel(), _dev_ptr(structure, "structure"),
                             structure.numel(), _stream(stream), C.byref(h))
    if rc not in (VF_OK, VF_EFAIL):
        raise VFError(rc, "vf_batch_build")
    return rc, h


def vf_build_prepare(n: int, b: int, eps: float, is_filter: bool, seed: int, opts, workspace,
                     structure, max_shard: int = 0):
    """Handle of a prepared sharded build (vf_build_prepare)."""
    h = C.c_void_p()
    _check(_lib.vf_build_prepare(n, max_shard, b, eps, int(is_filter), seed,
                                 C.byref(opts) if opts else None,
                                 _dev_ptr(workspace, "workspace"), workspace.numel(),
                                 _dev_ptr(structure, "structure"), structure.numel(),
                                 C.byref(h)), "vf_build_prepare")
    return h


def vf_build_launch(handle, keys, values=None, stream=None) -> None:
    _check(_lib.vf_build_launch(handle, _dev_ptr(keys, "keys"),
                                None if values is None else _dev_ptr(values, "values"),
                                _stream(stream)), "vf_build_launch")


def vf_build_finish(handle, stream=None) -> int:
    """Returns VF_OK or VF_EFAIL; raises on the other codes."""
    rc = _lib.vf_build_finish(handle, _stream(stream))
    if rc not in (VF_OK, VF_EFAIL):
        raise VFError(rc, "vf_build_finish")
    return rc


def vf_batch_prepare(n, b, seed, opts, workspace, structure, stream=None):
    """Returns the handle of a prepared batch (host arrays n and b)."""
    n, b = _host_arrays(n, b)
    h = C.c_void_p()
    _check(_lib.vf_batch_prepare(n.size, n.ctypes.data, b.ctypes.data, seed,
                                 C.byref(opts) if opts else None,
                                 _dev_ptr(workspace, "workspace"), workspace.numel(),
                                 _dev_ptr(structure, "structure"), structure.numel(),
                                 _stream(stream), C.byref(h)), "vf_batch_prepare")
    return h


def vf_batch_launch(handle, keys, values, stream=None) -> None:
    _check(_lib.vf_batch_launch(handle, _dev_ptr(keys, "keys"), _dev_ptr(values, "values"),
                                _stream(stream)), "vf_batch_launch")


def vf_batch_finish(handle, stream=None) -> int:
    """Returns VF_OK or VF_EFAIL; raises on the other codes."""
    rc = _lib.vf_batch_finish(handle, _stream(stream))
    if rc not in (VF_OK, VF_EFAIL):
        raise VFError(rc, "vf_batch_finish")
    return rc


def vf_batch_query(handle, inst, keys, out, stream=None) -> None:
    _check(_lib.vf_batch_query(handle, _dev_ptr(inst, "inst"), _dev_ptr(keys, "keys"),
                               keys.numel(), _dev_ptr(out, "out"), _stream(stream)),
           "vf_batch_query")


def vf_batch_item(handle, i: int) -> dict:
    it = BatchItem()
    _check(_lib.vf_batch_item(handle, i, C.byref(it)), "vf_batch_item")
    return it.as_dict()


VF_STAGE_CLOCK_WORDS = 4096 * 32


def vf_stage_clocks(reset: bool = False):
    """Stage clocks of the build kernel (profiling build only): clears them
    (reset) or returns a (4096, 32) uint64 array of counters."""
    import numpy as np
    if reset:
        _check(_lib.vf_stage_clocks(None, 0, 1), "vf_stage_clocks")
        return None
    out = np.zeros(VF_STAGE_CLOCK_WORDS, np.uint64)
    _check(_lib.vf_stage_clocks(out.ctypes.data, out.size, 0), "vf_stage_clocks")
    return out.reshape(4096, 32)


def vf_last_error() -> str:
    """The calling thread's last VF_EHIP: the failing HIP call and its error."""
    return (_lib.vf_last_error() or b"").decode(errors="replace")


def vf_batch_tuning() -> dict:
    t = Tuning()
    _check(_lib.vf_batch_tuning(C.byref(t)), "vf_batch_tuning")
    return t.as_dict()


_CELL_DTYPE = {1: torch.uint8, 2: torch.int16, 4: torch.int32, 8: torch.int64}


@dataclass
class Structure:
    """A built VFunc or VFilter with the device buffers it lives in.

    ``workspace`` is only needed during the build and may be dropped
    (``release_workspace``); ``structure`` must stay alive with the handle."""
    handle: C.c_void_p
    rc: int
    is_filter: bool
    b: int
    structure: torch.Tensor
    workspace: torch.Tensor | None

    @classmethod
    def build(cls, keys: torch.Tensor, values: torch.Tensor | None = None, *, b: int,
              eps: float = 0.0, seed: int = 0, h: int | None = None, sigma: int | None = None,
              c: tuple | None = None, tmax: int | None = None, mwhc: bool = False,
              max_window: int | None = None, packed: bool = False,
              ring_cols: int | None = None, stream=None):
        is_filter = values is None
        opts = vf_default_opts(h=h, sigma=sigma, tmax=tmax, mwhc=int(mwhc),
                               max_window=max_window, packed=int(packed),
                               ring_cols=ring_cols)
        if c is not None:
            opts.c_num, opts.c_den = c
        sz = vf_plan(keys.numel(), b, eps, is_filter, opts)
        dev = keys.device
        ws = torch.empty(sz.workspace_bytes, dtype=torch.uint8, device=dev)
        st = torch.empty(sz.structure_bytes, dtype=torch.uint8, device=dev)
        if is_filter:
            rc, hd = vfilter_build(keys, b, eps, seed, opts, ws, st, stream)
        else:
            rc, hd = vf_build(keys, values, b, eps, seed, opts, ws, st, stream)
        return cls(hd, rc, is_filter, b, st, ws)

    @classmethod
    def prepare(cls, n: int, *, b: int, filter: bool, eps: float = 0.0, seed: int = 0,
                h: int | None = None, max_shard: int = 0, sigma: int | None = None,
                tmax: int | None = None, mwhc: bool = False, packed: bool = False,
                device=None):
        """A structure whose build is enqueued by launch() (capturable into a
        graph) and read back by finish(); shards sized for max_shard keys
        (0: the plan's bound)."""
        opts = vf_default_opts(h=h, sigma=sigma, tmax=tmax, mwhc=int(mwhc), packed=int(packed))
        sz = vf_plan(n, b, eps, filter, opts)
        dev = torch.device(device if device is not None else "cuda")
        ws = torch.empty(sz.workspace_bytes, dtype=torch.uint8, device=dev)
        st = torch.empty(sz.structure_bytes, dtype=torch.uint8, device=dev)
        hd = vf_build_prepare(n, b, eps, filter, seed, opts, ws, st, max_shard)
        return cls(hd, VF_OK, filter, b, st, ws)

    def launch(self, keys: torch.Tensor, values: torch.Tensor | None = None,
               stream=None) -> None:
        vf_build_launch(self.handle, keys, values, stream)

    def finish(self, stream=None) -> int:
        self.rc = vf_build_finish(self.handle, stream)
        return self.rc

    def release_workspace(self) -> None:
        self.workspace = None

    @property
    def info(self) -> dict:
        return vf_info(self.handle)

    @property
    def failures(self) -> list:
        return vf_failures(self.handle)

    def cells(self) -> torch.Tensor:
        """Device view of the S * V cells (cell_bytes each); for a packed
        structure the bit string of S * V b-bit fields as 64-bit words."""
        i = self.info
        if i["packed"]:
            nw = (i["S"] * i["V"] * i["b"] + 63) // 64
            return self.structure[: 8 * nw].view(torch.int64)
        nbytes = i["S"] * i["V"] * i["cell_bytes"]
        return self.structure[:nbytes].view(_CELL_DTYPE[i["cell_bytes"]]).view(i["S"], i["V"])

    def local_seeds(self) -> torch.Tensor:
        i = self.info
        off = i["local_seeds"] - self.structure.data_ptr()
        return self.structure[off: off + i["S"]]

    def query(self, keys: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        with _on(stream):
            if out is None:
                dt = torch.uint8 if self.is_filter else _CELL_DTYPE[self.info["cell_bytes"]]
                out = torch.empty(keys.numel(), dtype=dt, device=keys.device)
            if self.is_filter:
                vfilter_contains(self.handle, keys, out, stream)
            else:
                vf_query(self.handle, keys, out, stream)
        _used_on(stream, keys, out)
        return out

    def query_grouped(self, keys: torch.Tensor, out: torch.Tensor | None = None,
                      workspace: torch.Tensor | None = None, stream=None):
        """As query, with the keys grouped by shard first; workspace is a
        uint8 device tensor (default: one chunk for all keys).  Tensors made
        here are allocated on `stream`, and every tensor the call hands to
        the library is marked as used there, so the caching allocator does
        not reuse it while the call's kernels may still run."""
        with _on(stream):
            if workspace is None:
                workspace = torch.empty(vf_query_grouped_bytes(self.handle, keys.numel()),
                                        dtype=torch.uint8, device=keys.device)
            if out is None:
                dt = torch.uint8 if self.is_filter else _CELL_DTYPE[self.info["cell_bytes"]]
                out = torch.empty(keys.numel(), dtype=dt, device=keys.device)
            if self.is_filter:
                vfilter_contains_grouped(self.handle, keys, out, workspace, stream)
            else:
                vf_query_grouped(self.handle, keys, out, workspace, stream)
        _used_on(stream, keys, out, workspace)
        return out

    def free(self) -> None:
        if self.handle:
            vf_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


@dataclass
class Batch:
    """A batch of independent static functions built by one launch per cell
    width (``vf_batch_build``); instance i has keys[off[i]:off[i+1]]."""
    handle: C.c_void_p
    rc: int
    structure: torch.Tensor
    workspace: torch.Tensor | None

    @classmethod
    def build(cls, keys: torch.Tensor, values: torch.Tensor, n, b, *, seed: int = 0,
              sigma: int | None = None, c: tuple | None = None, tmax: int | None = None,
              max_window: int | None = None, packed: bool = False, small: int = 0,
              ring_cols: int | None = None, stream=None):
        opts = vf_default_opts(sigma=sigma, tmax=tmax, max_window=max_window,
                               packed=int(packed), small=small, ring_cols=ring_cols)
        if c is not None:
            opts.c_num, opts.c_den = c
        sz = vf_batch_plan(n, b, opts)
        dev = keys.device
        ws = torch.empty(sz.workspace_bytes, dtype=torch.uint8, device=dev)
        st = torch.empty(sz.structure_bytes, dtype=torch.uint8, device=dev)
        rc, hd = vf_batch_build(keys, values, n, b, seed, opts, ws, st, stream)
        return cls(hd, rc, st, ws)

    @classmethod
    def prepare(cls, n, b, *, seed: int = 0, device=None, sigma: int | None = None,
                c: tuple | None = None, tmax: int | None = None,
                max_window: int | None = None, packed: bool = False, small: int = 0,
                stream=None):
        """A batch whose build is enqueued by launch() (capturable into a
        graph) and read back by finish()."""
        opts = vf_default_opts(sigma=sigma, tmax=tmax, max_window=max_window,
                               packed=int(packed), small=small)
        if c is not None:
            opts.c_num, opts.c_den = c
        sz = vf_batch_plan(n, b, opts)
        dev = torch.device(device if device is not None else "cuda")
        ws = torch.empty(sz.workspace_bytes, dtype=torch.uint8, device=dev)
        st = torch.empty(sz.structure_bytes, dtype=torch.uint8, device=dev)
        hd = vf_batch_prepare(n, b, seed, opts, ws, st, stream)
        return cls(hd, VF_OK, st, ws)

    def launch(self, keys: torch.Tensor, values: torch.Tensor, stream=None) -> None:
        vf_batch_launch(self.handle, keys, values, stream)

    def finish(self, stream=None) -> int:
        self.rc = vf_batch_finish(self.handle, stream)
        return self.rc

    @property
    def info(self) -> dict:
        return vf_info(self.handle)

    @property
    def failures(self) -> list:
        return vf_failures(self.handle)

    def item(self, i: int) -> dict:
        return vf_batch_item(self.handle, i)

    def cells(self, i: int) -> torch.Tensor:
        """Device view of instance i's V cells (packed: its bit string as
        64-bit words)."""
        it = self.item(i)
        off = it["cells"] - self.structure.data_ptr()
        if it["packed"]:
            nw = (it["V"] * it["b"] + 63) // 64
            return self.structure[off: off + 8 * nw].view(torch.int64)
        nbytes = it["V"] * it["cell_bytes"]
        return self.structure[off: off + nbytes].view(_CELL_DTYPE[it["cell_bytes"]])

    def query(self, inst: torch.Tensor, keys: torch.Tensor, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
        vf_batch_query(self.handle, inst, keys, out, stream)
        return out

    def free(self) -> None:
        if self.handle:
            vf_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
