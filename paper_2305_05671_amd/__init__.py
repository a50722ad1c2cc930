"""Python binding of libelsar.so, the MI355X (gfx950) learned-partition sort.

Argument marshalling only: every step of the sort runs in the library's HIP
kernels.  PyTorch provides device memory (uint8 tensors on ``cuda``) and the
current stream.  Importing this package on a machine without the built library
raises; there is no CPU fallback.

Names follow the C ABI in ``include/elsar.h``:

* :func:`elsar_sort` -- the whole method (sample + fit, partition, in-bucket
  sort, concatenation) on device-resident records.
* :class:`Model` -- ``elsar_model_create`` / ``elsar_sample_fit`` /
  ``elsar_partition`` / ``elsar_sort_buckets`` step by step, plus inspection.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libelsar.so")

RMI, MLP, AUTO, RADIX, SPLINE = 0, 1, 2, 3, 4
MLP_PARAMS = 4801
MLP_GRAD_ROWS = 128
MLP_STEPS_NONE = 0xFFFFFFFF
OK, E_INVALID_ARG, E_NO_MEMORY, E_HIP, E_UNSUPPORTED, E_MODEL_REJECTED = range(6)


class FitParams(ctypes.Structure):
    _fields_ = [
        ("record_bytes", ctypes.c_uint32),
        ("key_bytes", ctypes.c_uint32),
        ("num_buckets", ctypes.c_uint32),
        ("num_leaves", ctypes.c_uint32),
        ("sample_size", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
        ("kind", ctypes.c_uint32),
        ("accept_ratio", ctypes.c_float),
        ("mlp_steps", ctypes.c_uint32),
        ("region_pct", ctypes.c_uint32),
        ("key_len_offset", ctypes.c_uint32),
    ]


class ModelInfo(ctypes.Structure):
    _fields_ = [
        ("kind_used", ctypes.c_uint32),
        ("mlp_rejected", ctypes.c_uint32),
        ("num_buckets", ctypes.c_uint32),
        ("num_leaves", ctypes.c_uint32),
        ("sample_size", ctypes.c_uint64),
        ("n_fit", ctypes.c_uint64),
        ("root_a0", ctypes.c_float),
        ("root_a1", ctypes.c_float),
        ("max_sample_bucket", ctypes.c_uint32),
        ("opt_sample_bucket", ctypes.c_uint32),
        ("mlp_leaves", ctypes.c_uint32),
        ("spline_segments", ctypes.c_uint32),
        ("rmi_max_sample_bucket", ctypes.c_uint32),
        ("eq_max_sample_bucket", ctypes.c_uint32),
        ("net_max_sample_bucket", ctypes.c_uint32),
        ("rmi_gate_passed", ctypes.c_uint32),
        ("perfect_sample_bucket", ctypes.c_float),
    ]


class PartitionStats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64),
        ("num_buckets", ctypes.c_uint32),
        ("spill_count", ctypes.c_uint32),
        ("mid_buckets", ctypes.c_uint32),
        ("big_buckets", ctypes.c_uint32),
        ("max_bucket", ctypes.c_uint32),
        ("mid_records", ctypes.c_uint32),
        ("big_records", ctypes.c_uint32),
        ("split_segments", ctypes.c_uint32),
        ("split_segment_cap", ctypes.c_uint32),
        ("split_overflow", ctypes.c_uint32),
    ]


class Timings(ctypes.Structure):
    _fields_ = [
        ("sample_fit_ms", ctypes.c_float),
        ("partition_ms", ctypes.c_float),
        ("scan_ms", ctypes.c_float),
        ("bucket_sort_lds_ms", ctypes.c_float),
        ("bucket_sort_rest_ms", ctypes.c_float),
        ("total_ms", ctypes.c_float),
        ("calls", ctypes.c_uint32),
    ]


class Job(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("d_out", ctypes.c_void_p), ("n", ctypes.c_uint64)]


HOST_SAMPLE_FIRST_CHUNK = 1


class HostStats(ctypes.Structure):
    _fields_ = [
        ("chunk_records", ctypes.c_uint64),
        ("pass_records", ctypes.c_uint64),
        ("passes", ctypes.c_uint32),
        ("num_buckets", ctypes.c_uint32),
        ("runs", ctypes.c_uint32),
        ("copy_passes", ctypes.c_uint32),
        ("link_bytes", ctypes.c_uint64),
        ("fit_ms", ctypes.c_float),
        ("count_ms", ctypes.c_float),
        ("passes_ms", ctypes.c_float),
        ("total_ms", ctypes.c_float),
    ]


class ElsarError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {status_string(status)} ({status})")
        self.status = status


_lib = None
_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t


def lib():
    """Load libelsar.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int
        sig = {
            "elsar_fit_params_default": ([ctypes.POINTER(FitParams)], st),
            "elsar_model_create": ([ctypes.POINTER(FitParams), _U64, ctypes.POINTER(_P)], st),
            "elsar_model_destroy": ([_P], None),
            "elsar_fit_workspace_size": ([_P, _U64, ctypes.POINTER(_SZ)], st),
            "elsar_sample_fit": ([_P, _P, _U64, _P, _SZ, _P], st),
            "elsar_partition_size": ([_P, _U64, ctypes.POINTER(_SZ)], st),
            "elsar_partition": ([_P, _P, _U64, _P, _SZ, _P, _P], st),
            "elsar_sort_buckets": ([_P, _P, _SZ, _U64, _P, _P, _P], st),
            "elsar_sort_workspace_size": ([ctypes.POINTER(FitParams), _U64, ctypes.POINTER(_SZ)], st),
            "elsar_sort": ([_P, _U64, _P, ctypes.POINTER(FitParams), _P, _SZ, _P], st),
            "elsar_sort_noalloc": ([_P, _U64, _P, ctypes.POINTER(FitParams), _P], st),
            "elsar_model_info_get": ([_P, ctypes.POINTER(ModelInfo)], st),
            "elsar_sort_batch_model_info": ([ctypes.POINTER(Job), ctypes.c_uint32, ctypes.POINTER(FitParams), _P, _SZ,
                                             ctypes.c_uint32, ctypes.POINTER(ModelInfo)], st),
            "elsar_model_leaves": ([_P, _P, _P, _P, _P, _P], st),
            "elsar_partition_stats_get": ([_P, _P, _SZ, ctypes.POINTER(PartitionStats)], st),
            "elsar_model_mlp_get": ([_P, _P, _P, _P, _P], st),
            "elsar_model_spline_get": ([_P, _P, _P, _P], st),
            "elsar_sort_batch_workspace_size": ([ctypes.POINTER(Job), ctypes.c_uint32, ctypes.POINTER(FitParams),
                                                 ctypes.POINTER(_SZ)], st),
            "elsar_sort_batch": ([ctypes.POINTER(Job), ctypes.c_uint32, ctypes.POINTER(FitParams), _P, _SZ, _P], st),
            "elsar_sort_host_workspace_size": ([ctypes.POINTER(FitParams), _U64, _U64, _U64, ctypes.POINTER(_SZ)],
                                               st),
            "elsar_sort_host": ([_P, _U64, _P, _P, ctypes.POINTER(FitParams), _U64, _U64, ctypes.c_uint32, _P, _SZ,
                                 _P, ctypes.POINTER(HostStats)], st),
            "elsar_mlp_forward": ([_P, _P, _P, _U64, _P], st),
            "elsar_mlp_gradient": ([_P, _P, _P, _P, _P, _P], st),
            "elsar_mlp_train_step": ([_P, _P, _P, _P, _P, ctypes.c_uint32, ctypes.c_float, _P, _P, _P, _P], st),
            "elsar_set_timing": ([ctypes.c_int], st),
            "elsar_timings_get": ([ctypes.POINTER(Timings)], st),
            "elsar_status_string": ([ctypes.c_int], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().elsar_status_string(s).decode()


def _check(fn: str, s: int):
    if s != OK:
        raise ElsarError(fn, s)


def fit_params(record_bytes=100, key_bytes=10, num_buckets=0, num_leaves=0, sample_size=0, seed=0,
               kind=RMI, accept_ratio=1.5, mlp_steps=0, region_pct=0, key_len_offset=0) -> FitParams:
    p = FitParams()
    _check("elsar_fit_params_default", lib().elsar_fit_params_default(ctypes.byref(p)))
    p.record_bytes, p.key_bytes = record_bytes, key_bytes
    p.num_buckets, p.num_leaves = num_buckets, num_leaves
    p.sample_size, p.seed, p.kind = sample_size, seed, kind
    p.accept_ratio, p.mlp_steps = accept_ratio, mlp_steps
    p.region_pct = region_pct
    p.key_len_offset = key_len_offset
    return p


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev_bytes(nbytes: int, device):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _check_records(t, record_bytes):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("records must be a contiguous uint8 CUDA tensor")
    if t.numel() % record_bytes:
        raise ValueError("tensor size is not a whole number of records")
    return t.numel() // record_bytes


def sort_workspace_size(n: int, params: FitParams) -> int:
    sz = _SZ()
    _check("elsar_sort_workspace_size", lib().elsar_sort_workspace_size(ctypes.byref(params), n, ctypes.byref(sz)))
    return sz.value


def elsar_sort(records, out=None, params: FitParams | None = None, workspace=None, stream=None):
    """Sort device-resident records (uint8 tensor of n*R bytes) into ``out``
    (a new tensor unless given; may be ``records`` itself for in place)."""
    params = params or fit_params()
    n = _check_records(records, params.record_bytes)
    if out is None:
        import torch
        out = torch.empty_like(records)
    if _check_records(out, params.record_bytes) != n:
        raise ValueError("out must hold n records")
    need = sort_workspace_size(n, params)
    if workspace is None or workspace.numel() < need:
        workspace = _dev_bytes(need, records.device)
    _check("elsar_sort", lib().elsar_sort(records.data_ptr(), n, out.data_ptr(), ctypes.byref(params),
                                          workspace.data_ptr(), workspace.numel(), _stream(stream)))
    return out


NOALLOC_SCRATCH_BYTES = 256 << 20
MAX_DEVICE_RECORDS = 400_000_000  # ELSAR_MAX_DEVICE_RECORDS: the largest in-HBM sort


def elsar_sort_noalloc(records, out, params: FitParams | None = None, stream=None):
    """elsar_sort_noalloc: the sort with the library's own fixed device scratch
    as workspace (no device allocation in the call).  ``out`` must be given
    (may be ``records``)."""
    params = params or fit_params()
    n = _check_records(records, params.record_bytes)
    if _check_records(out, params.record_bytes) != n:
        raise ValueError("out must hold n records")
    _check("elsar_sort_noalloc", lib().elsar_sort_noalloc(records.data_ptr(), n, out.data_ptr(),
                                                          ctypes.byref(params), _stream(stream)))
    return out


def _job_table(inputs, outputs, record_bytes):
    if outputs is None:
        outputs = inputs
    if len(outputs) != len(inputs):
        raise ValueError("one output per input")
    table = (Job * max(len(inputs), 1))()
    for i, (a, b) in enumerate(zip(inputs, outputs)):
        n = _check_records(a, record_bytes)
        if _check_records(b, record_bytes) != n:
            raise ValueError(f"job {i}: output size differs from input")
        table[i].d_in, table[i].d_out, table[i].n = a.data_ptr(), b.data_ptr(), n
    return table


def sort_batch_workspace_size(inputs, params: FitParams | None = None, outputs=None) -> int:
    params = params or fit_params()
    table = _job_table(inputs, outputs, params.record_bytes)
    sz = _SZ()
    _check("elsar_sort_batch_workspace_size",
           lib().elsar_sort_batch_workspace_size(table, len(inputs), ctypes.byref(params), ctypes.byref(sz)))
    return sz.value


def sort_batch(inputs, outputs=None, params: FitParams | None = None, workspace=None, stream=None):
    """elsar_sort_batch: sort every job (a uint8 CUDA tensor of n*R bytes) into
    the matching output (in place when ``outputs`` is None).  Returns the
    workspace so that a later call with the same tensors can reuse it (and
    with it the recorded graph)."""
    params = params or fit_params()
    table = _job_table(inputs, outputs, params.record_bytes)
    sz = _SZ()
    _check("elsar_sort_batch_workspace_size",
           lib().elsar_sort_batch_workspace_size(table, len(inputs), ctypes.byref(params), ctypes.byref(sz)))
    if workspace is None or workspace.numel() < sz.value:
        workspace = _dev_bytes(sz.value, inputs[0].device)
    _check("elsar_sort_batch", lib().elsar_sort_batch(table, len(inputs), ctypes.byref(params),
                                                      workspace.data_ptr(), workspace.numel(), _stream(stream)))
    return workspace


def sort_batch_model_info(inputs, job: int, workspace, outputs=None, params: FitParams | None = None) -> ModelInfo:
    """elsar_sort_batch_model_info: the model the last sort_batch call with
    these tensors, parameters and workspace fitted for job ``job``."""
    params = params or fit_params()
    table = _job_table(inputs, outputs, params.record_bytes)
    i = ModelInfo()
    _check("elsar_sort_batch_model_info",
           lib().elsar_sort_batch_model_info(table, len(inputs), ctypes.byref(params), workspace.data_ptr(),
                                             workspace.numel(), job, ctypes.byref(i)))
    return i


def sort_host_workspace_size(n: int, params: FitParams | None = None, chunk_records: int = 0,
                             pass_records: int = 0) -> int:
    params = params or fit_params()
    sz = _SZ()
    _check("elsar_sort_host_workspace_size",
           lib().elsar_sort_host_workspace_size(ctypes.byref(params), n, chunk_records, pass_records,
                                                ctypes.byref(sz)))
    return sz.value


def sort_host(h_in, h_out, params: FitParams | None = None, chunk_records: int = 0, pass_records: int = 0,
              workspace=None, stream=None, h_frag=None, first_chunk_sample: bool = False) -> HostStats:
    """elsar_sort_host: records in host memory (uint8 CPU tensors; pinned ones,
    made with pin_memory=True, copy fastest) sorted into h_out.  h_frag holds
    the sorted runs: a host tensor of the same size, ``h_in`` itself (the input
    is then overwritten), or None for a new one (pinned when h_in is).  The
    device workspace is sized for group passes of ``pass_records`` records (0:
    the whole input in one pass) unless one is given; ``pass_records`` also
    bounds the group passes of a given workspace.  Synchronous; returns the
    call's statistics."""
    import torch
    params = params or fit_params()
    if h_frag is None:
        h_frag = torch.empty(h_in.numel(), dtype=torch.uint8, pin_memory=bool(h_in.is_pinned()))
    for t in (h_in, h_out, h_frag):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or t.is_cuda or not t.is_contiguous():
            raise TypeError("host records must be contiguous uint8 CPU tensors")
    n = h_in.numel() // params.record_bytes
    if h_in.numel() % params.record_bytes or h_out.numel() != h_in.numel() or h_frag.numel() != h_in.numel():
        raise ValueError("input, output and fragment store must hold the same whole number of records")
    if workspace is None:
        workspace = _dev_bytes(sort_host_workspace_size(n, params, chunk_records, pass_records), "cuda")
    st = HostStats()
    flags = HOST_SAMPLE_FIRST_CHUNK if first_chunk_sample else 0
    _check("elsar_sort_host", lib().elsar_sort_host(h_in.data_ptr(), n, h_out.data_ptr(), h_frag.data_ptr(),
                                                    ctypes.byref(params), chunk_records, pass_records, flags,
                                                    workspace.data_ptr(), workspace.numel(), _stream(stream),
                                                    ctypes.byref(st)))
    return st


class Model:
    """elsar_model: fit, partition and sort step by step."""

    def __init__(self, n: int, params: FitParams | None = None):
        self.params = params or fit_params()
        self.n = n
        h = _P()
        _check("elsar_model_create", lib().elsar_model_create(ctypes.byref(self.params), n, ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.elsar_model_destroy(h)
            self._h = None

    def sample_fit(self, records, workspace=None, stream=None):
        n = _check_records(records, self.params.record_bytes)
        sz = _SZ()
        _check("elsar_fit_workspace_size", lib().elsar_fit_workspace_size(self._h, n, ctypes.byref(sz)))
        if workspace is None or workspace.numel() < sz.value:
            workspace = _dev_bytes(sz.value, records.device)
        s = lib().elsar_sample_fit(self._h, records.data_ptr(), n, workspace.data_ptr(), workspace.numel(),
                                   _stream(stream))
        self._fit_ws = workspace  # keep alive until the stream has used it
        # kind MLP reports a rejected network (the linear root is kept and usable)
        self.rejected = s == E_MODEL_REJECTED
        if not self.rejected:
            _check("elsar_sample_fit", s)
        return self

    def partition_size(self, n: int) -> int:
        sz = _SZ()
        _check("elsar_partition_size", lib().elsar_partition_size(self._h, n, ctypes.byref(sz)))
        return sz.value

    def partition(self, records, part=None, offsets=None, stream=None):
        import torch
        n = _check_records(records, self.params.record_bytes)
        need = self.partition_size(n)
        if part is None or part.numel() < need:
            part = _dev_bytes(need, records.device)
        B = self.info().num_buckets
        if offsets is None:
            offsets = torch.empty(B + 1, dtype=torch.int64, device=records.device)
        _check("elsar_partition", lib().elsar_partition(self._h, records.data_ptr(), n, part.data_ptr(),
                                                        part.numel(), offsets.data_ptr(), _stream(stream)))
        return part, offsets

    def sort_buckets(self, part, offsets, n: int, out, stream=None):
        _check("elsar_sort_buckets", lib().elsar_sort_buckets(self._h, part.data_ptr(), part.numel(), n,
                                                              offsets.data_ptr(), out.data_ptr(),
                                                              _stream(stream)))
        return out

    def info(self) -> ModelInfo:
        i = ModelInfo()
        _check("elsar_model_info_get", lib().elsar_model_info_get(self._h, ctypes.byref(i)))
        return i

    def leaves(self):
        import numpy as np
        L = self.info().num_leaves
        base = np.zeros(L, np.uint64)
        c = np.zeros(L, np.float32)
        b = np.zeros(L, np.float32)
        lo = np.zeros(L, np.uint32)
        hi = np.zeros(L, np.uint32)
        _check("elsar_model_leaves", lib().elsar_model_leaves(self._h, base.ctypes.data, c.ctypes.data,
                                                              b.ctypes.data, lo.ctypes.data, hi.ctypes.data))
        return base, c, b, lo, hi

    def mlp(self):
        """(params[4801] f32, knots[9] u64, bound[L+1] u64, first[L+1] u32) of the MLP root."""
        import numpy as np
        L = self.info().mlp_leaves
        params = np.zeros(MLP_PARAMS, np.float32)
        knots = np.zeros(9, np.uint64)
        bound = np.zeros(L + 1, np.uint64)
        first = np.zeros(L + 1, np.uint32)
        _check("elsar_model_mlp_get", lib().elsar_model_mlp_get(self._h, params.ctypes.data, knots.ctypes.data,
                                                                bound.ctypes.data, first.ctypes.data))
        return params, knots, bound, first

    def spline(self):
        """(knots[K+1] u64, bound[L+1] u64, first[L+1] u32) of the equi-depth leaves and the spline root."""
        import numpy as np
        i = self.info()
        knots = np.zeros(i.spline_segments + 1, np.uint64)
        bound = np.zeros(i.mlp_leaves + 1, np.uint64)
        first = np.zeros(i.mlp_leaves + 1, np.uint32)
        _check("elsar_model_spline_get", lib().elsar_model_spline_get(self._h, knots.ctypes.data, bound.ctypes.data,
                                                                      first.ctypes.data))
        return knots, bound, first

    def partition_stats(self, part) -> PartitionStats:
        s = PartitionStats()
        _check("elsar_partition_stats_get", lib().elsar_partition_stats_get(self._h, part.data_ptr(), part.numel(),
                                                                            ctypes.byref(s)))
        return s


def set_timing(enabled: bool) -> None:
    _check("elsar_set_timing", lib().elsar_set_timing(1 if enabled else 0))


def timings() -> Timings:
    t = Timings()
    _check("elsar_timings_get", lib().elsar_timings_get(ctypes.byref(t)))
    return t


def mlp_forward(params, knots, codes):
    """elsar_mlp_forward: y of every code (host arrays in, float32 array out)."""
    import numpy as np
    params = np.ascontiguousarray(params, np.float32)
    knots = np.ascontiguousarray(knots, np.uint64)
    codes = np.ascontiguousarray(codes, np.uint64)
    if params.size != MLP_PARAMS or knots.size != 9:
        raise ValueError("params must hold 4801 values and knots 9")
    y = np.zeros(codes.size, np.float32)
    _check("elsar_mlp_forward", lib().elsar_mlp_forward(params.ctypes.data, knots.ctypes.data, codes.ctypes.data,
                                                        codes.size, y.ctypes.data))
    return y


def mlp_gradient(params, knots, codes, targets):
    """elsar_mlp_gradient: (loss, gradient[4801]) on MLP_GRAD_ROWS rows."""
    import numpy as np
    params = np.ascontiguousarray(params, np.float32)
    knots = np.ascontiguousarray(knots, np.uint64)
    codes = np.ascontiguousarray(codes, np.uint64)
    targets = np.ascontiguousarray(targets, np.float32)
    if params.size != MLP_PARAMS or knots.size != 9 or codes.size != MLP_GRAD_ROWS or targets.size != MLP_GRAD_ROWS:
        raise ValueError("params 4801, knots 9, codes and targets MLP_GRAD_ROWS each")
    g = np.zeros(MLP_PARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    _check("elsar_mlp_gradient", lib().elsar_mlp_gradient(params.ctypes.data, knots.ctypes.data, codes.ctypes.data,
                                                          targets.ctypes.data, g.ctypes.data, loss.ctypes.data))
    return float(loss[0]), g


def mlp_train_step(params, adam, knots, codes, targets, step: int, lr: float):
    """elsar_mlp_train_step: one training step (gradient, then the Adam update
    of step ``step``).  adam holds the first then the second moments.  Returns
    (params, adam, grad, loss) after the step."""
    import numpy as np
    params = np.ascontiguousarray(params, np.float32)
    adam = np.ascontiguousarray(adam, np.float32)
    knots = np.ascontiguousarray(knots, np.uint64)
    codes = np.ascontiguousarray(codes, np.uint64)
    targets = np.ascontiguousarray(targets, np.float32)
    if (params.size != MLP_PARAMS or adam.size != 2 * MLP_PARAMS or knots.size != 9
            or codes.size != MLP_GRAD_ROWS or targets.size != MLP_GRAD_ROWS):
        raise ValueError("params 4801, adam 9602, knots 9, codes and targets MLP_GRAD_ROWS each")
    p_out = np.zeros(MLP_PARAMS, np.float32)
    a_out = np.zeros(2 * MLP_PARAMS, np.float32)
    g = np.zeros(MLP_PARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    _check("elsar_mlp_train_step",
           lib().elsar_mlp_train_step(params.ctypes.data, adam.ctypes.data, knots.ctypes.data, codes.ctypes.data,
                                      targets.ctypes.data, step, lr, p_out.ctypes.data, a_out.ctypes.data,
                                      g.ctypes.data, loss.ctypes.data))
    return p_out, a_out, g, float(loss[0])
