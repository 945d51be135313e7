"""Python binding of liblor.so (ctypes). Argument marshalling only.

Every function has the name of the C entry point it calls and runs that
entry point on torch's current HIP stream (or the stream passed in). Device
buffers are torch tensors on a ROCm device; the library itself never
allocates device memory, so workspaces and outputs are allocated here with
torch when the caller does not pass them. When a stream is passed, those
allocations are made on that stream (torch's caching allocator then hands a
freed workspace only to later work of the same stream, which runs after the
kernels that used it). There is no fallback: if the built library is
missing, loading raises.

Unsigned 32-bit keys travel in torch.int32 tensors and 64-bit keys in
torch.int64 tensors (same bits).
"""
from __future__ import annotations

import ctypes
import functools
import inspect
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblor.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "lor.h")

LOR_OK, LOR_EINVAL, LOR_EALPHABET, LOR_ETOOLARGE, LOR_EWORKSPACE, LOR_EHIP, LOR_ESTALE = range(7)

_lib = None


class LorError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str):
        self.status = status
        self.detail = detail
        super().__init__(f"{fn}: status {status} ({_status_string(status)}): {detail}")


class lor_rmq(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("n", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("kind", ctypes.c_int32)]


class lor_overlap(ctypes.Structure):
    _fields_ = [("length", ctypes.c_int64), ("seq_p", ctypes.c_int32), ("seq_q", ctypes.c_int32),
                ("off_p", ctypes.c_int64), ("off_q", ctypes.c_int64)]


class lor_plan(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("digit_bits", ctypes.c_int32), ("radix_items_u32", ctypes.c_int32),
                ("radix_items_u64", ctypes.c_int32), ("merge_items", ctypes.c_int32), ("plcp_steps", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class lor_timing(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


def header_functions() -> list:
    """Names of the functions include/lor.h declares."""
    with open(HEADER_PATH) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lor_[a-z0-9_]+)\s*\(", text)))


def lib():
    """Load liblor.so (after torch, so both use the same HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime liblor.so links against)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(python -m paper_1404_3448_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "lor_status_string": ([I32], ctypes.c_char_p),
        "lor_last_error": ([], ctypes.c_char_p),
        "lor_version": ([], I32),
        "lor_build_sa_workspace": ([I64, I32], SZ),
        "lor_build_sa": ([P, P, I32, P, P, P, SZ, P], I32),
        "lor_build_sa_static": ([P, P, I32, P, P, P], I32),
        "lor_suffix_array_workspace": ([I64], SZ),
        "lor_suffix_array_i32": ([P, I64, I32, P, P, SZ, P], I32),
        "lor_build_lcp_workspace": ([I64], SZ),
        "lor_build_lcp": ([P, I64, P, P, P, P, SZ, P], I32),
        "lor_rmq_bytes": ([I64], SZ),
        "lor_rmq_build": ([P, I64, P, SZ, ctypes.POINTER(lor_rmq), P], I32),
        "lor_rmq_query": ([ctypes.POINTER(lor_rmq), P, P, I32, P, P, I64, P, P, P], I32),
        "lor_rmq_compact_bytes": ([I64], SZ),
        "lor_rmq_compact_build": ([P, I64, P, SZ, ctypes.POINTER(lor_rmq), P], I32),
        "lor_longest_overlap_workspace": ([I64, I32], SZ),
        "lor_longest_overlap": ([P, P, I64, P, I32, ctypes.POINTER(lor_overlap), P, SZ, P], I32),
        "lor_longest_overlap_batched_workspace": ([I64, I32], SZ),
        "lor_longest_overlap_batched": ([P, P, I32, P, P, P, SZ, P], I32),
        "lor_longest_overlap_batched_state": ([P, P, I32, P, P, P, P, P, SZ, P], I32),
        "lor_longest_overlap_ref_workspace": ([I64, I32], SZ),
        "lor_overlap_matrix_workspace": ([I64, I32], SZ),
        "lor_overlap_matrix": ([P, P, I64, P, I32, P, P, SZ, P], I32),
        "lor_longest_overlap_ref": ([P, P, I32, P, P, SZ, P], I32),
        "lor_longest_overlap_batched_graph_create": ([P, P, I32, P, P, P, SZ, P, ctypes.POINTER(P)], I32),
        "lor_longest_overlap_batched_graph_launch": ([P, P], I32),
        "lor_longest_overlap_batched_graph_status": ([P, P], I32),
        "lor_longest_overlap_batched_graph_levels": ([P], I32),
        "lor_longest_overlap_batched_graph_destroy": ([P], None),
        "lor_sort_pairs_workspace": ([I64, I32], SZ),
        "lor_sort_pairs_u32": ([P, P, I64, I32, I32, P, SZ, P], I32),
        "lor_sort_pairs_u64": ([P, P, I64, I32, I32, P, SZ, P], I32),
        "lor_sort_pairs_split_u32": ([P, P, I64, I32, I32, P, SZ, P], I32),
        "lor_plan_default": ([ctypes.POINTER(lor_plan)], None),
        "lor_plan_get": ([ctypes.POINTER(lor_plan)], None),
        "lor_plan_set": ([ctypes.POINTER(lor_plan)], I32),
        "lor_check": ([P, P], I32),
        "lor_timing_enable": ([I32], None),
        "lor_timing_only": ([ctypes.c_char_p], None),
        "lor_timing_reset": ([], None),
        "lor_timing_read": ([ctypes.POINTER(lor_timing), I32], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _status_string(s: int) -> str:
    try:
        return lib().lor_status_string(s).decode()
    except Exception:
        return "?"


def _check(fn: str, status: int):
    if status != LOR_OK:
        raise LorError(fn, status, lib().lor_last_error().decode())


def _on_stream(fn):
    """Run `fn` with the `stream` keyword argument (when given) as torch's
    current stream, so that the workspaces and outputs it allocates belong to
    the stream its kernels are enqueued on."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapper(*args, **kwargs):
        stream = sig.bind_partial(*args, **kwargs).arguments.get("stream")
        if stream is None:
            return fn(*args, **kwargs)
        import torch
        with torch.cuda.stream(stream):
            return fn(*args, **kwargs)
    return wrapper


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _workspace(nbytes: int, device, ws=None):
    import torch
    if ws is not None:
        if ws.numel() * ws.element_size() < nbytes:
            raise ValueError(f"workspace holds {ws.numel() * ws.element_size()} bytes, {nbytes} needed")
        return ws
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _need(t, dtype, n, name):
    import torch
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{name}: need a contiguous {dtype} device tensor of >= {n} elements")


def _offsets(offsets) -> np.ndarray:
    o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if o.ndim != 1 or o.size < 2:
        raise ValueError("offsets: need int64[num_seqs + 1]")
    return o


# ----------------------------------------------------------- suffix array

def lor_build_sa_workspace(total_bases: int, num_seqs: int) -> int:
    return int(lib().lor_build_sa_workspace(total_bases, num_seqs))


@_on_stream
def lor_build_sa(seqs, offsets, joined_out=None, sa_out=None, ws=None, stream=None):
    """Suffix array of the separator-joined text. Returns (sa, joined)."""
    import torch
    o = _offsets(offsets)
    k = o.size - 1
    N = int(o[-1]) + k
    dev = seqs.device
    _need(seqs, torch.uint8, int(o[-1]), "seqs")
    if joined_out is None:
        joined_out = torch.empty(max(N, 1), dtype=torch.uint8, device=dev)
    if sa_out is None:
        sa_out = torch.empty(max(N, 1), dtype=torch.int32, device=dev)
    _need(joined_out, torch.uint8, N, "joined_out")
    _need(sa_out, torch.int32, N, "sa_out")
    nbytes = lor_build_sa_workspace(int(o[-1]), k)
    ws = _workspace(nbytes, dev, ws)
    st = lib().lor_build_sa(_ptr(seqs), o.ctypes.data_as(ctypes.c_void_p), k, _ptr(joined_out), _ptr(sa_out),
                            _ptr(ws), ws.numel() * ws.element_size(), _stream(stream))
    _check("lor_build_sa", st)
    return sa_out[:N], joined_out[:N]


STATIC_SCRATCH_BYTES = 64 << 20   # LOR_STATIC_SCRATCH_BYTES in include/lor.h


@_on_stream
def lor_build_sa_static(seqs, offsets, joined_out, sa_out, stream=None):
    """lor_build_sa with the library's fixed per-GPU workspace: the caller
    passes the outputs and nothing is allocated. Returns (sa, joined)."""
    import torch
    o = _offsets(offsets)
    k = o.size - 1
    N = int(o[-1]) + k
    _need(seqs, torch.uint8, int(o[-1]), "seqs")
    _need(joined_out, torch.uint8, N, "joined_out")
    _need(sa_out, torch.int32, N, "sa_out")
    st = lib().lor_build_sa_static(_ptr(seqs), o.ctypes.data_as(ctypes.c_void_p), k, _ptr(joined_out),
                                   _ptr(sa_out), _stream(stream))
    _check("lor_build_sa_static", st)
    return sa_out[:N], joined_out[:N]


def lor_suffix_array_workspace(n: int) -> int:
    return int(lib().lor_suffix_array_workspace(n))


@_on_stream
def lor_suffix_array_i32(text, alphabet_max: int, sa_out=None, ws=None, stream=None):
    """DC3 suffix array of an int32 text with symbols in 1..alphabet_max."""
    import torch
    n = text.numel()
    _need(text, torch.int32, n, "text")
    if sa_out is None:
        sa_out = torch.empty(max(n, 1), dtype=torch.int32, device=text.device)
    _need(sa_out, torch.int32, n, "sa_out")
    nbytes = lor_suffix_array_workspace(n)
    ws = _workspace(nbytes, text.device, ws)
    st = lib().lor_suffix_array_i32(_ptr(text), n, int(alphabet_max), _ptr(sa_out), _ptr(ws),
                                    ws.numel() * ws.element_size(), _stream(stream))
    _check("lor_suffix_array_i32", st)
    return sa_out[:n]


# -------------------------------------------------------------------- LCP

def lor_build_lcp_workspace(n: int) -> int:
    return int(lib().lor_build_lcp_workspace(n))


@_on_stream
def lor_build_lcp(text, sa, lcp_out=None, isa_out=None, want_isa=False, ws=None, stream=None):
    """LCP (and optionally ISA) of `text` given its suffix array. Returns (lcp, isa|None)."""
    import torch
    n = text.numel()
    _need(text, torch.uint8, n, "text")
    _need(sa, torch.int32, n, "sa")
    if lcp_out is None:
        lcp_out = torch.empty(max(n, 1), dtype=torch.int32, device=text.device)
    if isa_out is None and want_isa:
        isa_out = torch.empty(max(n, 1), dtype=torch.int32, device=text.device)
    _need(lcp_out, torch.int32, n, "lcp_out")
    if isa_out is not None:
        _need(isa_out, torch.int32, n, "isa_out")
    nbytes = lor_build_lcp_workspace(n)
    ws = _workspace(nbytes, text.device, ws)
    st = lib().lor_build_lcp(_ptr(text), n, _ptr(sa), _ptr(lcp_out), _ptr(isa_out), _ptr(ws),
                             ws.numel() * ws.element_size(), _stream(stream))
    _check("lor_build_lcp", st)
    return lcp_out[:n], (isa_out[:n] if isa_out is not None else None)


# -------------------------------------------------------------------- RMQ

class Rmq:
    """A built sparse table (full or compact): the C handle plus the tensor
    that owns its memory."""

    def __init__(self, handle: lor_rmq, table):
        self.handle = handle
        self.table = table

    @property
    def n(self):
        return int(self.handle.n)

    @property
    def levels(self):
        return int(self.handle.levels)

    @property
    def compact(self) -> bool:
        return int(self.handle.kind) == 1


def lor_rmq_bytes(n: int) -> int:
    return int(lib().lor_rmq_bytes(n))


def lor_rmq_compact_bytes(n: int) -> int:
    return int(lib().lor_rmq_compact_bytes(n))


@_on_stream
def lor_rmq_build(lcp, table=None, stream=None) -> Rmq:
    import torch
    n = lcp.numel()
    _need(lcp, torch.int32, n, "lcp")
    nbytes = lor_rmq_bytes(n)
    if table is None:
        table = torch.empty(max(nbytes // 4, 1), dtype=torch.int32, device=lcp.device)
    h = lor_rmq()
    st = lib().lor_rmq_build(_ptr(lcp), n, _ptr(table), table.numel() * table.element_size(), ctypes.byref(h),
                             _stream(stream))
    _check("lor_rmq_build", st)
    return Rmq(h, table)


@_on_stream
def lor_rmq_compact_build(lcp, table=None, stream=None) -> Rmq:
    import torch
    n = lcp.numel()
    _need(lcp, torch.int32, n, "lcp")
    nbytes = lor_rmq_compact_bytes(n)
    if table is None:
        table = torch.empty(max(nbytes // 4, 1), dtype=torch.int32, device=lcp.device)
    h = lor_rmq()
    st = lib().lor_rmq_compact_build(_ptr(lcp), n, _ptr(table), table.numel() * table.element_size(),
                                     ctypes.byref(h), _stream(stream))
    _check("lor_rmq_compact_build", st)
    return Rmq(h, table)


@_on_stream
def lor_rmq_query(rmq: Rmq, lcp, isa, mode: int, qi, qj, min_out=None, argmin_out=None, want_argmin=False,
                  stream=None):
    """mode 0: ranges [qi, qj] of LCP; mode 1: lcp of suffix pairs (qi, qj). Returns (min, argmin|None)."""
    import torch
    nq = qi.numel()
    _need(qi, torch.int32, nq, "qi")
    _need(qj, torch.int32, nq, "qj")
    if min_out is None:
        min_out = torch.empty(max(nq, 1), dtype=torch.int32, device=qi.device)
    if argmin_out is None and want_argmin:
        argmin_out = torch.empty(max(nq, 1), dtype=torch.int32, device=qi.device)
    st = lib().lor_rmq_query(ctypes.byref(rmq.handle), _ptr(lcp), _ptr(isa), int(mode), _ptr(qi), _ptr(qj), nq,
                             _ptr(min_out), _ptr(argmin_out), _stream(stream))
    _check("lor_rmq_query", st)
    return min_out[:nq], (argmin_out[:nq] if argmin_out is not None else None)


# --------------------------------------------------------- longest overlap

def lor_longest_overlap_workspace(n: int, num_seqs: int) -> int:
    return int(lib().lor_longest_overlap_workspace(n, num_seqs))


@_on_stream
def lor_longest_overlap(sa, lcp, offsets, ws=None, stream=None) -> tuple:
    """(length, seq_p, off_p, seq_q, off_q) of the longest region shared by two sequences."""
    o = _offsets(offsets)
    k = o.size - 1
    n = int(o[-1]) + k
    nbytes = lor_longest_overlap_workspace(n, k)
    ws = _workspace(nbytes, sa.device, ws)
    out = lor_overlap()
    st = lib().lor_longest_overlap(_ptr(sa), _ptr(lcp), n, o.ctypes.data_as(ctypes.c_void_p), k, ctypes.byref(out),
                                   _ptr(ws), ws.numel() * ws.element_size(), _stream(stream))
    _check("lor_longest_overlap", st)
    return (int(out.length), int(out.seq_p), int(out.off_p), int(out.seq_q), int(out.off_q))


# ------------------------------------------------ batched longest overlap

def lor_longest_overlap_batched_workspace(total_bases: int, num_pairs: int) -> int:
    return int(lib().lor_longest_overlap_batched_workspace(total_bases, num_pairs))


@_on_stream
def lor_longest_overlap_batched(seqs, offsets, out=None, ws=None, stream=None, plan=None):
    """Longest overlap of every pair (sequences 2p, 2p+1). Returns an int64
    device tensor [num_pairs, 4] of (length, off_p, off_q, seq_p | seq_q << 8)
    views of the lor_overlap records (see records_to_tuples)."""
    import torch
    o = _offsets(offsets)
    if (o.size - 1) % 2:
        raise ValueError("offsets: need int64[2 * num_pairs + 1]")
    P = (o.size - 1) // 2
    _need(seqs, torch.uint8, int(o[-1]), "seqs")
    if out is None:
        out = torch.empty(P * ctypes.sizeof(lor_overlap), dtype=torch.uint8, device=seqs.device)
    nbytes = lor_longest_overlap_batched_workspace(int(o[-1]), P)
    ws = _workspace(nbytes, seqs.device, ws)
    pl = None
    if plan is not None:
        pl = ctypes.byref(plan if isinstance(plan, lor_plan) else make_plan(**plan))
    st = lib().lor_longest_overlap_batched(_ptr(seqs), o.ctypes.data_as(ctypes.c_void_p), P, pl, _ptr(out),
                                           _ptr(ws), ws.numel() * ws.element_size(), _stream(stream))
    _check("lor_longest_overlap_batched", st)
    return out


@_on_stream
def lor_longest_overlap_batched_state(seqs, offsets, out=None, lcp_out=None, isa_out=None, ws=None, stream=None,
                                      plan=None):
    """lor_longest_overlap_batched that also returns the batch's LCP and ISA
    over the tagged text: pair p's own LCP / ISA are lcp[s_p:s_p+n_p] and
    isa[s_p:s_p+n_p] - s_p (pair_starts gives s_p). Returns (records, lcp, isa)."""
    import torch
    o = _offsets(offsets)
    if (o.size - 1) % 2:
        raise ValueError("offsets: need int64[2 * num_pairs + 1]")
    P = (o.size - 1) // 2
    N = int(o[-1]) + 2 * P
    _need(seqs, torch.uint8, int(o[-1]), "seqs")
    if out is None:
        out = torch.empty(P * ctypes.sizeof(lor_overlap), dtype=torch.uint8, device=seqs.device)
    if lcp_out is None:
        lcp_out = torch.empty(N, dtype=torch.int32, device=seqs.device)
    if isa_out is None:
        isa_out = torch.empty(N, dtype=torch.int32, device=seqs.device)
    _need(lcp_out, torch.int32, N, "lcp_out")
    _need(isa_out, torch.int32, N, "isa_out")
    nbytes = lor_longest_overlap_batched_workspace(int(o[-1]), P)
    ws = _workspace(nbytes, seqs.device, ws)
    pl = None
    if plan is not None:
        pl = ctypes.byref(plan if isinstance(plan, lor_plan) else make_plan(**plan))
    st = lib().lor_longest_overlap_batched_state(_ptr(seqs), o.ctypes.data_as(ctypes.c_void_p), P, pl, _ptr(out),
                                                 _ptr(lcp_out), _ptr(isa_out), _ptr(ws),
                                                 ws.numel() * ws.element_size(), _stream(stream))
    _check("lor_longest_overlap_batched_state", st)
    return out, lcp_out[:N], isa_out[:N]


def pair_starts(offsets) -> np.ndarray:
    """s_p for every pair of a batched offsets array, and the total after the last."""
    o = _offsets(offsets)
    lens = o[2::2] - o[0:-1:2] + 2
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


def lor_longest_overlap_ref_workspace(total_bases: int, num_queries: int) -> int:
    return int(lib().lor_longest_overlap_ref_workspace(total_bases, num_queries))


@_on_stream
def lor_longest_overlap_ref(seqs, offsets, out=None, ws=None, stream=None):
    """Longest substring every query (sequences 1..Q) shares with the
    reference (sequence 0). Returns the device lor_overlap records as bytes
    (see records_to_tuples)."""
    import torch
    o = _offsets(offsets)
    Q = o.size - 2
    if Q < 1:
        raise ValueError("offsets: need int64[num_queries + 2] with num_queries >= 1")
    _need(seqs, torch.uint8, int(o[-1]), "seqs")
    if out is None:
        out = torch.empty(Q * ctypes.sizeof(lor_overlap), dtype=torch.uint8, device=seqs.device)
    ws = _workspace(lor_longest_overlap_ref_workspace(int(o[-1]), Q), seqs.device, ws)
    st = lib().lor_longest_overlap_ref(_ptr(seqs), o.ctypes.data_as(ctypes.c_void_p), Q, _ptr(out), _ptr(ws),
                                       ws.numel() * ws.element_size(), _stream(stream))
    _check("lor_longest_overlap_ref", st)
    return out


def lor_overlap_matrix_workspace(n: int, num_seqs: int) -> int:
    return int(lib().lor_overlap_matrix_workspace(n, num_seqs))


@_on_stream
def lor_overlap_matrix(sa, lcp, offsets, out=None, ws=None, stream=None):
    """All-pairs longest overlap of the sequences of one joined text: device
    lor_overlap records, k x k, row a / column b (see records_to_tuples)."""
    import torch
    o = _offsets(offsets)
    k = o.size - 1
    n = sa.numel()
    _need(sa, torch.int32, n, "sa")
    _need(lcp, torch.int32, n, "lcp")
    if out is None:
        out = torch.empty(k * k * ctypes.sizeof(lor_overlap), dtype=torch.uint8, device=sa.device)
    ws = _workspace(lor_overlap_matrix_workspace(n, k), sa.device, ws)
    st = lib().lor_overlap_matrix(_ptr(sa), _ptr(lcp), n, o.ctypes.data_as(ctypes.c_void_p), k, _ptr(out), _ptr(ws),
                                  ws.numel() * ws.element_size(), _stream(stream))
    _check("lor_overlap_matrix", st)
    return out


class BatchedGraph:
    """A batched call captured as a HIP graph (lor_longest_overlap_batched_graph_*).
    Holds the tensors it is bound to; launch() enqueues a replay, status()
    waits and raises LorError (LOR_ESTALE) when the replay no longer fits the
    data in `seqs`."""

    def __init__(self, handle, seqs, out, ws, offsets):
        self._h = handle
        self.seqs, self.out, self.ws, self.offsets = seqs, out, ws, offsets

    @property
    def levels(self) -> int:
        return int(lib().lor_longest_overlap_batched_graph_levels(self._h))

    def launch(self, stream=None):
        _check("lor_longest_overlap_batched_graph_launch",
               lib().lor_longest_overlap_batched_graph_launch(self._h, _stream(stream)))
        return self.out

    def status(self, stream=None) -> int:
        st = lib().lor_longest_overlap_batched_graph_status(self._h, _stream(stream))
        _check("lor_longest_overlap_batched_graph_status", st)
        return st

    def close(self):
        if self._h:
            lib().lor_longest_overlap_batched_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lor_longest_overlap_batched_graph_create(seqs, offsets, stream, out=None, ws=None, plan=None) -> BatchedGraph:
    """Capture lor_longest_overlap_batched for these buffers as a HIP graph
    (stream: a created torch stream, not the null stream). `out` holds valid
    records on return."""
    import torch
    o = _offsets(offsets)
    if (o.size - 1) % 2:
        raise ValueError("offsets: need int64[2 * num_pairs + 1]")
    P = (o.size - 1) // 2
    _need(seqs, torch.uint8, int(o[-1]), "seqs")
    with torch.cuda.stream(stream):   # the graph's buffers belong to the stream it replays on
        if out is None:
            out = torch.empty(P * ctypes.sizeof(lor_overlap), dtype=torch.uint8, device=seqs.device)
        nbytes = lor_longest_overlap_batched_workspace(int(o[-1]), P)
        ws = _workspace(nbytes, seqs.device, ws)
    pl = None
    if plan is not None:
        pl = ctypes.byref(plan if isinstance(plan, lor_plan) else make_plan(**plan))
    h = ctypes.c_void_p()
    st = lib().lor_longest_overlap_batched_graph_create(_ptr(seqs), o.ctypes.data_as(ctypes.c_void_p), P, pl,
                                                        _ptr(out), _ptr(ws), ws.numel() * ws.element_size(),
                                                        _stream(stream), ctypes.byref(h))
    _check("lor_longest_overlap_batched_graph_create", st)
    return BatchedGraph(h, seqs, out, ws, o)


def records_to_tuples(out) -> list:
    """Device lor_overlap records -> [(length, seq_p, off_p, seq_q, off_q), ...]."""
    raw = out.cpu().numpy().tobytes()
    n = len(raw) // ctypes.sizeof(lor_overlap)
    arr = (lor_overlap * n).from_buffer_copy(raw)
    return [(int(r.length), int(r.seq_p), int(r.off_p), int(r.seq_q), int(r.off_q)) for r in arr]


# ------------------------------------------------------------- radix sort

def lor_sort_pairs_workspace(n: int, key_bytes: int) -> int:
    return int(lib().lor_sort_pairs_workspace(n, key_bytes))


def _sort_pairs(fn, key_bytes, keys, vals, bit_lo, bit_hi, ws, stream):
    import torch
    n = keys.numel()
    _need(keys, torch.int32 if key_bytes == 4 else torch.int64, n, "keys")
    _need(vals, torch.int32, n, "vals")
    nbytes = lor_sort_pairs_workspace(n, key_bytes)
    ws = _workspace(nbytes, keys.device, ws)
    st = getattr(lib(), fn)(_ptr(keys), _ptr(vals), n, int(bit_lo), int(bit_hi), _ptr(ws),
                            ws.numel() * ws.element_size(), _stream(stream))
    _check(fn, st)
    return keys, vals


@_on_stream
def lor_sort_pairs_u32(keys, vals, bit_lo=0, bit_hi=32, ws=None, stream=None):
    """Stable in-place sort of (keys: int32 bits, vals: int32) by key bits [bit_lo, bit_hi)."""
    return _sort_pairs("lor_sort_pairs_u32", 4, keys, vals, bit_lo, bit_hi, ws, stream)


@_on_stream
def lor_sort_pairs_u64(keys, vals, bit_lo=0, bit_hi=64, ws=None, stream=None):
    """Stable in-place sort of (keys: int64 bits, vals: int32) by key bits [bit_lo, bit_hi)."""
    return _sort_pairs("lor_sort_pairs_u64", 8, keys, vals, bit_lo, bit_hi, ws, stream)


@_on_stream
def lor_sort_pairs_split_u32(keys, vals, bit_lo=0, bit_hi=32, ws=None, stream=None):
    """The same sort with the paper's design (per-chunk one-bit splits, then
    pairwise merges of sorted chunks)."""
    return _sort_pairs("lor_sort_pairs_split_u32", 4, keys, vals, bit_lo, bit_hi, ws, stream)


# ----------------------------------------------------------------- plans

def lor_plan_default() -> lor_plan:
    p = lor_plan()
    lib().lor_plan_default(ctypes.byref(p))
    return p


def lor_plan_get() -> lor_plan:
    p = lor_plan()
    lib().lor_plan_get(ctypes.byref(p))
    return p


def lor_plan_set(plan=None):
    """Set the process-wide plan (a lor_plan, a dict of its fields, or None for the defaults)."""
    if plan is None:
        _check("lor_plan_set", lib().lor_plan_set(None))
        return
    p = plan if isinstance(plan, lor_plan) else make_plan(**plan)
    _check("lor_plan_set", lib().lor_plan_set(ctypes.byref(p)))


def make_plan(**fields) -> lor_plan:
    p = lor_plan_default()
    for k, v in fields.items():
        if k != "version":
            setattr(p, k, int(v))
    return p


# ----------------------------------------------------------------- timing

def lor_check(ws, stream=None) -> int:
    """Status the device left in a call's workspace header (synchronises the stream)."""
    return int(lib().lor_check(_ptr(ws), _stream(stream)))


def lor_timing_enable(on: bool = True):
    lib().lor_timing_enable(1 if on else 0)


def lor_timing_only(family=None):
    """Limit event timing to one kernel family (None: every family)."""
    lib().lor_timing_only(family.encode() if family else None)


def lor_timing_reset():
    lib().lor_timing_reset()


def lor_timing_read() -> dict:
    """{family: {"launches", "ms", "bytes"}} for every kernel family timed since the last reset."""
    cap = 64
    arr = (lor_timing * cap)()
    k = lib().lor_timing_read(arr, cap)
    return {arr[i].name.decode(): {"launches": int(arr[i].launches), "ms": float(arr[i].ms),
                                   "bytes": float(arr[i].bytes)} for i in range(min(k, cap))}


# ------------------------------------------------------------- whole path

@_on_stream
def longest_overlap_region(seqs, offsets, want_isa=False, stream=None):
    """Join -> SA -> LCP -> overlap on the device. Returns dict with sa, joined, lcp, isa, overlap."""
    sa, joined = lor_build_sa(seqs, offsets, stream=stream)
    lcp, isa = lor_build_lcp(joined, sa, want_isa=want_isa, stream=stream)
    ov = lor_longest_overlap(sa, lcp, offsets, stream=stream)
    return {"sa": sa, "joined": joined, "lcp": lcp, "isa": isa, "overlap": ov}
