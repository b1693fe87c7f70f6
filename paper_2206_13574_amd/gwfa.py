"""Python binding of the HIP graph wavefront alignment library (libgwfa.so).

Argument marshalling only: every step of the alignment runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  If the built
library is missing this module raises at import; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgwfa.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2206_13574_amd/build.py "
                      "(or __graft_entry__.build()); there is no fallback path")

# torch first: the library then binds to the HIP runtime torch has loaded,
# so both use one runtime (one set of devices, streams and allocations)
import torch as _torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# ---- error / status codes (include/gwfa.h) ---------------------------------
OK = 0
ERR_ARG, ERR_VERTEX, ERR_ALPHABET, ERR_EMPTY_LABEL = -1, -2, -3, -4
ERR_NOMEM, ERR_DEVICE, ERR_PATH_CAP, ERR_UNSUPPORTED, ERR_FORMAT = -5, -6, -7, -8, -9
GFA_FORWARD = 1
ST_OK, ST_MAX_SCORE, ST_ARENA, ST_BAD_INPUT, ST_UNREACHABLE = 0, 1, 2, 3, 4
PRUNE_NONE, PRUNE_HEURISTIC, PRUNE_LEARNED = 0, 1, 2

RESULT_DTYPE = np.dtype([("dist", "<i4"), ("end_v", "<i4"), ("end_off", "<i4"), ("status", "<i4"),
                         ("path_off", "<i8"), ("path_len", "<i4"), ("n_scores", "<i4"), ("work", "<i8"),
                         ("t_begin", "<i8"), ("t_end", "<i8"), ("start_off", "<i4"), ("clip", "<i4")])
assert RESULT_DTYPE.itemsize == 64


class Opts(ctypes.Structure):
    _fields_ = [("prune", ctypes.c_int32), ("a_diff", ctypes.c_int32), ("keep_threshold", ctypes.c_float),
                ("traceback", ctypes.c_int32), ("max_score", ctypes.c_int32), ("end_vertex", ctypes.c_int32),
                ("mlp_gate", ctypes.c_int32), ("mlp_period", ctypes.c_int32), ("query_end_free", ctypes.c_int32),
                ("walk_end_free", ctypes.c_int32)]


_P = ctypes.c_void_p
_i32, _i64 = ctypes.c_int32, ctypes.c_int64

_SIGS = {
    "gwfa_opts_default": (None, [ctypes.POINTER(Opts)]),
    "gwfa_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "gwfa_last_error": (ctypes.c_char_p, [_P]),
    "gwfa_ctx_create": (ctypes.c_int, [ctypes.c_int, _P, ctypes.POINTER(_P)]),
    "gwfa_ctx_destroy": (None, [_P]),
    "gwfa_ctx_config": (ctypes.c_int, [_P, _i32, _i32, _i32, _i32, _i32]),
    "gwfa_graph_create": (ctypes.c_int, [_P, _i32, _P, _P, _i64, _P, _P, ctypes.POINTER(_P)]),
    "gwfa_graph_destroy": (None, [_P]),
    "gwfa_pack_dev": (ctypes.c_int, [_P, _P, _i64, _P, _P, _P]),
    "gwfa_packed_words": (_i64, [_i64]),
    "gwfa_align_batch": (ctypes.c_int, [_P, _P, _i32, _P, _P, _P, ctypes.POINTER(Opts), _P, _P, _i64, _P]),
    "gwfa_align": (ctypes.c_int, [_P, _P, _P, _i32, _i32, ctypes.POINTER(Opts), _P, _P, _i64]),
    "gwfa_align_batch_dev": (ctypes.c_int, [_P, _P, _i32, _P, _P, _P, _P, ctypes.POINTER(Opts), _P, _P, _i64,
                                            _P, _P]),
    "gwfa_align_global_dev": (ctypes.c_int, [_P, _P, _i32, _P, _P, _P, _P, _P, ctypes.POINTER(Opts), _P, _P, _i64,
                                             _P, _P]),
    "gwfa_align_at_dev": (ctypes.c_int, [_P, _P, _i32, _P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(Opts), _P, _P,
                                         _i64, _P, _P]),
    "gwfa_align_dump_dev": (ctypes.c_int, [_P, _P, _i32, _P, _P, _P, _P, ctypes.POINTER(Opts), _P, _P, _i64,
                                           _P, _P, _i64, _P, _P]),
    "gwfa_align_batch_static_dev": (ctypes.c_int, [_P, _P, _i32, _P, _P, _P, _P, ctypes.POINTER(Opts), _P, _P,
                                                   _i64, _P, _P]),
    "gwfa_mlp_load": (ctypes.c_int, [_P, _P, _i64, _P]),
    "gwfa_mlp_grad_dev": (ctypes.c_int, [_P, _P, _i64, _i64, _P, _P, ctypes.c_float, _P, _P, _P, _P]),
    "gwfa_mlp_adam_dev": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _i32, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, _P]),
    "gwfa_mlp_cast_dev": (ctypes.c_int, [_P, _P, _P, _i64, _P]),
    "gwfa_mlp_logits_dev": (ctypes.c_int, [_P, _P, _i64, _i64, _P, _P, _P, _P]),
    "gwfa_label_entries": (ctypes.c_int, [_i32, _P, _P, _i64, _P, _P, _i32, _P, _P, _P, _i64, _P, _P, _P, _P,
                                          _P, _P, _P, _P, _i32]),
    "gwfa_stats": (ctypes.c_int, [_P, _P, _i32]),
    "gwfa_cigar_dev": (ctypes.c_int, [_P, _P, _i32, _P, _P, _P, _P, _P, _i64, _P, _P, _P, _P]),
    "gwfa_plan_create": (ctypes.c_int, [_P, _P, _i32, _P, _P, _P, _P, ctypes.POINTER(Opts), _P, _P, _i64, _P,
                                        ctypes.POINTER(_P)]),
    "gwfa_plan_launch": (ctypes.c_int, [_P, _P]),
    "gwfa_plan_finish": (ctypes.c_int, [_P, _P]),
    "gwfa_plan_destroy": (None, [_P]),
    "gwfa_gfa_load": (ctypes.c_int, [ctypes.c_char_p, _i32, ctypes.POINTER(_P), _P]),
    "gwfa_gfa_parse": (ctypes.c_int, [ctypes.c_char_p, _i64, _i32, ctypes.POINTER(_P), _P]),
    "gwfa_gfa_sizes": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "gwfa_gfa_graph": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "gwfa_gfa_vertex": (_i32, [_P, ctypes.c_char_p, _i32]),
    "gwfa_gfa_name": (ctypes.c_char_p, [_P, _i32, _P]),
    "gwfa_gfa_free": (None, [_P]),
}

MLP_N = 4801                      # parameters of the pruning network
DUMP_WORDS = 16                   # 4-byte words per trace record
DUMP_FIELDS = ("read", "score", "i", "v", "off", "W", "k", "attempt")
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class GwfaError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        msg = f"{where}: {_lib.gwfa_strerror(code).decode()} ({code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


def _check(code: int, where: str, ctx=None):
    if code != OK:
        detail = _lib.gwfa_last_error(ctx).decode() if ctx else ""
        raise GwfaError(code, where, detail)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(_P)


def _tptr(t):
    return _P(t.data_ptr()) if t is not None else None


def exported_symbols():
    return list(_SIGS)


def opts(prune: int = PRUNE_NONE, a_diff: int = 0, keep_threshold: float = 0.0, traceback: bool = True,
         max_score: int = -1, end_vertex: int = -1, mlp_gate: int = 0, mlp_period: int = 1,
         query_end_free: int = 0, walk_end_free: bool = False) -> Opts:
    o = Opts()
    _lib.gwfa_opts_default(ctypes.byref(o))
    o.prune, o.a_diff, o.keep_threshold = int(prune), int(a_diff), float(keep_threshold)
    o.traceback, o.max_score, o.end_vertex = int(bool(traceback)), int(max_score), int(end_vertex)
    o.mlp_gate, o.mlp_period = int(mlp_gate), int(mlp_period)
    o.query_end_free = int(query_end_free)
    o.walk_end_free = int(bool(walk_end_free))
    return o


def packed_words(n_bases: int) -> int:
    return int(_lib.gwfa_packed_words(int(n_bases)))


class Context:
    """A library context on a CUDA/HIP device, running on torch's current
    stream of that device (or an explicit torch stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = int(device)
        self.tdev = torch.device("cuda", self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.tdev)
        h = _P()
        _check(_lib.gwfa_ctx_create(self.device, _P(self.stream.cuda_stream), ctypes.byref(h)), "gwfa_ctx_create")
        self.h = h
        self._mlp = None

    def close(self):
        if getattr(self, "h", None):
            _lib.gwfa_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def config(self, lanes: int = 256, groups: int = 0, dir_log2_max: int = 16, list_cap: int = 1 << 15,
               dir_factor: int = 16):
        _check(_lib.gwfa_ctx_config(self.h, lanes, groups, dir_log2_max, list_cap, dir_factor), "gwfa_ctx_config",
               self.h)

    def stats(self, reset: bool = False) -> dict:
        out = np.zeros(16, dtype=np.int64)
        _check(_lib.gwfa_stats(self.h, _np_ptr(out), int(reset)), "gwfa_stats", self.h)
        keys = ["entries", "crossings", "pages", "chunks", "admitted", "reruns", "mlp_evals", "pruned", "scores",
                "ticks_expand", "ticks_rounds", "ticks_merge", "ticks_prune", "r13", "r14", "r15"]
        return dict(zip(keys, out.tolist()))

    def mlp_load(self, bf16_weights: np.ndarray, feat_scale: np.ndarray):
        w = np.ascontiguousarray(bf16_weights, dtype=np.uint16)
        sc = np.ascontiguousarray(feat_scale, dtype=np.float32)
        _check(_lib.gwfa_mlp_load(self.h, _np_ptr(w), len(w), _np_ptr(sc)), "gwfa_mlp_load", self.h)


class Graph:
    """Graph uploaded to the device (packed labels + out-edge CSR)."""

    def __init__(self, ctx: Context, seq, seg_off, edge_src, edge_dst):
        self.ctx = ctx
        seq = np.ascontiguousarray(np.frombuffer(seq, dtype=np.uint8) if isinstance(seq, (bytes, bytearray))
                                   else seq, dtype=np.uint8)
        seg_off = np.ascontiguousarray(seg_off, dtype=np.int64)
        src = np.ascontiguousarray(edge_src, dtype=np.int32)
        dst = np.ascontiguousarray(edge_dst, dtype=np.int32)
        self.n_vtx = len(seg_off) - 1
        h = _P()
        _check(_lib.gwfa_graph_create(ctx.h, self.n_vtx, _np_ptr(seq), _np_ptr(seg_off), len(src), _np_ptr(src),
                                      _np_ptr(dst), ctypes.byref(h)), "gwfa_graph_create", ctx.h)
        self.h = h

    @classmethod
    def of(cls, ctx: Context, g) -> "Graph":
        return cls(ctx, g.seq, g.seg_off, g.edge_src, g.edge_dst)

    def close(self):
        if getattr(self, "h", None):
            _lib.gwfa_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class DeviceBatch:
    """Queries resident in device memory (torch tensors)."""
    ascii: object        # uint8 [n_bases]
    packed: object       # int64 [packed_words]
    read_off: object     # int64 [n+1]
    v_start: object      # int32 [n]
    order: object        # int32 [n] longest first
    n: int
    bases: int


def upload_reads(ctx: Context, seq: np.ndarray, off: np.ndarray, v_start: np.ndarray) -> DeviceBatch:
    torch = ctx.torch
    seq = np.ascontiguousarray(seq, dtype=np.uint8)
    if not seq.flags.writeable:          # a view of bytes: torch wants writable memory
        seq = seq.copy()
    off = np.ascontiguousarray(off, dtype=np.int64)
    vs = np.ascontiguousarray(v_start, dtype=np.int32)
    n = len(vs)
    lens = off[1:] - off[:-1]
    order = np.argsort(-lens, kind="stable").astype(np.int32)
    dev = ctx.tdev
    return DeviceBatch(
        ascii=torch.from_numpy(seq if len(seq) else np.zeros(1, np.uint8)).to(dev),
        packed=torch.zeros(packed_words(len(seq)), dtype=torch.int64, device=dev),
        read_off=torch.from_numpy(off).to(dev),
        v_start=torch.from_numpy(vs if n else np.zeros(1, np.int32)).to(dev),
        order=torch.from_numpy(order if n else np.zeros(1, np.int32)).to(dev),
        n=n, bases=int(len(seq)))


@dataclass
class DeviceOut:
    res: object          # uint8 [n*40]
    path: object         # int32 [path_cap] or None
    path_used: object    # int64 [1]
    err: object          # int32 [1]


def alloc_out(ctx: Context, n: int, path_cap: int) -> DeviceOut:
    torch = ctx.torch
    dev = ctx.tdev
    return DeviceOut(res=torch.zeros(max(n, 1) * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev),
                     path=torch.zeros(path_cap, dtype=torch.int32, device=dev) if path_cap > 0 else None,
                     path_used=torch.zeros(1, dtype=torch.int64, device=dev),
                     err=torch.zeros(1, dtype=torch.int32, device=dev))


def pack_dev(ctx: Context, batch: DeviceBatch, err) -> None:
    """ASCII -> 2-bit packing of the queries on the device."""
    _check(_lib.gwfa_pack_dev(ctx.h, _tptr(batch.ascii), batch.bases, _tptr(batch.packed), _tptr(err),
                              _P(ctx.stream.cuda_stream)), "gwfa_pack_dev", ctx.h)


def align_dev(ctx: Context, graph: Graph, batch: DeviceBatch, out: DeviceOut, o: Opts, v_end=None,
              start_off=None, start_hi=None) -> None:
    """Aligns a device-resident batch (already packed) on ctx's stream.
    v_end: optional int32 device tensor of per-query end vertices (global
    form, gwfa_align_global_dev); start_off: optional int32 device tensor of
    per-query start offsets in the start vertex and start_hi the ends of free
    start windows (gwfa_align_at_dev)."""
    path_cap = int(out.path.numel()) if out.path is not None else 0
    if start_off is not None:
        _check(_lib.gwfa_align_at_dev(ctx.h, graph.h, batch.n, _tptr(batch.packed), _tptr(batch.read_off),
                                      _tptr(batch.v_start), _tptr(start_off), _tptr(start_hi), _tptr(v_end),
                                      _tptr(batch.order),
                                      ctypes.byref(o), _tptr(out.res), _tptr(out.path), path_cap,
                                      _tptr(out.path_used), _P(ctx.stream.cuda_stream)), "gwfa_align_at_dev", ctx.h)
        return
    if v_end is not None:
        _check(_lib.gwfa_align_global_dev(ctx.h, graph.h, batch.n, _tptr(batch.packed), _tptr(batch.read_off),
                                          _tptr(batch.v_start), _tptr(v_end), _tptr(batch.order), ctypes.byref(o),
                                          _tptr(out.res), _tptr(out.path), path_cap, _tptr(out.path_used),
                                          _P(ctx.stream.cuda_stream)), "gwfa_align_global_dev", ctx.h)
        return
    _check(_lib.gwfa_align_batch_dev(ctx.h, graph.h, batch.n, _tptr(batch.packed), _tptr(batch.read_off),
                                     _tptr(batch.v_start), _tptr(batch.order), ctypes.byref(o), _tptr(out.res),
                                     _tptr(out.path), path_cap, _tptr(out.path_used),
                                     _P(ctx.stream.cuda_stream)), "gwfa_align_batch_dev", ctx.h)


def align_static_dev(ctx: Context, graph: Graph, batch: DeviceBatch, out: DeviceOut, o: Opts) -> None:
    """gwfa_align_batch_static_dev: align_dev that allocates nothing (its
    working memory is the library's static device array)."""
    path_cap = int(out.path.numel()) if out.path is not None else 0
    _check(_lib.gwfa_align_batch_static_dev(ctx.h, graph.h, batch.n, _tptr(batch.packed), _tptr(batch.read_off),
                                            _tptr(batch.v_start), _tptr(batch.order), ctypes.byref(o),
                                            _tptr(out.res), _tptr(out.path), path_cap, _tptr(out.path_used),
                                            _P(ctx.stream.cuda_stream)), "gwfa_align_batch_static_dev", ctx.h)


def step_dev(ctx: Context, graph: Graph, batch: DeviceBatch, out: DeviceOut, o: Opts, v_end=None,
             start_off=None, start_hi=None) -> None:
    """One pass of the whole path on resident queries: pack, then align."""
    pack_dev(ctx, batch, out.err)
    align_dev(ctx, graph, batch, out, o, v_end, start_off, start_hi)


def fetch(out: DeviceOut, n: int):
    """Results (structured numpy array) and the path buffer (numpy)."""
    res = np.frombuffer(out.res.cpu().numpy().tobytes(), dtype=RESULT_DTYPE)[:n].copy()
    used = int(out.path_used.cpu().item())
    path = out.path[:min(used, out.path.numel())].cpu().numpy() if out.path is not None else None
    return res, path, used


def align(ctx: Context, graph: Graph, seq, off, v_start, o: Opts = None, path_cap: int = None, v_end=None,
          start_off=None, start_hi=None):
    """Convenience: host queries in, results out (through the device-side
    entry points).  v_end: optional per-query end vertices (global form);
    start_off: optional per-query start offsets in the start vertex; start_hi:
    optional ends of free start windows (needs start_off).
    Returns (results, paths) with paths a list of int32 arrays (or None when
    traceback is off)."""
    if o is None:
        o = opts()
    seq = np.ascontiguousarray(np.frombuffer(seq, dtype=np.uint8) if isinstance(seq, (bytes, bytearray)) else seq,
                               dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.int64)
    n = len(off) - 1
    batch = upload_reads(ctx, seq, off, v_start)
    if path_cap is None:
        path_cap = (int(off[-1]) + 64 * n) if o.traceback else 0
    out = alloc_out(ctx, n, path_cap)
    def dev_i32(x):
        return None if x is None else ctx.torch.from_numpy(
            np.ascontiguousarray(x, dtype=np.int32) if n else np.zeros(1, np.int32)).to(ctx.tdev)

    step_dev(ctx, graph, batch, out, o, dev_i32(v_end), dev_i32(start_off), dev_i32(start_hi))
    ctx.torch.cuda.synchronize(ctx.tdev)
    if int(out.err.cpu().item()) != 0:
        raise GwfaError(ERR_ALPHABET, "gwfa_pack_dev")
    res, path, used = fetch(out, n)
    paths = None
    if o.traceback:
        if used > path_cap:
            raise GwfaError(ERR_PATH_CAP, "align", f"needs {used} ids, buffer {path_cap}")
        paths = [path[r["path_off"]:r["path_off"] + r["path_len"]] if r["path_off"] >= 0 else None for r in res]
    return res, paths


def align_one(ctx: Context, graph: Graph, q, v_start: int, o: Opts = None, path_cap: int = None):
    """gwfa_align: one query from host memory.  Returns (code, result, walk)
    with walk None unless it was traced and fits."""
    if o is None:
        o = opts()
    qa = np.ascontiguousarray(np.frombuffer(q, dtype=np.uint8) if isinstance(q, (bytes, bytearray)) else q,
                              dtype=np.uint8)
    if path_cap is None:
        path_cap = len(qa) + 64
    res = np.zeros(1, dtype=RESULT_DTYPE)
    path = np.zeros(max(path_cap, 1), dtype=np.int32)
    code = _lib.gwfa_align(ctx.h, graph.h, _np_ptr(qa), len(qa), int(v_start), ctypes.byref(o), _np_ptr(res),
                           _np_ptr(path) if path_cap > 0 else None, int(path_cap))
    walk = None
    if code == OK and o.traceback and res[0]["path_off"] >= 0:
        walk = path[res[0]["path_off"]:res[0]["path_off"] + res[0]["path_len"]].copy()
    return code, res[0], walk


def align_host(ctx: Context, graph: Graph, seq, off, v_start, o: Opts = None, path_cap: int = 0):
    """The host-buffer entry point gwfa_align_batch (validates everything on
    the host first)."""
    if o is None:
        o = opts()
    seq = np.ascontiguousarray(np.frombuffer(seq, dtype=np.uint8) if isinstance(seq, (bytes, bytearray)) else seq,
                               dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.int64)
    vs = np.ascontiguousarray(v_start, dtype=np.int32)
    n = len(off) - 1
    res = np.zeros(max(n, 1), dtype=RESULT_DTYPE)
    path = np.zeros(max(path_cap, 1), dtype=np.int32)
    needed = ctypes.c_int64(0)
    code = _lib.gwfa_align_batch(ctx.h, graph.h, n, _np_ptr(seq), _np_ptr(off), _np_ptr(vs), ctypes.byref(o),
                                 _np_ptr(res), _np_ptr(path) if path_cap else None, int(path_cap),
                                 ctypes.byref(needed))
    return code, res[:n], path[:path_cap], int(needed.value)


# ---- trace dumps and training of the pruning network -----------------------

def align_dump_dev(ctx: Context, graph: Graph, batch: DeviceBatch, out: DeviceOut, o: Opts, dump, dump_count) -> None:
    """align_dev that also writes one trace record per wavefront entry and
    score into `dump` (float32 tensor [cap, 16]); `dump_count` (int64 [1])
    receives the number of records produced."""
    path_cap = int(out.path.numel()) if out.path is not None else 0
    _check(_lib.gwfa_align_dump_dev(ctx.h, graph.h, batch.n, _tptr(batch.packed), _tptr(batch.read_off),
                                    _tptr(batch.v_start), _tptr(batch.order), ctypes.byref(o), _tptr(out.res),
                                    _tptr(out.path), path_cap, _tptr(out.path_used), _tptr(dump),
                                    int(dump.shape[0]), _tptr(dump_count), _P(ctx.stream.cuda_stream)),
           "gwfa_align_dump_dev", ctx.h)


def split_dump(records: np.ndarray) -> dict:
    """Host view of trace records (numpy float32 [n, 16]): features [n, 8]
    and the integer fields."""
    rec = np.ascontiguousarray(records, dtype=np.float32)
    ints = rec[:, 8:16].view(np.int32)
    d = {name: ints[:, j].copy() for j, name in enumerate(DUMP_FIELDS)}
    d["feat"] = rec[:, :8].copy()
    return d


def final_attempt_mask(d: dict) -> np.ndarray:
    """Records of the last attempt of each query (earlier attempts were
    restarted with more working memory)."""
    if len(d["read"]) == 0:
        return np.zeros(0, dtype=bool)
    last = np.full(int(d["read"].max()) + 1, -1, dtype=np.int64)
    np.maximum.at(last, d["read"], d["attempt"].astype(np.int64))
    return d["attempt"] == last[d["read"]]


def mlp_grad_dev(ctx: Context, feat, label, scale: np.ndarray, w_bf16, grad, loss, pos_weight: float = 1.0,
                 n: int = None) -> None:
    """Mean loss gradient of the samples (feat float32 [n, stride>=8],
    label uint8 [n]) for bfloat16 weights w_bf16 (int16/uint16 view, 4801);
    overwrites grad (float32 [4801]) and loss (float32 [1])."""
    n = int(feat.shape[0]) if n is None else int(n)
    sc = np.ascontiguousarray(scale, dtype=np.float32)
    _check(_lib.gwfa_mlp_grad_dev(ctx.h, _tptr(feat), n, int(feat.stride(0)), _tptr(label), _np_ptr(sc),
                                  float(pos_weight), _tptr(w_bf16), _tptr(grad), _tptr(loss),
                                  _P(ctx.stream.cuda_stream)), "gwfa_mlp_grad_dev", ctx.h)


def mlp_adam_dev(ctx: Context, master, m1, m2, grad, w_bf16, step: int, lr: float, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8) -> None:
    _check(_lib.gwfa_mlp_adam_dev(ctx.h, _tptr(master), _tptr(m1), _tptr(m2), _tptr(grad), _tptr(w_bf16),
                                  int(step), float(lr), float(beta1), float(beta2), float(eps),
                                  _P(ctx.stream.cuda_stream)), "gwfa_mlp_adam_dev", ctx.h)


def mlp_cast_dev(ctx: Context, src, dst) -> None:
    _check(_lib.gwfa_mlp_cast_dev(ctx.h, _tptr(src), _tptr(dst), int(src.numel()), _P(ctx.stream.cuda_stream)),
           "gwfa_mlp_cast_dev", ctx.h)


def mlp_logits_dev(ctx: Context, feat, scale: np.ndarray, w_bf16, out, n: int = None) -> None:
    n = int(feat.shape[0]) if n is None else int(n)
    sc = np.ascontiguousarray(scale, dtype=np.float32)
    _check(_lib.gwfa_mlp_logits_dev(ctx.h, _tptr(feat), n, int(feat.stride(0)), _np_ptr(sc), _tptr(w_bf16),
                                    _tptr(out), _P(ctx.stream.cuda_stream)), "gwfa_mlp_logits_dev", ctx.h)


def label_entries(g, seq, off, v_start, read, score, i, v, offs, n_threads: int = 0):
    """Host labels of trace entries (see gwfa_label_entries): returns
    (cost, label, dist) numpy arrays."""
    gseq = np.ascontiguousarray(np.frombuffer(g.seq, dtype=np.uint8) if isinstance(g.seq, (bytes, bytearray))
                                else g.seq, dtype=np.uint8)
    goff = np.ascontiguousarray(g.seg_off, dtype=np.int64)
    src = np.ascontiguousarray(g.edge_src, dtype=np.int32)
    dst = np.ascontiguousarray(g.edge_dst, dtype=np.int32)
    seq = np.ascontiguousarray(np.frombuffer(seq, dtype=np.uint8) if isinstance(seq, (bytes, bytearray)) else seq,
                               dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.int64)
    vs = np.ascontiguousarray(v_start, dtype=np.int32)
    cols = [np.ascontiguousarray(a, dtype=np.int32) for a in (read, score, i, v, offs)]
    ne = len(cols[0])
    cost = np.zeros(max(ne, 1), dtype=np.int32)
    label = np.zeros(max(ne, 1), dtype=np.uint8)
    dist = np.zeros(max(len(vs), 1), dtype=np.int32)
    code = _lib.gwfa_label_entries(len(goff) - 1, _np_ptr(gseq), _np_ptr(goff), len(src), _np_ptr(src),
                                   _np_ptr(dst), len(vs), _np_ptr(seq), _np_ptr(off), _np_ptr(vs), ne,
                                   *[_np_ptr(c) for c in cols], _np_ptr(cost), _np_ptr(label), _np_ptr(dist),
                                   int(n_threads))
    _check(code, "gwfa_label_entries")
    return cost[:ne], label[:ne], dist[:len(vs)]


def align_dump(ctx: Context, graph: Graph, seq, off, v_start, o: Opts = None, dump_cap: int = 1 << 22):
    """Convenience: host queries in, (results, trace records as a dict of
    numpy columns restricted to each query's final attempt, records
    produced) out."""
    if o is None:
        o = opts(traceback=False)
    torch = ctx.torch
    seq = np.ascontiguousarray(np.frombuffer(seq, dtype=np.uint8) if isinstance(seq, (bytes, bytearray)) else seq,
                               dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.int64)
    n = len(off) - 1
    batch = upload_reads(ctx, seq, off, v_start)
    out = alloc_out(ctx, n, (int(off[-1]) + 64 * n) if o.traceback else 0)
    dump = torch.empty((max(int(dump_cap), 1), DUMP_WORDS), dtype=torch.float32, device=ctx.tdev)
    count = torch.zeros(1, dtype=torch.int64, device=ctx.tdev)
    pack_dev(ctx, batch, out.err)
    align_dump_dev(ctx, graph, batch, out, o, dump, count)
    torch.cuda.synchronize(ctx.tdev)
    if int(out.err.cpu().item()) != 0:
        raise GwfaError(ERR_ALPHABET, "gwfa_pack_dev")
    res, _, _ = fetch(out, n)
    produced = int(count.cpu().item())
    rec = dump[:min(produced, int(dump_cap))].cpu().numpy()
    d = split_dump(rec)
    keep = final_attempt_mask(d)
    d = {k: v[keep] for k, v in d.items()}
    return res, d, produced


class Plan:
    """The alignment of one resident batch captured as a HIP graph
    (gwfa_plan_*): launch() replays it on ctx's stream; finish() completes
    any re-runs for overflowed queries (synchronising)."""

    def __init__(self, ctx: Context, graph: Graph, batch: DeviceBatch, out: DeviceOut, o: Opts):
        self.ctx, self.keep = ctx, (graph, batch, out)
        path_cap = int(out.path.numel()) if out.path is not None else 0
        h = _P()
        _check(_lib.gwfa_plan_create(ctx.h, graph.h, batch.n, _tptr(batch.packed), _tptr(batch.read_off),
                                     _tptr(batch.v_start), _tptr(batch.order), ctypes.byref(o), _tptr(out.res),
                                     _tptr(out.path), path_cap, _tptr(out.path_used), ctypes.byref(h)),
               "gwfa_plan_create", ctx.h)
        self.h = h

    def launch(self):
        _check(_lib.gwfa_plan_launch(self.h, _P(self.ctx.stream.cuda_stream)), "gwfa_plan_launch", self.ctx.h)

    def finish(self):
        _check(_lib.gwfa_plan_finish(self.h, _P(self.ctx.stream.cuda_stream)), "gwfa_plan_finish", self.ctx.h)

    def close(self):
        if getattr(self, "h", None):
            _lib.gwfa_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


CIGAR_OPS = {7: "=", 8: "X", 1: "I", 2: "D", 4: "S"}


def cigar_dev(ctx: Context, graph: Graph, batch: DeviceBatch, out: DeviceOut, cigar_cap: int = None):
    """Base-level alignments of a finished alignment call (gwfa_cigar_dev):
    returns (ops uint32 numpy, off int64 [n], len int32 [n])."""
    torch = ctx.torch
    n = batch.n
    if cigar_cap is None:
        cigar_cap = 4 * int(batch.bases) + 64 * n
    cig = torch.zeros(max(cigar_cap, 1), dtype=torch.int32, device=ctx.tdev)
    coff = torch.zeros(max(n, 1), dtype=torch.int64, device=ctx.tdev)
    clen = torch.zeros(max(n, 1), dtype=torch.int32, device=ctx.tdev)
    used = torch.zeros(1, dtype=torch.int64, device=ctx.tdev)
    _check(_lib.gwfa_cigar_dev(ctx.h, graph.h, n, _tptr(batch.packed), _tptr(batch.read_off), _tptr(out.res),
                               _tptr(out.path), _tptr(cig), int(cigar_cap), _tptr(coff), _tptr(clen), _tptr(used),
                               _P(ctx.stream.cuda_stream)), "gwfa_cigar_dev", ctx.h)
    torch.cuda.synchronize(ctx.tdev)
    u = int(used.cpu().item())
    return (cig[:min(u, cigar_cap)].cpu().numpy().view(np.uint32), coff[:n].cpu().numpy(), clen[:n].cpu().numpy())


def cigar_string(ops: np.ndarray) -> str:
    return "".join(f"{int(w) >> 4}{CIGAR_OPS[int(w) & 15]}" for w in ops)


class GFA:
    """A sequence graph read from GFA 1 text (gwfa_gfa_*; host memory, no
    device).  Segment i is vertex 2i and its reverse complement 2i+1 (or
    vertex i with forward_only).  `graph` holds the arguments of
    gwfa_graph_create as a synth.Graph."""

    def __init__(self, path: str = None, text=None, forward_only: bool = False):
        from . import synth
        h = _P()
        line = ctypes.c_int64(0)
        flags = GFA_FORWARD if forward_only else 0
        if text is not None:
            data = text.encode() if isinstance(text, str) else bytes(text)
            rc = _lib.gwfa_gfa_parse(data, len(data), flags, ctypes.byref(h), ctypes.byref(line))
        else:
            rc = _lib.gwfa_gfa_load(os.fsencode(path), flags, ctypes.byref(h), ctypes.byref(line))
        if rc != OK:
            raise GwfaError(rc, "gwfa_gfa_parse" if text is not None else "gwfa_gfa_load",
                            f"line {line.value}" if line.value else "")
        self.h = h
        nv, nb, ne, ns, nsk = (ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(),
                               ctypes.c_int64())
        _check(_lib.gwfa_gfa_sizes(h, ctypes.byref(nv), ctypes.byref(nb), ctypes.byref(ne), ctypes.byref(ns),
                                   ctypes.byref(nsk)), "gwfa_gfa_sizes")
        seq = np.zeros(max(nb.value, 1), np.uint8)
        off = np.zeros(nv.value + 1, np.int64)
        src = np.zeros(max(ne.value, 1), np.int32)
        dst = np.zeros(max(ne.value, 1), np.int32)
        _check(_lib.gwfa_gfa_graph(h, _np_ptr(seq), _np_ptr(off), _np_ptr(src), _np_ptr(dst)), "gwfa_gfa_graph")
        self.n_segments = ns.value
        self.n_skipped = nsk.value
        self.graph = synth.Graph(seq[:nb.value], off, src[:ne.value].copy(), dst[:ne.value].copy(),
                                 pos=np.arange(nv.value, dtype=np.int64), meta=dict(source="gfa"))

    def vertex(self, name: str, reverse: bool = False) -> int:
        v = _lib.gwfa_gfa_vertex(self.h, name.encode(), int(bool(reverse)))
        if v < 0:
            raise GwfaError(v, "gwfa_gfa_vertex", name)
        return int(v)

    def name(self, v: int):
        rev = ctypes.c_int32(0)
        p = _lib.gwfa_gfa_name(self.h, int(v), ctypes.byref(rev))
        if p is None:
            raise GwfaError(ERR_VERTEX, "gwfa_gfa_name", str(v))
        return p.decode(), bool(rev.value)

    def close(self):
        if getattr(self, "h", None):
            _lib.gwfa_gfa_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
