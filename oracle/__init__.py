"""CPU oracle for graph wavefront alignment -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library in
``paper_2206_13574_amd``) never imports, links or calls it, and the two
share no code.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc by
``oracle/build.py``); this module only marshals arguments:

* :func:`dp_dense`   -- Eq. 1 (Section 2.2), dense rows + in-row fixpoint.
* :func:`dp_dense_global` -- the same rows, global form: the cell at the end
  of the end vertex.
* :func:`dp_capped`  -- Eq. 1 with values saturated at D+1 (exact if d* <= D).
* :func:`dp_batch`   -- many reads, OpenMP over reads.
* :func:`ed_global`, :func:`ed_banded` -- textbook pairwise edit distance.
* :func:`gwf`        -- Algorithms 1-4 (Sections 2.4-2.5), extension mode,
  optional pruning heuristic; also returns wavefront work counts.
* :mod:`oracle.mlp_ref` -- float64 reference of the pruning MLP.
* ``orc_rev_labels`` (labels.c) -- reverse form of Eq. 1 (cost to finish
  from a cell), the reference of the learned pruning's training labels.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.orc_dp_dense.argtypes = [i32, P, P, i64, P, P, P, i32, i32, P]
    lib.orc_dp_dense.restype = ctypes.c_int
    lib.orc_dp_dense_at.argtypes = [i32, P, P, i64, P, P, P, i32, i32, i32, i32, i32, i32, P]
    lib.orc_dp_dense_at.restype = ctypes.c_int
    lib.orc_dp_dense_global.argtypes = [i32, P, P, i64, P, P, P, i32, i32, i32, P]
    lib.orc_dp_dense_global.restype = ctypes.c_int
    lib.orc_dp_capped.argtypes = [i32, P, P, i64, P, P, P, i32, i32, i32, P]
    lib.orc_dp_capped.restype = ctypes.c_int
    lib.orc_dp_batch.argtypes = [i32, P, P, i64, P, P, i32, P, P, P, P, P, i32]
    lib.orc_dp_batch.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_ed_global.argtypes = [P, i64, P, i64]
    lib.orc_ed_global.restype = i64
    lib.orc_ed_banded.argtypes = [P, i64, P, i64, i64]
    lib.orc_ed_banded.restype = i64
    lib.orc_gwf.argtypes = [i32, P, P, i64, P, P, P, i32, i32, i32, i32, i32, i32, i32, i32, i32, P, P, P, i32,
                            P, i64, P]
    lib.orc_dp_dense_clip.argtypes = [i32, P, P, i64, P, P, P, i32, i32, i32, i32, i32, i32, i32, P]
    lib.orc_dp_dense_clip.restype = ctypes.c_int
    lib.orc_gwf.restype = ctypes.c_int
    lib.orc_rev_labels.argtypes = [i32, P, P, i64, P, P, P, i32, i32, P, P, P, P, i64, P]
    lib.orc_rev_labels.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _u8(x) -> np.ndarray:
    if isinstance(x, (bytes, bytearray)):
        return np.frombuffer(bytes(x), dtype=np.uint8).copy()
    if isinstance(x, str):
        return np.frombuffer(x.encode(), dtype=np.uint8).copy()
    return np.ascontiguousarray(x, dtype=np.uint8)


@dataclass
class OGraph:
    """Graph in the oracle's own form: ASCII labels concatenated, int64 label
    offsets (n+1), and an edge list."""
    seq: np.ndarray      # uint8 ASCII
    off: np.ndarray      # int64, n+1
    src: np.ndarray      # int32
    dst: np.ndarray      # int32

    @property
    def n(self) -> int:
        return int(len(self.off) - 1)

    @classmethod
    def of(cls, g) -> "OGraph":
        """Accepts any object with seq/seg_off/edge_src/edge_dst (or
        seq/off/src/dst) attributes, or an (labels, edges) pair."""
        if isinstance(g, OGraph):
            return g
        if isinstance(g, tuple):
            labels, edges = g
            seq = _u8("".join(labels))
            off = np.zeros(len(labels) + 1, dtype=np.int64)
            off[1:] = np.cumsum([len(s) for s in labels])
            e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
            return cls(seq, off, np.ascontiguousarray(e[:, 0]), np.ascontiguousarray(e[:, 1]))
        seq = getattr(g, "seq")
        off = getattr(g, "seg_off", None)
        if off is None:
            off = getattr(g, "off")
        src = getattr(g, "edge_src", None)
        if src is None:
            src = getattr(g, "src")
        dst = getattr(g, "edge_dst", None)
        if dst is None:
            dst = getattr(g, "dst")
        return cls(_u8(seq), np.ascontiguousarray(off, dtype=np.int64),
                   np.ascontiguousarray(src, dtype=np.int32), np.ascontiguousarray(dst, dtype=np.int32))

    def _args(self):
        return (self.n, _ptr(self.seq), _ptr(self.off), len(self.src), _ptr(self.src), _ptr(self.dst))


def dp_dense(g, q, v_s: int):
    """Eq. 1 dense.  Returns (d*, end_v, end_j, max_sweeps_per_row)."""
    lib = _load()
    G = OGraph.of(g)
    qq = _u8(q)
    out = np.zeros(4, dtype=np.int32)
    rc = lib.orc_dp_dense(*G._args(), _ptr(qq), len(qq), int(v_s), _ptr(out))
    if rc != 0:
        raise RuntimeError("orc_dp_dense failed")
    return int(out[0]), int(out[1]), int(out[2]), int(out[3])


def dp_dense_at(g, q, v_s: int, j0: int = 0, v_e: int = -1, j1: int = -1, wfree: bool = False):
    """Eq. 1 dense with the walk starting after the first j bases of v_s, j
    free in j0..j1 (j1 = -1: j = j0); extension form (v_e = -1: (d*, end_v,
    end_j)) or global form with end vertex v_e ((d, v_e, |v_e|), d = -1 when
    unreachable); wfree: the walk may end anywhere inside v_e ((d, v_e, j))."""
    lib = _load()
    G = OGraph.of(g)
    qq = _u8(q)
    out = np.zeros(4, dtype=np.int32)
    rc = lib.orc_dp_dense_at(*G._args(), _ptr(qq), len(qq), int(v_s), int(j0), int(j1), int(v_e), int(bool(wfree)),
                             _ptr(out))
    if rc != 0:
        raise RuntimeError("orc_dp_dense_at failed")
    return int(out[0]), int(out[1]), int(out[2])


def dp_dense_clip(g, q, v_s: int, e: int, j0: int = 0, j1: int = -1, v_e: int = -1, wfree: bool = False):
    """dp_dense_at with a free end gap of up to e query bases: the best over
    rows |q| - e .. |q| (ties: the largest row).  Returns (d, end_v, end_j,
    clip) with clip = query bases left unaligned; d = -1 when the global
    form's end vertex is unreachable."""
    lib = _load()
    G = OGraph.of(g)
    qq = _u8(q)
    out = np.zeros(4, dtype=np.int32)
    rc = lib.orc_dp_dense_clip(*G._args(), _ptr(qq), len(qq), int(v_s), int(j0), int(j1), int(v_e), int(bool(wfree)),
                               int(e), _ptr(out))
    if rc != 0:
        raise RuntimeError("orc_dp_dense_clip failed")
    return int(out[0]), int(out[1]), int(out[2]), int(out[3])


def dp_dense_global(g, q, v_s: int, v_e: int) -> int:
    """Eq. 1 dense, global form: H at (|q|, v_e, |v_e|), or -1 when v_e cannot
    be reached from v_s."""
    lib = _load()
    G = OGraph.of(g)
    qq = _u8(q)
    out = np.zeros(2, dtype=np.int32)
    rc = lib.orc_dp_dense_global(*G._args(), _ptr(qq), len(qq), int(v_s), int(v_e), _ptr(out))
    if rc != 0:
        raise RuntimeError("orc_dp_dense_global failed")
    return int(out[0])


def dp_capped(g, q, v_s: int, D: int):
    """Eq. 1 saturated at D+1.  Returns (d*, end_v, end_j) or (-1, -1, -1)
    when d* > D."""
    lib = _load()
    G = OGraph.of(g)
    qq = _u8(q)
    out = np.zeros(3, dtype=np.int32)
    rc = lib.orc_dp_capped(*G._args(), _ptr(qq), len(qq), int(v_s), int(D), _ptr(out))
    if rc != 0:
        raise RuntimeError("orc_dp_capped failed")
    return int(out[0]), int(out[1]), int(out[2])


def dp_batch(g, reads: np.ndarray, read_off: np.ndarray, v_start: np.ndarray,
             caps: np.ndarray, n_threads: int = 0) -> np.ndarray:
    """Many reads; caps[r] < 0 selects the dense form.  Returns an (n, 3)
    int32 array (d*, end_v, end_j); d* = -1 means saturated (> cap)."""
    lib = _load()
    G = OGraph.of(g)
    reads = _u8(reads)
    read_off = np.ascontiguousarray(read_off, dtype=np.int64)
    v_start = np.ascontiguousarray(v_start, dtype=np.int32)
    caps = np.ascontiguousarray(caps, dtype=np.int32)
    n = len(v_start)
    out = np.zeros((n, 3), dtype=np.int32)
    fails = lib.orc_dp_batch(*G._args(), n, _ptr(reads), _ptr(read_off), _ptr(v_start),
                             _ptr(caps), _ptr(out), int(n_threads))
    if fails:
        raise RuntimeError(f"orc_dp_batch: {fails} reads failed")
    return out


def num_threads() -> int:
    return int(_load().orc_num_threads())


def ed_global(a, b) -> int:
    lib = _load()
    aa, bb = _u8(a), _u8(b)
    return int(lib.orc_ed_global(_ptr(aa), len(aa), _ptr(bb), len(bb)))


def ed_banded(a, b, D: int) -> int:
    """Edit distance if <= D, else -1."""
    lib = _load()
    aa, bb = _u8(a), _u8(b)
    return int(lib.orc_ed_banded(_ptr(aa), len(aa), _ptr(bb), len(bb), int(D)))


def gwf(g, q, v_s: int, a_diff: int = 0, max_score: int = -1, counts_cap: int = 0, v_e: int = -1, j0: int = 0,
        j1: int = -1, e: int = 0, wfree: bool = False, entries_cap: int = 0):
    """Algorithms 1-4 in extension mode (v_e = -1) or in the global form with
    end vertex v_e (wfree: ending anywhere inside v_e); the walk starts after the first j bases of v_s, j free in
    j0..j1 (j1 = -1: j = j0); up to e trailing query bases may stay unaligned
    (`clip` in the result: how many did).  Returns a dict with dist, end_v, end_j, status (0 ok,
    1 max_score, 2 end vertex unreachable), work (sum |F_s|), diagonals,
    crossings and optionally the per-score |F_s| list; with entries_cap > 0
    also "entries", an (m, 5) int32 array of (score, v, k, offset, W~) for
    every entry of every extended wavefront (at most entries_cap rows)."""
    lib = _load()
    G = OGraph.of(g)
    qq = _u8(q)
    out = np.zeros(5, dtype=np.int32)
    work = np.zeros(3, dtype=np.int64)
    counts = np.zeros(max(counts_cap, 1), dtype=np.int32)
    ent = np.zeros((max(entries_cap, 1), 5), dtype=np.int32)
    ent_n = np.zeros(1, dtype=np.int64)
    rc = lib.orc_gwf(*G._args(), _ptr(qq), len(qq), int(v_s), int(j0), int(j1), int(v_e), int(bool(wfree)), int(e),
                     int(a_diff), int(max_score),
                     _ptr(out), _ptr(work), _ptr(counts) if counts_cap else None, int(counts_cap),
                     _ptr(ent) if entries_cap else None, int(entries_cap), _ptr(ent_n) if entries_cap else None)
    if rc != 0:
        raise RuntimeError("orc_gwf failed")
    res = dict(dist=int(out[0]), end_v=int(out[1]), end_j=int(out[2]), status=int(out[3]), clip=int(out[4]),
               work=int(work[0]), diagonals=int(work[1]), crossings=int(work[2]))
    if counts_cap:
        res["counts"] = counts[: min(counts_cap, max(res["dist"], 0) + 1)].tolist()
    if entries_cap:
        res["entries"] = ent[: min(int(ent_n[0]), entries_cap)].copy()
        res["entries_total"] = int(ent_n[0])
    return res


def spell_walk(g, walk, end_j: int) -> bytes:
    """sigma(v_1) ... sigma(v_n)[1..end_j] for a vertex walk (Section 2.1)."""
    G = OGraph.of(g)
    parts = []
    for idx, v in enumerate(walk):
        a, b = int(G.off[v]), int(G.off[v + 1])
        if idx == len(walk) - 1:
            b = a + int(end_j)
        parts.append(G.seq[a:b].tobytes())
    return b"".join(parts)


def is_walk(g, walk) -> bool:
    G = OGraph.of(g)
    es = set(zip(G.src.tolist(), G.dst.tolist()))
    return all((int(a), int(b)) in es for a, b in zip(walk[:-1], walk[1:]))
