"""Single-linkage dendrograms of minimum spanning trees on MI355X (gfx950).

Thin binding over ``libpandora.so`` (C ABI in ``include/pandora.h``): it only
checks and marshals torch tensors; every step of the method runs in the
library's HIP kernels.  PyTorch supplies device memory and the stream.

    ep, vp = dendrogram(u, v, w)             # one tree, device tensors
    ep, vp = dendrogram_batched(voff, u, v, w)  # a forest, tree-local ids

The library is not optional: importing this package raises if it has not
been built (``python -m paper_2401_06089_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpandora.so")

OK = 0
INVALID_ARG = 1
NOT_A_TREE = 2
NAN_WEIGHT = 3
OUT_OF_MEMORY = 4
HIP_ERROR = 5
BAD_VERTEX = 6


class PandoraError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pandora status {status}: {msg}")
        self.status = status


_lib = None


class Tuning(ctypes.Structure):
    """Mirror of pandora_tuning_t (speed knobs only; results never change)."""
    _fields_ = [("sync_free_max_edges", ctypes.c_int32), ("jump_steps", ctypes.c_int32),
                ("chain_digit_bits", ctypes.c_int32), ("sort_tile_cfg", ctypes.c_int32),
                ("persist_max_edges", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2401_06089_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.pandora_dendrogram.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    lib.pandora_dendrogram.restype = ctypes.c_int
    lib.pandora_dendrogram_noalloc.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    lib.pandora_dendrogram_noalloc.restype = ctypes.c_int
    lib.pandora_dendrogram_batched.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp]
    lib.pandora_dendrogram_batched.restype = ctypes.c_int
    lib.pandora_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
    lib.pandora_workspace_bytes.restype = ctypes.c_size_t
    lib.pandora_last_stats.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.pandora_last_stats.restype = ctypes.c_int
    lib.pandora_release_workspaces.argtypes = []
    lib.pandora_release_workspaces.restype = None
    lib.pandora_profile_enable.argtypes = [ctypes.c_uint32]
    lib.pandora_profile_enable.restype = ctypes.c_int
    lib.pandora_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.pandora_profile_read.restype = ctypes.c_int
    lib.pandora_profile_name.argtypes = [ctypes.c_int]
    lib.pandora_profile_name.restype = ctypes.c_char_p
    lib.pandora_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.pandora_set_tuning.restype = ctypes.c_int
    lib.pandora_set_thread_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.pandora_set_thread_tuning.restype = ctypes.c_int
    lib.pandora_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.pandora_get_tuning.restype = ctypes.c_int
    lib.pandora_graph_create.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_void_p)]
    lib.pandora_graph_create.restype = ctypes.c_int
    lib.pandora_graph_create_batched.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp,
                                                 ctypes.POINTER(ctypes.c_void_p)]
    lib.pandora_graph_create_batched.restype = ctypes.c_int
    lib.pandora_graph_launch.argtypes = [vp, vp]
    lib.pandora_graph_launch.restype = ctypes.c_int
    lib.pandora_graph_destroy.argtypes = [vp]
    lib.pandora_graph_destroy.restype = None
    lib.pandora_status_string.argtypes = [ctypes.c_int]
    lib.pandora_status_string.restype = ctypes.c_char_p
    lib.pandora_dendrogram_async.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    lib.pandora_dendrogram_async.restype = ctypes.c_int
    lib.pandora_dendrogram_batched_async.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp]
    lib.pandora_dendrogram_batched_async.restype = ctypes.c_int
    lib.pandora_stream_status.argtypes = [vp]
    lib.pandora_stream_status.restype = ctypes.c_int
    lib.pandora_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
    lib.pandora_set_workspace.restype = ctypes.c_int
    lib.pandora_flat_clusters.argtypes = [ctypes.c_int64, vp, vp, vp, ctypes.c_int32, vp, vp, vp, vp,
                                          ctypes.POINTER(ctypes.c_int64), vp]
    lib.pandora_flat_clusters.restype = ctypes.c_int
    lib.pandora_emst.argtypes = [ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_int32, vp, vp, vp, vp, vp]
    lib.pandora_emst.restype = ctypes.c_int
    lib.pandora_flat_clusters_workspace_bytes.argtypes = [ctypes.c_int64]
    lib.pandora_flat_clusters_workspace_bytes.restype = ctypes.c_size_t
    _lib = lib
    return lib


def library() -> ctypes.CDLL:
    """The loaded ctypes handle of libpandora.so."""
    return _load()


def status_string(status: int) -> str:
    return _load().pandora_status_string(int(status)).decode()


def _check(status: int):
    if status != OK:
        raise PandoraError(status, status_string(status))


def _dptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _as_dev(t, dtype, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError("inputs must be device tensors")
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return t.contiguous()


# Per-call tuning: a function edges -> tuning dict (or None), installed by
# autotune.install.  By default the table shipped for this GPU architecture is
# used when there is one (set PANDORA_AUTOTUNE=0 to disable).
_tuning_hook = None
_tuning_checked = False


def _set_tuning_hook(fn) -> None:
    global _tuning_hook, _tuning_checked
    _tuning_hook = fn
    _tuning_checked = True


def _apply_tuning(edges: int) -> None:
    global _tuning_checked
    if not _tuning_checked:
        _tuning_checked = True
        if os.environ.get("PANDORA_AUTOTUNE", "1") != "0":
            from . import autotune
            table = autotune.load()
            if table is not None:
                autotune.install(table)
    if _tuning_hook is not None:
        t = _tuning_hook(int(edges))
        set_thread_tuning(t)


def dendrogram_into(n: int, u, v, w, edge_parent, vertex_parent, stream=None) -> int:
    """Raw call: writes into preallocated int32 device tensors; returns the status."""
    _apply_tuning(int(n) - 1)
    return _load().pandora_dendrogram(int(n), _dptr(u), _dptr(v), _dptr(w), _dptr(edge_parent),
                                      _dptr(vertex_parent), _stream_handle(stream))


def dendrogram(u: torch.Tensor, v: torch.Tensor, w: torch.Tensor,
               n: Optional[int] = None, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Dendrogram of one tree with n = len(w) + 1 vertices.

    u, v: int32 device tensors of edge endpoints; w: float32 weights.
    Returns (edge_parent[n-1], vertex_parent[n]) as int32 device tensors.
    """
    m = w.numel()
    if n is None:
        n = m + 1
    if n != m + 1 or u.numel() != m or v.numel() != m:
        raise ValueError("a tree with n vertices has n-1 edges")
    dev = w.device
    u = _as_dev(u, torch.int32, dev)
    v = _as_dev(v, torch.int32, dev)
    w = _as_dev(w, torch.float32, dev)
    with torch.cuda.device(dev):
        ep = torch.empty(m, dtype=torch.int32, device=dev)
        vp = torch.empty(n, dtype=torch.int32, device=dev)
        _check(dendrogram_into(n, u, v, w, ep, vp, stream))
    return ep, vp


# Largest tree pandora_dendrogram_noalloc accepts (its fixed scratch array).
NOALLOC_SCRATCH_BYTES = 64 << 20
NOALLOC_MAX_VERTICES = 798594


def dendrogram_noalloc_into(n: int, u, v, w, edge_parent, vertex_parent, stream=None) -> int:
    """Raw call of the entry point that allocates nothing (its scratch is a
    fixed device array; trees above NOALLOC_MAX_VERTICES give OUT_OF_MEMORY).
    Writes into preallocated int32 device tensors; returns the status."""
    _apply_tuning(int(n) - 1)
    return _load().pandora_dendrogram_noalloc(int(n), _dptr(u), _dptr(v), _dptr(w), _dptr(edge_parent),
                                              _dptr(vertex_parent), _stream_handle(stream))


def flat_clusters(u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, min_cluster_size: int,
                  n: Optional[int] = None, stream=None):
    """HDBSCAN* flat clusters (excess of mass) of one tree with n = len(w) + 1
    vertices; every weight must be > 0.

    Returns (labels[n] int32, stability[k] float64, edge_parent[n-1],
    vertex_parent[n]) as device tensors: labels number the k chosen clusters
    by their smallest vertex id, -1 is noise."""
    m = w.numel()
    if n is None:
        n = m + 1
    if n != m + 1 or u.numel() != m or v.numel() != m:
        raise ValueError("a tree with n vertices has n-1 edges")
    mcs = int(min_cluster_size)
    dev = w.device
    u = _as_dev(u, torch.int32, dev)
    v = _as_dev(v, torch.int32, dev)
    w = _as_dev(w, torch.float32, dev)
    with torch.cuda.device(dev):
        ep = torch.empty(m, dtype=torch.int32, device=dev)
        vp = torch.empty(n, dtype=torch.int32, device=dev)
        labels = torch.empty(n, dtype=torch.int32, device=dev)
        stab = torch.empty(max(n // max(mcs, 1), 1), dtype=torch.float64, device=dev)
        k = ctypes.c_int64(0)
        _apply_tuning(m)
        st = _load().pandora_flat_clusters(int(n), _dptr(u), _dptr(v), _dptr(w), mcs, _dptr(ep), _dptr(vp),
                                           _dptr(labels), _dptr(stab), ctypes.byref(k), _stream_handle(stream))
        _check(st)
    return labels, stab[:k.value], ep, vp


def flat_clusters_into(n: int, u, v, w, min_cluster_size: int, edge_parent, vertex_parent, labels,
                       stability=None, stream=None) -> Tuple[int, int]:
    """Raw call into preallocated device tensors; returns (status, number of clusters)."""
    _apply_tuning(int(n) - 1)
    k = ctypes.c_int64(0)
    st = _load().pandora_flat_clusters(int(n), _dptr(u), _dptr(v), _dptr(w), int(min_cluster_size),
                                       _dptr(edge_parent), _dptr(vertex_parent), _dptr(labels),
                                       _dptr(stability), ctypes.byref(k), _stream_handle(stream))
    return st, int(k.value)


def emst(points: torch.Tensor, min_pts: int, stream=None):
    """Mutual-reachability MST of an (n, dim) float32 device tensor of points
    (dim <= 4).  Returns (u, v, w64, w32): the n-1 edges in ascending (weight,
    u, v) order, u < v, with fp64 and fp32 weights."""
    if points.dim() != 2:
        raise ValueError("points must be an (n, dim) tensor")
    n, dim = points.shape
    dev = points.device
    p = _as_dev(points, torch.float32, dev)
    with torch.cuda.device(dev):
        m = max(n - 1, 0)
        u = torch.empty(m, dtype=torch.int32, device=dev)
        v = torch.empty(m, dtype=torch.int32, device=dev)
        w64 = torch.empty(m, dtype=torch.float64, device=dev)
        w32 = torch.empty(m, dtype=torch.float32, device=dev)
        _check(_load().pandora_emst(int(n), int(dim), _dptr(p), int(min_pts), _dptr(u), _dptr(v), _dptr(w64),
                                    _dptr(w32), _stream_handle(stream)))
    return u, v, w64, w32


def hdbscan(points: torch.Tensor, min_pts: int, min_cluster_size: int, stream=None):
    """HDBSCAN* end to end on the GPU: the mutual-reachability MST, its
    dendrogram and the excess-of-mass flat clusters.  Returns (labels[n],
    stability[k]) as device tensors (labels numbered by smallest point index,
    -1 = noise).

    Clouds where min_pts or more points coincide are refused (INVALID_ARG):
    their mutual-reachability distance is 0, where the density level
    lambda = 1/w of the flat-cluster step is not finite."""
    u, v, _, w32 = emst(points, min_pts, stream=stream)
    try:
        labels, stab, _, _ = flat_clusters(u, v, w32, min_cluster_size, n=points.shape[0], stream=stream)
    except PandoraError as e:
        if e.status == INVALID_ARG and int(min_cluster_size) >= 2:
            raise PandoraError(INVALID_ARG, "min_pts or more points coincide (mutual-reachability distance 0, "
                                            "lambda = 1/w not finite): flat clusters need every MST weight > 0") from e
        raise
    return labels, stab


def flat_clusters_workspace_bytes(n: int) -> int:
    return int(_load().pandora_flat_clusters_workspace_bytes(int(n)))


def dendrogram_batched(voff, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor,
                       stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Dendrograms of B trees at once.  voff: host int64 offsets (B+1, numpy or
    CPU tensor); tree b owns vertices [voff[b], voff[b+1]) and edges
    [voff[b]-b, voff[b+1]-b-1).  u, v and the outputs use tree-local ids."""
    voff_t = torch.as_tensor(voff, dtype=torch.int64).cpu().contiguous()
    B = voff_t.numel() - 1
    if B < 1:
        raise ValueError("need at least one tree")
    N = int(voff_t[-1])
    M = N - B
    if w.numel() != M or u.numel() != M or v.numel() != M:
        raise ValueError("edge arrays must hold voff[-1] - B entries")
    dev = w.device
    u = _as_dev(u, torch.int32, dev)
    v = _as_dev(v, torch.int32, dev)
    w = _as_dev(w, torch.float32, dev)
    with torch.cuda.device(dev):
        ep = torch.empty(M, dtype=torch.int32, device=dev)
        vp = torch.empty(N, dtype=torch.int32, device=dev)
        _apply_tuning(M)
        st = _load().pandora_dendrogram_batched(
            B, ctypes.c_void_p(voff_t.data_ptr()), _dptr(u), _dptr(v), _dptr(w), _dptr(ep), _dptr(vp),
            _stream_handle(stream))
        _check(st)
    return ep, vp


def _hold_for(stream, dev, *tensors):
    """The caching allocator may reuse a tensor's memory as soon as its last
    reference is gone, judged by the stream it was allocated on.  A
    stream-ordered call reads and writes later, on `stream`: tie every tensor
    it uses to that stream so that no memory is reused before it has run."""
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    for t in tensors:
        if t is not None and t.numel() > 0:
            t.record_stream(s)


def dendrogram_async(u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, n: Optional[int] = None,
                     stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Stream-ordered dendrogram: enqueues the call and returns at once.

    The outputs are valid once the stream has passed the call; input errors
    are reported by stream_status(stream).  Every tensor the call uses is tied
    to the stream, so the caller may drop its references right away."""
    m = w.numel()
    if n is None:
        n = m + 1
    if n != m + 1 or u.numel() != m or v.numel() != m:
        raise ValueError("a tree with n vertices has n-1 edges")
    dev = w.device
    u = _as_dev(u, torch.int32, dev)
    v = _as_dev(v, torch.int32, dev)
    w = _as_dev(w, torch.float32, dev)
    with torch.cuda.device(dev):
        ep = torch.empty(m, dtype=torch.int32, device=dev)
        vp = torch.empty(n, dtype=torch.int32, device=dev)
        _apply_tuning(m)
        _check(_load().pandora_dendrogram_async(int(n), _dptr(u), _dptr(v), _dptr(w), _dptr(ep), _dptr(vp),
                                                _stream_handle(stream)))
        _hold_for(stream, dev, u, v, w, ep, vp)
    return ep, vp


def dendrogram_batched_async(voff, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor,
                             stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Stream-ordered dendrogram_batched (see dendrogram_async)."""
    voff_t = torch.as_tensor(voff, dtype=torch.int64).cpu().contiguous()
    B = voff_t.numel() - 1
    if B < 1:
        raise ValueError("need at least one tree")
    N = int(voff_t[-1])
    M = N - B
    if w.numel() != M or u.numel() != M or v.numel() != M:
        raise ValueError("edge arrays must hold voff[-1] - B entries")
    dev = w.device
    u = _as_dev(u, torch.int32, dev)
    v = _as_dev(v, torch.int32, dev)
    w = _as_dev(w, torch.float32, dev)
    with torch.cuda.device(dev):
        ep = torch.empty(M, dtype=torch.int32, device=dev)
        vp = torch.empty(N, dtype=torch.int32, device=dev)
        _apply_tuning(M)
        _check(_load().pandora_dendrogram_batched_async(
            B, ctypes.c_void_p(voff_t.data_ptr()), _dptr(u), _dptr(v), _dptr(w), _dptr(ep), _dptr(vp),
            _stream_handle(stream)))
        _hold_for(stream, dev, u, v, w, ep, vp)
    return ep, vp


def stream_status(stream=None) -> int:
    """Waits for the stream; returns (and clears) the deferred status of its
    stream-ordered calls."""
    return int(_load().pandora_stream_status(_stream_handle(stream)))


def set_workspace(buffer: Optional[torch.Tensor], stream=None) -> None:
    """Caller-owned scratch for calls on `stream` (a device tensor of at least
    workspace_bytes(...) bytes, 256-byte aligned), or None to return to
    library-owned scratch.  Keep the tensor alive while it is installed."""
    if buffer is None:
        _check(_load().pandora_set_workspace(_stream_handle(stream), None, 0))
        return
    if buffer.device.type != "cuda" or not buffer.is_contiguous():
        raise ValueError("the workspace must be a contiguous device tensor")
    nbytes = buffer.numel() * buffer.element_size()
    _check(_load().pandora_set_workspace(_stream_handle(stream), ctypes.c_void_p(buffer.data_ptr()), nbytes))


def workspace_bytes(n_total_vertices: int, trees: int = 1) -> int:
    return int(_load().pandora_workspace_bytes(int(n_total_vertices), int(trees)))


def last_stats() -> dict:
    buf = (ctypes.c_int64 * 7)()
    k = _load().pandora_last_stats(buf, 7)
    names = ["levels", "sum_level_edges", "jump_launches", "tail_levels", "tail_entry_edges", "sync_free",
             "persistent"]
    return {names[i]: int(buf[i]) for i in range(k)}


def get_tuning() -> dict:
    t = Tuning()
    _check(_load().pandora_get_tuning(ctypes.byref(t)))
    return t.as_dict()


def set_tuning(**kw) -> dict:
    """Update process-wide tuning knobs; returns the previous values.

    Explicit knobs win: this also turns off the autotuned table for the rest
    of the process (``autotune.install`` brings a table back)."""
    old = get_tuning()
    t = Tuning(**{**old, **kw})
    _check(_load().pandora_set_tuning(ctypes.byref(t)))
    _set_tuning_hook(None)
    set_thread_tuning(None)
    return old


def set_thread_tuning(tuning: Optional[dict]) -> None:
    """Tuning for calls made by this thread only (None: use the process-wide one)."""
    if tuning is None:
        _check(_load().pandora_set_thread_tuning(None))
    else:
        _check(_load().pandora_set_thread_tuning(ctypes.byref(Tuning(**tuning))))


def release_workspaces():
    _load().pandora_release_workspaces()


PROFILE_ALL = 0xFFFFFFFF


def profile_enable(mask: int = PROFILE_ALL) -> None:
    """Clear the per-kernel profiler and time the kernel kinds in `mask`
    (bit k = kind k; 0 turns profiling off)."""
    _load().pandora_profile_enable(int(mask) & 0xFFFFFFFF)


def profile_read() -> dict:
    """{kind name: {"ms", "bytes", "launches"}} accumulated since profile_enable."""
    lib = _load()
    cap = 32
    ms = (ctypes.c_double * cap)()
    by = (ctypes.c_double * cap)()
    ln = (ctypes.c_int64 * cap)()
    k = lib.pandora_profile_read(ms, by, ln, cap)
    return {lib.pandora_profile_name(i).decode(): {"kind": i, "ms": ms[i], "bytes": by[i], "launches": int(ln[i])}
            for i in range(k)}


class Graph:
    """A dendrogram call captured once into a HIP graph and replayed.

    The inputs (device tensors u, v, w; host offsets voff for a forest) are
    bound at creation; replace their contents in place and call launch() to
    build the dendrogram of the new data.  Outputs live in edge_parent and
    vertex_parent.  Replays must not overlap.
    """

    def __init__(self, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, n: Optional[int] = None,
                 voff=None):
        lib = _load()
        self._h = ctypes.c_void_p()
        dev = w.device
        self.u = _as_dev(u, torch.int32, dev)
        self.v = _as_dev(v, torch.int32, dev)
        self.w = _as_dev(w, torch.float32, dev)
        m = w.numel()
        _apply_tuning(m)
        with torch.cuda.device(dev):
            if voff is None:
                n = m + 1 if n is None else int(n)
                if n != m + 1:
                    raise ValueError("a tree with n vertices has n-1 edges")
                self.edge_parent = torch.empty(m, dtype=torch.int32, device=dev)
                self.vertex_parent = torch.empty(n, dtype=torch.int32, device=dev)
                st = lib.pandora_graph_create(n, _dptr(self.u), _dptr(self.v), _dptr(self.w),
                                              _dptr(self.edge_parent), _dptr(self.vertex_parent),
                                              ctypes.byref(self._h))
            else:
                self.voff = torch.as_tensor(voff, dtype=torch.int64).cpu().contiguous()
                B = self.voff.numel() - 1
                N = int(self.voff[-1])
                self.edge_parent = torch.empty(N - B, dtype=torch.int32, device=dev)
                self.vertex_parent = torch.empty(N, dtype=torch.int32, device=dev)
                st = lib.pandora_graph_create_batched(
                    B, ctypes.c_void_p(self.voff.data_ptr()), _dptr(self.u), _dptr(self.v), _dptr(self.w),
                    _dptr(self.edge_parent), _dptr(self.vertex_parent), ctypes.byref(self._h))
        _check(st)

    def launch(self, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
        _check(_load().pandora_graph_launch(self._h, _stream_handle(stream)))
        return self.edge_parent, self.vertex_parent

    def close(self):
        if self._h:
            _load().pandora_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
