"""The C ABI without a GPU: libpandora.so loads, exports exactly the functions
include/pandora.h declares, and its host-side entry points behave as the
header says (argument errors come back before any launch, tuning knobs are
validated and scoped per thread, workspace sizes follow the level bounds).
No call here reaches a kernel."""
import ctypes
import os
import re
import subprocess
import threading

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pandora.h")
LIB = os.path.join(ROOT, "paper_2401_06089_amd", "libpandora.so")

OK, INVALID_ARG = 0, 1


class Tuning(ctypes.Structure):
    _fields_ = [("sync_free_max_edges", ctypes.c_int32), ("jump_steps", ctypes.c_int32),
                ("chain_digit_bits", ctypes.c_int32), ("sort_tile_cfg", ctypes.c_int32),
                ("persist_max_edges", ctypes.c_int32)]


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2401_06089_amd import build
        build.build()
    L = ctypes.CDLL(LIB)
    L.pandora_status_string.restype = ctypes.c_char_p
    L.pandora_profile_name.restype = ctypes.c_char_p
    L.pandora_workspace_bytes.restype = ctypes.c_size_t
    L.pandora_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
    L.pandora_dendrogram.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 6
    L.pandora_dendrogram_batched.argtypes = [ctypes.c_int32] + [ctypes.c_void_p] * 7
    L.pandora_graph_create.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 6
    L.pandora_graph_create_batched.argtypes = [ctypes.c_int32] + [ctypes.c_void_p] * 7
    L.pandora_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.pandora_last_stats.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.pandora_dendrogram_async.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 6
    L.pandora_dendrogram_noalloc.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 6
    L.pandora_dendrogram_batched_async.argtypes = [ctypes.c_int32] + [ctypes.c_void_p] * 7
    L.pandora_set_workspace.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    L.pandora_flat_clusters.argtypes = ([ctypes.c_int64] + [ctypes.c_void_p] * 3 + [ctypes.c_int32]
                                        + [ctypes.c_void_p] * 6)
    L.pandora_emst.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 5
    L.pandora_flat_clusters_workspace_bytes.restype = ctypes.c_size_t
    L.pandora_flat_clusters_workspace_bytes.argtypes = [ctypes.c_int64]
    yield L
    L.pandora_set_thread_tuning(None)


def declared_functions():
    text = open(HEADER).read()
    return set(re.findall(r"PANDORA_API\s+[\w\s\*]*?\b(pandora_\w+)\s*\(", text))


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("pandora_dendrogram", "pandora_dendrogram_batched", "pandora_workspace_bytes",
                 "pandora_graph_create", "pandora_graph_launch", "pandora_set_tuning"):
        assert must in names
    for must in ("pandora_dendrogram_async", "pandora_dendrogram_batched_async", "pandora_stream_status",
                 "pandora_set_workspace", "pandora_flat_clusters", "pandora_flat_clusters_workspace_bytes",
                 "pandora_emst"):
        assert must in names
    assert "pandora_dendrogram_noalloc" in names
    assert len(names) == 24


def test_library_exports_exactly_the_declared_functions(lib):
    names = declared_functions()
    for nm in names:
        assert hasattr(lib, nm), f"{nm} declared but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.split() and ln.split()[-1].startswith("pandora_")}
    assert exported == names
    # internal launchers stay hidden
    assert "launch_" not in out


def test_status_strings(lib):
    seen = set()
    for code in range(7):
        s = lib.pandora_status_string(code).decode()
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 7
    assert lib.pandora_status_string(99).decode() == "unknown status"


def test_argument_errors_come_back_before_any_launch(lib):
    d = ctypes.c_void_p(16)   # never dereferenced: every call below fails validation first
    assert lib.pandora_dendrogram(0, d, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram(-5, d, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram(2**31, d, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram(1_200_000_000, d, d, d, d, d, None) == INVALID_ARG   # ids would not fit
    assert lib.pandora_dendrogram(10, None, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram(10, d, d, d, None, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram(10, d, d, d, d, None, None) == INVALID_ARG
    # the entry point with a fixed scratch array: the same checks, and trees
    # beyond that array come back as OUT_OF_MEMORY before any launch
    assert lib.pandora_dendrogram_noalloc(0, d, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram_noalloc(10, None, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram_noalloc(10, d, d, d, d, None, None) == INVALID_ARG
    assert lib.pandora_dendrogram_noalloc(1_200_000_000, d, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram_noalloc(798_595, d, d, d, d, d, None) == 4   # OUT_OF_MEMORY
    assert lib.pandora_dendrogram_noalloc(50_000_000, d, d, d, d, d, None) == 4

    def voff(*xs):
        return (ctypes.c_int64 * len(xs))(*xs)
    assert lib.pandora_dendrogram_batched(0, voff(0), d, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram_batched(2, None, d, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram_batched(2, voff(1, 3, 5), d, d, d, d, d, None) == INVALID_ARG   # voff[0] != 0
    assert lib.pandora_dendrogram_batched(2, voff(0, 3, 3), d, d, d, d, d, None) == INVALID_ARG   # empty tree
    assert lib.pandora_dendrogram_batched(2, voff(0, 4, 2), d, d, d, d, d, None) == INVALID_ARG   # decreasing
    assert lib.pandora_dendrogram_batched(1, voff(0, 2**31), d, d, d, d, d, None) == INVALID_ARG  # too many vertices
    assert lib.pandora_dendrogram_batched(2, voff(0, 3, 5), None, d, d, d, d, None) == INVALID_ARG

    g = ctypes.c_void_p()
    assert lib.pandora_graph_create(10, d, d, d, d, d, None) == INVALID_ARG            # no out pointer
    assert lib.pandora_graph_create(0, d, d, d, d, d, ctypes.byref(g)) == INVALID_ARG
    assert lib.pandora_graph_create_batched(2, voff(0, 4, 2), d, d, d, d, d, ctypes.byref(g)) == INVALID_ARG
    assert lib.pandora_graph_launch(None, None) == INVALID_ARG
    lib.pandora_graph_destroy(None)   # a no-op
    assert lib.pandora_last_stats(None, 6) == -INVALID_ARG
    # the stream-ordered variants validate the same way, before touching the device
    assert lib.pandora_dendrogram_async(0, d, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram_async(10, d, None, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram_batched_async(2, voff(0, 4, 2), d, d, d, d, d, None) == INVALID_ARG
    assert lib.pandora_dendrogram_batched_async(2, voff(0, 3, 5), d, d, d, None, d, None) == INVALID_ARG
    # caller scratch must be 256-byte aligned and non-empty
    assert lib.pandora_set_workspace(None, ctypes.c_void_p(4096 + 8), 1 << 20) == INVALID_ARG
    assert lib.pandora_set_workspace(None, ctypes.c_void_p(4096), 0) == INVALID_ARG
    # flat clusters: sizes, minimum cluster size and required pointers
    k = ctypes.c_int64(-1)
    kp = ctypes.cast(ctypes.byref(k), ctypes.c_void_p)
    assert lib.pandora_flat_clusters(0, d, d, d, 5, d, d, d, None, kp, None) == INVALID_ARG
    assert lib.pandora_flat_clusters(10, d, d, d, 1, d, d, d, None, kp, None) == INVALID_ARG
    assert lib.pandora_flat_clusters(10, d, d, d, 5, d, d, None, None, kp, None) == INVALID_ARG
    assert lib.pandora_flat_clusters(10, d, None, d, 5, d, d, d, None, kp, None) == INVALID_ARG
    assert lib.pandora_flat_clusters(10, d, d, d, 5, None, d, d, None, kp, None) == INVALID_ARG
    assert lib.pandora_flat_clusters(1_200_000_000, d, d, d, 5, d, d, d, None, kp, None) == INVALID_ARG
    assert k.value == -1
    # point clouds: sizes, dimension, min_pts and required pointers
    assert lib.pandora_emst(0, 2, d, 2, d, d, None, d, None) == INVALID_ARG
    assert lib.pandora_emst(10, 0, d, 2, d, d, None, d, None) == INVALID_ARG
    assert lib.pandora_emst(10, 5, d, 2, d, d, None, d, None) == INVALID_ARG
    assert lib.pandora_emst(10, 2, d, 0, d, d, None, d, None) == INVALID_ARG
    assert lib.pandora_emst(10, 2, d, 11, d, d, None, d, None) == INVALID_ARG   # more than n
    assert lib.pandora_emst(100, 2, d, 33, d, d, None, d, None) == INVALID_ARG
    assert lib.pandora_emst(10, 2, None, 2, d, d, None, d, None) == INVALID_ARG
    assert lib.pandora_emst(10, 2, d, 2, d, d, None, None, None) == INVALID_ARG
    assert lib.pandora_emst((1 << 24) + 1, 2, d, 2, d, d, None, d, None) == INVALID_ARG


def test_tuning_validation_and_thread_scope(lib):
    old = Tuning()
    assert lib.pandora_get_tuning(ctypes.byref(old)) == OK
    try:
        for bad in (dict(jump_steps=0), dict(jump_steps=5000), dict(chain_digit_bits=7),
                    dict(sort_tile_cfg=4), dict(sort_tile_cfg=-1), dict(sync_free_max_edges=-1),
                    dict(persist_max_edges=-1)):
            t = Tuning(0, 16, 0, 3, 0)
            for k, v in bad.items():
                setattr(t, k, v)
            assert lib.pandora_set_tuning(ctypes.byref(t)) == INVALID_ARG, bad
            assert lib.pandora_set_thread_tuning(ctypes.byref(t)) == INVALID_ARG, bad
        assert lib.pandora_set_tuning(None) == INVALID_ARG

        glob = Tuning(1000, 8, 9, 1, 5000)
        assert lib.pandora_set_tuning(ctypes.byref(glob)) == OK
        mine = Tuning(0, 32, 8, 2, 0)
        assert lib.pandora_set_thread_tuning(ctypes.byref(mine)) == OK
        got = Tuning()
        lib.pandora_get_tuning(ctypes.byref(got))
        assert (got.jump_steps, got.sort_tile_cfg) == (32, 2)

        seen = {}

        def other():
            t = Tuning()
            lib.pandora_get_tuning(ctypes.byref(t))
            seen["t"] = (t.sync_free_max_edges, t.jump_steps, t.chain_digit_bits, t.sort_tile_cfg,
                         t.persist_max_edges)
        th = threading.Thread(target=other)
        th.start()
        th.join()
        assert seen["t"] == (1000, 8, 9, 1, 5000)       # another thread sees the process-wide knobs

        assert lib.pandora_set_thread_tuning(None) == OK
        lib.pandora_get_tuning(ctypes.byref(got))
        assert (got.jump_steps, got.sort_tile_cfg) == (8, 1)
    finally:
        lib.pandora_set_thread_tuning(None)
        lib.pandora_set_tuning(ctypes.byref(old))


def test_workspace_bytes_follow_the_level_bounds(lib):
    assert lib.pandora_workspace_bytes(0, 1) == 0
    assert lib.pandora_workspace_bytes(5, 0) == 0
    assert lib.pandora_workspace_bytes(3, 4) == 0            # fewer vertices than trees
    assert lib.pandora_workspace_bytes(1, 1) == 0            # no edges, nothing to sort
    assert lib.pandora_workspace_bytes(7, 7) == 0
    assert lib.pandora_workspace_bytes(2**31, 1) == 0
    # the level tables' vertex ids must fit int32 (about 2n of them)
    assert lib.pandora_workspace_bytes(1_073_741_000, 1) > 0
    assert lib.pandora_workspace_bytes(1_073_742_000, 1) == 0
    assert lib.pandora_workspace_bytes(2**31 - 1, 1) == 0
    sizes = [lib.pandora_workspace_bytes(n, 1) for n in (10, 1000, 10**5, 10**6, 10**7)]
    assert all(a < b for a, b in zip(sizes, sizes[1:]))
    per_edge = lib.pandora_workspace_bytes(10**7, 1) / (10**7 - 1)
    assert 60 <= per_edge <= 160                             # ~90 B per edge plus fixed blocks
    # a forest with the same vertex count needs about the same space
    f = lib.pandora_workspace_bytes(10**6, 1000)
    t = lib.pandora_workspace_bytes(10**6, 1)
    assert 0.9 * t <= f <= 1.2 * t
    # flat clusters: the dendrogram's workspace plus about 245 bytes per edge (per-edge arrays,
    # and cluster-tree arrays and 104-byte exact stability accumulators sized for the most
    # clusters any minimum cluster size allows)
    assert lib.pandora_flat_clusters_workspace_bytes(1) == 0
    assert lib.pandora_flat_clusters_workspace_bytes(1_073_742_000) == 0
    extra = lib.pandora_flat_clusters_workspace_bytes(10**7) - lib.pandora_workspace_bytes(10**7, 1)
    assert 220 <= extra / (10**7 - 1) <= 270


def test_profile_kinds(lib):
    n = lib.pandora_profile_enable(0)
    assert n >= 10
    names = [lib.pandora_profile_name(k).decode() for k in range(n)]
    assert all(names) and len(set(names)) == n
    assert lib.pandora_profile_name(n).decode() == ""
    ms = (ctypes.c_double * n)()
    assert lib.pandora_profile_read(ms, None, None, n) == n
    assert all(x == 0 for x in ms)


def test_explicit_tuning_turns_the_table_off():
    import paper_2401_06089_amd as pd
    from paper_2401_06089_amd import autotune
    table = {"arch": None, "buckets": [{"max_edges": 2**31 - 1, "tuning": dict(
        sync_free_max_edges=0, jump_steps=4, chain_digit_bits=8, sort_tile_cfg=0, persist_max_edges=0)}]}
    old = pd.get_tuning()
    try:
        autotune.install(table)
        pd._apply_tuning(1000)
        assert pd.get_tuning()["jump_steps"] == 4      # the table's entry, on this thread
        pd.set_tuning(jump_steps=24)
        pd._apply_tuning(1000)
        assert pd.get_tuning()["jump_steps"] == 24     # explicit knobs win from now on
    finally:
        autotune.install(None)
        pd.set_thread_tuning(None)
        pd.set_tuning(**old)
