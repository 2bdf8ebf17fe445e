"""Thin ctypes binding over libkz.so (the C ABI in include/kz.h).

Argument marshalling only: every step of kernelization runs in the HIP
library.  PyTorch supplies device memory and the stream.  If the library is
not built, importing this module raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # loads the HIP runtime first, so libkz.so shares torch's runtime and streams

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkz.so")

KZ_OK, KZ_EINVAL, KZ_ECOLOUR, KZ_EILLEGAL, KZ_EASYM, KZ_ESELFLOOP = 0, -1, -2, -3, -4, -5
KZ_EWORKSPACE, KZ_ENOMEM, KZ_EHIP, KZ_EAGAIN = -6, -7, -8, -9
KZ_DENSE_U8, KZ_BITSET_U64, KZ_CSR = 0, 1, 2

EXPORTED = ("kz_create", "kz_destroy", "kz_strerror", "kz_workspace_bytes", "kz_kernelize", "kz_kernelize_async",
            "kz_profile_enable", "kz_profile_read", "kz_batch_workspace_bytes", "kz_kernelize_batch",
            "kz_batch_autotune", "kz_batch_set_config", "kz_batch_get_config", "kz_gen_bitset",
            "kz_server_fixed_bytes", "kz_server_request_bytes", "kz_server_create", "kz_server_submit",
            "kz_server_progress", "kz_server_poll", "kz_server_destroy", "kz_server_configure", "kz_server_done", "kz_set_edge_path", "kz_colour_workspace_bytes", "kz_colour_jp",
            "kz_kernelize_noalloc", "kz_dom_workspace_bytes", "kz_dominance", "kz_clique_workspace_bytes",
            "kz_find_clique", "kz_struction_workspace_bytes", "kz_struction")
NOALLOC_SCRATCH_BYTES = 64 << 20   # KZ_NOALLOC_SCRATCH_BYTES
KZ_EDGE_BITSET, KZ_EDGE_MFMA_I8 = 0, 1
KZ_EAGAIN = -9
KZ_ETOOLARGE = -10
KERNELS = ("setup", "pack", "vertex", "edge", "apply", "unpack")


class kz_graph(C.Structure):
    _fields_ = [("format", C.c_int32), ("n", C.c_int32), ("adj", C.c_void_p), ("rows", C.c_void_p),
                ("row_words", C.c_int32), ("reserved0", C.c_int32), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("nnz", C.c_int64)]


class kz_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("rounds", C.c_int32), ("equals_input", C.c_int32),
                ("passes", C.c_int32), ("surviving_vertices", C.c_int64),
                ("surviving_edges", C.c_int64), ("input_edges", C.c_int64), ("edge_tests", C.c_int64)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class kz_dom_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("sweeps", C.c_int32), ("deleted_vertices", C.c_int64),
                ("deleted_edges", C.c_int64), ("input_edges", C.c_int64), ("events", C.c_int64),
                ("scans", C.c_int64)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


KZ_DOM_VERTEX, KZ_DOM_EDGE = 0, 1


class kz_struction_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("row_words", C.c_int32), ("nodes", C.c_int64), ("a_nodes", C.c_int64),
                ("c_nodes", C.c_int64), ("input_edges", C.c_int64)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class kz_clique_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("found", C.c_int32), ("nodes", C.c_int64), ("roots", C.c_int64)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class kz_request(C.Structure):
    _fields_ = [("n", C.c_int32), ("k", C.c_int32), ("row_words", C.c_int32), ("clique", C.c_int32),
                ("rows", C.c_void_p), ("colour", C.c_void_p), ("vmask", C.c_void_p), ("emask", C.c_void_p)]


class kz_out(C.Structure):
    _fields_ = [("result", kz_result), ("converged", C.c_int32), ("pad", C.c_int32), ("last_removed", C.c_int64)]


KZ_OUT_BYTES = C.sizeof(kz_out)


def kz_out_from_bytes(raw: bytes) -> dict:
    """A kz_out read back from memory, as a dict (the result's fields plus
    converged and last_removed)."""
    o = kz_out.from_buffer_copy(raw)
    d = o.result.as_dict()
    d["converged"] = int(o.converged)
    d["last_removed"] = int(o.last_removed)
    return d


class kz_colour_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("rounds", C.c_int32), ("colours", C.c_int32), ("pad", C.c_int32)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_ if name != "pad"}


class kz_server_config(C.Structure):
    _fields_ = [("split_n", C.c_int32), ("idle_us", C.c_int32), ("lease_us", C.c_int32), ("session_cus", C.c_int32),
                ("workers", C.c_int32), ("partition", C.c_int32), ("resident_limit", C.c_size_t)]


class kz_batch_config(C.Structure):
    _fields_ = [("waves", C.c_int32), ("chunk", C.c_int32), ("lpt", C.c_int32), ("workgroups", C.c_int32),
                ("share", C.c_int32)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


# numpy layouts of kz_batch_graph and kz_result (device arrays are filled from / read into these)
import numpy as np  # noqa: E402

BATCH_GRAPH_DTYPE = np.dtype([("n", "<i4"), ("k", "<i4"), ("row_words", "<i4"), ("clique", "<i4"),
                              ("row_offset", "<i8"), ("vertex_offset", "<i8")])
RESULT_DTYPE = np.dtype([("status", "<i4"), ("rounds", "<i4"), ("equals_input", "<i4"), ("passes", "<i4"),
                         ("surviving_vertices", "<i8"), ("surviving_edges", "<i8"), ("input_edges", "<i8"),
                         ("edge_tests", "<i8")])


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libkz.so is not built (run __graft_entry__.build()); there is no fallback")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.kz_create.restype = C.c_int
    lib.kz_create.argtypes = [C.POINTER(vp), C.c_int]
    lib.kz_destroy.restype = None
    lib.kz_destroy.argtypes = [vp]
    lib.kz_strerror.restype = C.c_char_p
    lib.kz_strerror.argtypes = [C.c_int]
    lib.kz_workspace_bytes.restype = C.c_int
    lib.kz_workspace_bytes.argtypes = [vp, C.POINTER(kz_graph), C.c_int32, C.POINTER(C.c_size_t)]
    lib.kz_kernelize.restype = C.c_int
    lib.kz_kernelize.argtypes = [vp, C.POINTER(kz_graph), vp, C.c_int32, vp, C.c_size_t, vp, vp, vp,
                                 C.POINTER(kz_result)]
    lib.kz_colour_workspace_bytes.restype = C.c_int
    lib.kz_colour_workspace_bytes.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
    lib.kz_colour_jp.restype = C.c_int
    lib.kz_colour_jp.argtypes = [vp, C.c_int32, vp, C.c_int32, vp, vp, C.c_size_t, vp, vp,
                                 C.POINTER(kz_colour_result)]
    lib.kz_kernelize_async.restype = C.c_int
    lib.kz_kernelize_async.argtypes = [vp, C.POINTER(kz_graph), vp, C.c_int32, vp, C.c_size_t, vp, vp, C.c_int32,
                                       C.c_int32, vp, vp]
    lib.kz_kernelize_noalloc.restype = C.c_int
    lib.kz_kernelize_noalloc.argtypes = [vp, C.POINTER(kz_graph), vp, C.c_int32, vp, vp, vp, C.POINTER(kz_result)]
    lib.kz_batch_workspace_bytes.restype = C.c_int
    lib.kz_batch_workspace_bytes.argtypes = [vp, vp, C.c_int32, C.POINTER(C.c_size_t)]
    lib.kz_kernelize_batch.restype = C.c_int
    lib.kz_kernelize_batch.argtypes = [vp, vp, vp, C.c_int32, vp, vp, vp, C.c_size_t, vp, vp, vp, vp]
    lib.kz_batch_autotune.restype = C.c_int
    lib.kz_batch_autotune.argtypes = [vp, vp, vp, C.c_int32, vp, vp, vp, C.c_size_t, vp, vp, vp, vp,
                                      C.POINTER(kz_batch_config)]
    lib.kz_batch_set_config.restype = C.c_int
    lib.kz_batch_set_config.argtypes = [vp, C.POINTER(kz_batch_config)]
    lib.kz_batch_get_config.restype = C.c_int
    lib.kz_batch_get_config.argtypes = [vp, C.POINTER(kz_batch_config)]
    lib.kz_profile_enable.restype = C.c_int
    lib.kz_profile_enable.argtypes = [vp, C.c_int]
    lib.kz_profile_read.restype = C.c_int
    lib.kz_profile_read.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.kz_server_fixed_bytes.restype = C.c_size_t
    lib.kz_server_fixed_bytes.argtypes = [C.c_int32]
    lib.kz_server_request_bytes.restype = C.c_size_t
    lib.kz_server_request_bytes.argtypes = [vp, C.POINTER(kz_request)]
    lib.kz_server_create.restype = C.c_int
    lib.kz_server_create.argtypes = [vp, vp, C.c_size_t, C.c_int32, vp, C.POINTER(vp)]
    lib.kz_server_submit.restype = C.c_int
    lib.kz_server_submit.argtypes = [vp, C.POINTER(kz_request), C.POINTER(C.c_uint64)]
    lib.kz_server_progress.restype = C.c_int
    lib.kz_server_progress.argtypes = [vp]
    lib.kz_server_poll.restype = C.c_int
    lib.kz_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(kz_result)]
    lib.kz_server_destroy.restype = None
    lib.kz_server_destroy.argtypes = [vp]
    lib.kz_server_done.restype = C.c_int
    lib.kz_server_done.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(kz_result), C.c_int32]
    lib.kz_server_configure.restype = C.c_int
    lib.kz_server_configure.argtypes = [vp, C.POINTER(kz_server_config)]
    lib.kz_set_edge_path.restype = C.c_int
    lib.kz_set_edge_path.argtypes = [vp, C.c_int32]
    lib.kz_gen_bitset.restype = C.c_int
    lib.kz_gen_bitset.argtypes = [vp, C.c_int32, vp, C.c_double, C.c_uint32, C.c_uint32, vp, vp, C.c_int32, vp, vp]
    lib.kz_dom_workspace_bytes.restype = C.c_int
    lib.kz_dom_workspace_bytes.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
    lib.kz_struction_workspace_bytes.restype = C.c_int
    lib.kz_struction_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
    lib.kz_struction.restype = C.c_int
    lib.kz_struction.argtypes = [vp, C.c_int32, vp, C.c_int32, C.c_int32, vp, C.c_size_t, vp, C.c_int32, C.c_int64,
                                 vp, vp, C.POINTER(kz_struction_result)]
    lib.kz_clique_workspace_bytes.restype = C.c_int
    lib.kz_clique_workspace_bytes.argtypes = [vp, C.c_int32, C.POINTER(C.c_size_t)]
    lib.kz_find_clique.restype = C.c_int
    lib.kz_find_clique.argtypes = [vp, vp, vp, C.c_int32, vp, vp, C.c_size_t, vp, vp, vp]
    lib.kz_dominance.restype = C.c_int
    lib.kz_dominance.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_int32, vp, C.c_size_t, vp, vp, vp,
                                 C.POINTER(kz_dom_result)]
    return lib


LIB = _load()


class KzError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        msg = LIB.kz_strerror(status).decode()
        super().__init__("%s%s (status %d)" % (where + ": " if where else "", msg, status))
        self.status = status


# ----------------------------------------------------------- C names
def kz_create(device: int = 0) -> int:
    h = C.c_void_p()
    st = LIB.kz_create(C.byref(h), int(device))
    if st != KZ_OK:
        raise KzError(st, "kz_create")
    return h.value


def kz_destroy(ctx: int) -> None:
    LIB.kz_destroy(ctx)


def kz_strerror(status: int) -> str:
    return LIB.kz_strerror(int(status)).decode()


def kz_workspace_bytes(ctx: int, graph: kz_graph, k: int) -> int:
    b = C.c_size_t(0)
    st = LIB.kz_workspace_bytes(ctx, C.byref(graph), int(k), C.byref(b))
    if st != KZ_OK:
        raise KzError(st, "kz_workspace_bytes")
    return int(b.value)


def kz_colour_workspace_bytes(n: int) -> int:
    b = C.c_size_t(0)
    st = LIB.kz_colour_workspace_bytes(int(n), C.byref(b))
    if st != 0:
        raise KzError(st, "kz_colour_workspace_bytes")
    return int(b.value)


def kz_colour_jp(ctx: int, n: int, rows_ptr: int, row_words: int, priority_ptr: int, ws_ptr: int, ws_bytes: int,
                 colour_ptr: int, stream: int) -> kz_colour_result:
    res = kz_colour_result()
    LIB.kz_colour_jp(ctx, int(n), rows_ptr, int(row_words), priority_ptr, ws_ptr, int(ws_bytes), colour_ptr, stream,
                     C.byref(res))
    return res


def kz_kernelize_async(ctx: int, graph: kz_graph, colour_ptr: int, k: int, ws_ptr: int, ws_bytes: int,
                       vmask_ptr: int, emask_ptr: int, first_pass: int, npasses: int, stream: int,
                       out_ptr: int | None) -> None:
    """Enqueues passes [first_pass, first_pass + npasses); raises on a
    host-detectable error (nothing enqueued then)."""
    st = LIB.kz_kernelize_async(ctx, C.byref(graph), colour_ptr, int(k), ws_ptr, int(ws_bytes), vmask_ptr,
                                emask_ptr, int(first_pass), int(npasses), stream, out_ptr)
    if st != 0:
        raise KzError(st, "kz_kernelize_async")


def kz_kernelize(ctx: int, graph: kz_graph, colour_ptr: int, k: int, ws_ptr: int, ws_bytes: int,
                 vmask_ptr: int, emask_ptr: int, stream: int) -> kz_result:
    res = kz_result()
    LIB.kz_kernelize(ctx, C.byref(graph), colour_ptr, int(k), ws_ptr, int(ws_bytes), vmask_ptr,
                     emask_ptr, stream, C.byref(res))
    return res


def kz_kernelize_noalloc(ctx: int, graph: kz_graph, colour_ptr: int, k: int, vmask_ptr: int, emask_ptr: int,
                         stream: int) -> kz_result:
    res = kz_result()
    LIB.kz_kernelize_noalloc(ctx, C.byref(graph), colour_ptr, int(k), vmask_ptr, emask_ptr, stream, C.byref(res))
    return res


def kz_profile_enable(ctx: int, on: bool) -> None:
    st = LIB.kz_profile_enable(ctx, 1 if on else 0)
    if st != KZ_OK:
        raise KzError(st, "kz_profile_enable")


def kz_profile_read(ctx: int, kernel: int) -> tuple[float, int]:
    ms, n = C.c_double(0.0), C.c_int64(0)
    st = LIB.kz_profile_read(ctx, int(kernel), C.byref(ms), C.byref(n))
    if st != KZ_OK:
        raise KzError(st, "kz_profile_read")
    return float(ms.value), int(n.value)


def kz_batch_workspace_bytes(ctx: int, graphs_host: np.ndarray) -> int:
    b = C.c_size_t(0)
    st = LIB.kz_batch_workspace_bytes(ctx, graphs_host.ctypes.data, len(graphs_host), C.byref(b))
    if st != KZ_OK:
        raise KzError(st, "kz_batch_workspace_bytes")
    return int(b.value)


def kz_kernelize_batch(ctx: int, graphs_host: np.ndarray, graphs_dev: int, G: int, rows: int, colour: int,
                       ws: int, ws_bytes: int, vmask: int, emask: int, results: int, stream: int) -> int:
    return int(LIB.kz_kernelize_batch(ctx, graphs_host.ctypes.data, graphs_dev, G, rows, colour, ws, ws_bytes,
                                      vmask, emask, results, stream))


def kz_batch_autotune(ctx: int, graphs_host: np.ndarray, graphs_dev: int, G: int, rows: int, colour: int,
                      ws: int, ws_bytes: int, vmask: int, emask: int, results: int, stream: int) -> dict:
    best = kz_batch_config()
    st = LIB.kz_batch_autotune(ctx, graphs_host.ctypes.data, graphs_dev, G, rows, colour, ws, ws_bytes,
                               vmask, emask, results, stream, C.byref(best))
    if st != KZ_OK:
        raise KzError(st, "kz_batch_autotune")
    return best.as_dict()


def kz_batch_set_config(ctx: int, cfg: dict) -> None:
    st = LIB.kz_batch_set_config(ctx, C.byref(kz_batch_config(**cfg)))
    if st != KZ_OK:
        raise KzError(st, "kz_batch_set_config")


def kz_batch_get_config(ctx: int) -> dict:
    cfg = kz_batch_config()
    st = LIB.kz_batch_get_config(ctx, C.byref(cfg))
    if st != KZ_OK:
        raise KzError(st, "kz_batch_get_config")
    return cfg.as_dict()


def kz_gen_bitset(ctx: int, sizes, p: float, seed: int, gid: int, planted, rows: int, row_words: int,
                  colour: int | None, stream: int | None) -> None:
    """Materialises a seeded random graph's bit rows on the device (see kz.h)."""
    sz = np.ascontiguousarray(np.asarray(sizes, np.int32))
    pl = None if planted is None else np.ascontiguousarray(np.asarray(planted, np.int32))
    st = LIB.kz_gen_bitset(ctx, len(sz), sz.ctypes.data, float(p), int(seed), int(gid),
                           None if pl is None else pl.ctypes.data, rows, int(row_words), colour, stream)
    if st != KZ_OK:
        raise KzError(st, "kz_gen_bitset")


def kz_set_edge_path(ctx: int, path: int) -> None:
    st = LIB.kz_set_edge_path(ctx, int(path))
    if st != KZ_OK:
        raise KzError(st, "kz_set_edge_path")


def kz_dom_workspace_bytes(n: int) -> int:
    need = C.c_size_t(0)
    st = LIB.kz_dom_workspace_bytes(int(n), C.byref(need))
    if st != KZ_OK:
        raise KzError(st, "kz_dom_workspace_bytes")
    return int(need.value)


def kz_dominance(ctx: int, mode: int, n: int, rows: int | None, row_words: int, ws: int, ws_bytes: int,
                 vmask: int | None, emask: int | None, stream: int | None) -> kz_dom_result:
    """Dominance reductions on device bit rows (see kz.h); the result's status is the return value."""
    res = kz_dom_result()
    LIB.kz_dominance(ctx, int(mode), int(n), rows, int(row_words), ws, int(ws_bytes), vmask, emask, stream,
                     C.byref(res))
    return res


def kz_clique_workspace_bytes(graph: "kz_graph", k: int) -> int:
    need = C.c_size_t(0)
    st = LIB.kz_clique_workspace_bytes(C.byref(graph), int(k), C.byref(need))
    if st != KZ_OK:
        raise KzError(st, "kz_clique_workspace_bytes")
    return int(need.value)


def kz_find_clique(ctx: int, graph: "kz_graph", colour: int | None, k: int, vmask: int | None, ws: int,
                   ws_bytes: int, clique: int | None, stream: int | None) -> kz_clique_result:
    """k-clique search (see kz.h); the result's status is the return value."""
    res = kz_clique_result()
    LIB.kz_find_clique(ctx, C.byref(graph), colour, int(k), vmask, ws, int(ws_bytes), clique, stream, C.byref(res))
    return res


def kz_struction_workspace_bytes(n: int, row_words: int) -> int:
    need = C.c_size_t(0)
    st = LIB.kz_struction_workspace_bytes(int(n), int(row_words), C.byref(need))
    if st != KZ_OK:
        raise KzError(st, "kz_struction_workspace_bytes")
    return int(need.value)


def kz_struction(ctx: int, n: int, rows: int | None, row_words: int, pivot: int, ws: int, ws_bytes: int,
                 out: int | None, out_row_words: int, out_nodes: int, map_: int | None,
                 stream: int | None) -> kz_struction_result:
    """Struction (see kz.h); out = None plans only.  The result's status is the return value."""
    res = kz_struction_result()
    LIB.kz_struction(ctx, int(n), rows, int(row_words), int(pivot), ws, int(ws_bytes), out, int(out_row_words),
                     int(out_nodes), map_, stream, C.byref(res))
    return res


def kz_server_fixed_bytes(max_slots: int) -> int:
    return int(LIB.kz_server_fixed_bytes(int(max_slots)))


def kz_server_request_bytes(srv: int, req: kz_request) -> int:
    return int(LIB.kz_server_request_bytes(srv, C.byref(req)))


def kz_server_create(ctx: int, arena: int, arena_bytes: int, max_slots: int, stream: int | None) -> int:
    srv = C.c_void_p()
    st = LIB.kz_server_create(ctx, arena, int(arena_bytes), int(max_slots), stream, C.byref(srv))
    if st != KZ_OK:
        raise KzError(st, "kz_server_create")
    return srv.value


def kz_server_submit(srv: int, req: kz_request) -> int | None:
    """Ticket, or None when the server cannot admit the request now (KZ_EAGAIN)."""
    t = C.c_uint64(0)
    st = LIB.kz_server_submit(srv, C.byref(req), C.byref(t))
    if st == KZ_EAGAIN:
        return None
    if st != KZ_OK:
        raise KzError(st, "kz_server_submit")
    return int(t.value)


def kz_server_progress(srv: int) -> int:
    st = LIB.kz_server_progress(srv)
    if st < 0:
        raise KzError(st, "kz_server_progress")
    return st


def kz_server_poll(srv: int, ticket: int) -> dict | None:
    """The request's result once it is done (the ticket is then retired), else None."""
    r = kz_result()
    st = LIB.kz_server_poll(srv, int(ticket), C.byref(r))
    if st < 0:
        raise KzError(st, "kz_server_poll")
    return r.as_dict() if st == 1 else None


def kz_server_destroy(srv: int) -> None:
    LIB.kz_server_destroy(srv)


def kz_server_done(srv: int, max_count: int = 256) -> list[tuple[int, dict]]:
    """Finished requests, oldest completion first: (ticket, result) pairs
    (retired)."""
    tickets = (C.c_uint64 * max_count)()
    res = (kz_result * max_count)()
    st = LIB.kz_server_done(srv, tickets, res, int(max_count))
    if st < 0:
        raise KzError(st, "kz_server_done")
    return [(int(tickets[i]), res[i].as_dict()) for i in range(st)]


def kz_server_configure(srv: int, split_n: int = 0, idle_us: int = 0, resident_limit: int = 0, lease_us: int = 0,
                        session_cus: int = 0, workers: int = 0, partition: int = 0) -> None:
    cfg = kz_server_config(int(split_n), int(idle_us), int(lease_us), int(session_cus), int(workers),
                           int(partition), int(resident_limit))
    st = LIB.kz_server_configure(srv, C.byref(cfg))
    if st != 0:
        raise KzError(st, "kz_server_configure")


# ----------------------------------------------------------- tensor helpers
_RAW_STREAM = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_handle(stream: torch.cuda.Stream | None, device: torch.device) -> int:
    """The HIP stream handle to launch on: `stream`'s, else the device's
    current stream (read without building a Stream object: this is on the
    per-call path)."""
    if stream is not None:
        return stream.cuda_stream
    if _RAW_STREAM is not None:
        return _RAW_STREAM(device.index if device.index is not None else torch.cuda.current_device())
    return torch.cuda.current_stream(device).cuda_stream


def _dev_ptr(t: torch.Tensor | None) -> int | None:
    if t is None or t.numel() == 0:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def graph_dense(adj: torch.Tensor) -> kz_graph:
    if adj.dtype != torch.uint8 or adj.dim() != 2 or adj.shape[0] != adj.shape[1]:
        raise ValueError("dense adjacency must be a square uint8 tensor")
    return kz_graph(format=KZ_DENSE_U8, n=adj.shape[0], adj=_dev_ptr(adj))


def graph_bitset(rows: torch.Tensor) -> kz_graph:
    if rows.dtype not in (torch.int64, torch.uint64) or rows.dim() != 2:
        raise ValueError("bitset rows must be a 2-D 64-bit tensor")
    return kz_graph(format=KZ_BITSET_U64, n=rows.shape[0], rows=_dev_ptr(rows), row_words=rows.shape[1])


def graph_csr(row_ptr: torch.Tensor, col_idx: torch.Tensor) -> kz_graph:
    if row_ptr.dtype != torch.int64 or col_idx.dtype != torch.int32:
        raise ValueError("CSR needs int64 row_ptr and int32 col_idx")
    return kz_graph(format=KZ_CSR, n=row_ptr.shape[0] - 1, row_ptr=_dev_ptr(row_ptr),
                    col_idx=_dev_ptr(col_idx) if col_idx.numel() else None, nnz=col_idx.shape[0])


class Kernelizer:
    """Holds a context and a growing device workspace on one GPU."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        self.ctx = kz_create(device)
        self._ws = None
        self._need = {}

    def close(self):
        if self.ctx:
            kz_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, on: bool) -> None:
        kz_profile_enable(self.ctx, on)

    def kernel_times(self) -> dict:
        """{kernel family: (total ms, launches)} since profiling was enabled."""
        return {name: kz_profile_read(self.ctx, i) for i, name in enumerate(KERNELS)}

    def set_edge_path(self, path: int) -> None:
        """KZ_EDGE_BITSET or KZ_EDGE_MFMA_I8 for later calls (workspace sizes are re-queried)."""
        kz_set_edge_path(self.ctx, path)
        self._need = {}

    def workspace(self, graph: kz_graph, k: int) -> torch.Tensor:
        key = (graph.format, graph.n, graph.row_words, graph.nnz, k)
        need = self._need.get(key)
        if need is None:
            need = self._need[key] = kz_workspace_bytes(self.ctx, graph, k)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def run(self, graph: kz_graph, colour: torch.Tensor, k: int, vmask: torch.Tensor,
            emask: torch.Tensor, stream: torch.cuda.Stream | None = None, check: bool = True) -> dict:
        if colour.dtype != torch.int32:
            raise ValueError("colour must be int32")
        ws = self.workspace(graph, k)
        res = kz_kernelize(self.ctx, graph, _dev_ptr(colour), k, ws.data_ptr(), ws.numel(),
                           _dev_ptr(vmask), _dev_ptr(emask), _stream_handle(stream, self.device))
        if check and res.status != KZ_OK:
            raise KzError(res.status, "kz_kernelize")
        return res.as_dict()

    def run_async(self, graph: kz_graph, colour: torch.Tensor, k: int, vmask: torch.Tensor,
                  emask: torch.Tensor, out: torch.Tensor | None, first_pass: int = 1, npasses: int = 32,
                  stream: torch.cuda.Stream | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
        """Enqueues passes [first_pass, first_pass + npasses) (no wait); `out`:
        a uint8 device tensor of KZ_OUT_BYTES receiving the kz_out in stream
        order.  Returns the workspace used (pass it again to continue)."""
        if colour.dtype != torch.int32:
            raise ValueError("colour must be int32")
        if out is not None and out.numel() * out.element_size() < KZ_OUT_BYTES:
            raise ValueError("out must hold a kz_out")
        if ws is None:
            ws = self.workspace(graph, k)
        kz_kernelize_async(self.ctx, graph, _dev_ptr(colour), k, ws.data_ptr(), ws.numel(), _dev_ptr(vmask),
                           _dev_ptr(emask), first_pass, npasses, _stream_handle(stream, self.device),
                           None if out is None else out.data_ptr())
        return ws

    def colour_jp(self, rows: torch.Tensor, n: int, priority: torch.Tensor,
                  stream: torch.cuda.Stream | None = None, check: bool = True) -> tuple[torch.Tensor, dict]:
        """Jones-Plassmann colouring of plain bit rows (uint64 [n, row_words]):
        (colour int32[n] on the device, result dict)."""
        if priority.dtype not in (torch.int64, torch.uint64) or priority.numel() != n:
            raise ValueError("priority must be n 64-bit values")
        rw = int(rows.shape[1]) if rows.dim() == 2 else (int(rows.numel()) // n if n else 0)
        ws = torch.empty(max(kz_colour_workspace_bytes(n), 256), dtype=torch.uint8, device=self.device)
        colour = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        res = kz_colour_jp(self.ctx, n, _dev_ptr(rows), rw, _dev_ptr(priority), ws.data_ptr(), ws.numel(),
                           colour.data_ptr(), _stream_handle(stream, self.device))
        if check and res.status != KZ_OK:
            raise KzError(res.status, "kz_colour_jp")
        return colour[:n], res.as_dict()

    def kernelize_dense(self, adj: torch.Tensor, colour: torch.Tensor, k: int, **kw):
        """(vmask u8[n], emask u8[n,n], result dict) for a dense uint8 adjacency."""
        n = adj.shape[0]
        vmask = torch.empty(n, dtype=torch.uint8, device=self.device)
        emask = torch.empty((n, n), dtype=torch.uint8, device=self.device)
        res = self.run(graph_dense(adj), colour, k, vmask, emask, **kw)
        return vmask, emask, res

    def kernelize_csr(self, row_ptr: torch.Tensor, col_idx: torch.Tensor, colour: torch.Tensor, k: int, **kw):
        """(vmask u8[n], emask u8[nnz] aligned with col_idx, result dict) for a CSR graph."""
        n = row_ptr.shape[0] - 1
        vmask = torch.empty(n, dtype=torch.uint8, device=self.device)
        emask = torch.empty(col_idx.shape[0], dtype=torch.uint8, device=self.device)
        res = self.run(graph_csr(row_ptr, col_idx), colour, k, vmask, emask, **kw)
        return vmask, emask, res

    def kernelize_bitset(self, rows: torch.Tensor, colour: torch.Tensor, k: int, **kw):
        """(vmask u8[n], emask int64[n,R] rows, result dict) for class-major bit rows."""
        vmask = torch.empty(rows.shape[0], dtype=torch.uint8, device=self.device)
        emask = torch.empty_like(rows)
        res = self.run(graph_bitset(rows), colour, k, vmask, emask, **kw)
        return vmask, emask, res


    def dominance(self, rows: torch.Tensor, mode: int, stream: torch.cuda.Stream | None = None,
                  check: bool = True):
        """Dominance reductions (KZ_DOM_VERTEX or KZ_DOM_EDGE) on plain bit
        rows int64 [n, R] (R >= ceil(n/64)): (vmask u8[n], emask int64[n, R],
        result dict)."""
        n, R = int(rows.shape[0]), int(rows.shape[1]) if rows.dim() == 2 else 0
        vmask = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        emask = torch.empty((max(n, 1), max(R, 1)), dtype=torch.int64, device=self.device)
        ws = torch.empty(max(kz_dom_workspace_bytes(n), 256), dtype=torch.uint8, device=self.device)
        res = kz_dominance(self.ctx, mode, n, _dev_ptr(rows), R, ws.data_ptr(), ws.numel(), _dev_ptr(vmask),
                           _dev_ptr(emask), _stream_handle(stream, self.device))
        if check and res.status != KZ_OK:
            raise KzError(res.status, "kz_dominance")
        return vmask[:n], emask[:n], res.as_dict()


    def find_clique(self, rows: torch.Tensor, colour: torch.Tensor, k: int, vmask: torch.Tensor | None = None,
                    stream: torch.cuda.Stream | None = None, check: bool = True):
        """The lexicographically smallest k-clique of class-major bit rows
        int64 [n, R] among the live vertices (vmask, or all): (clique int32[k]
        tensor, all -1 when none, result dict)."""
        g = graph_bitset(rows)
        ws = torch.empty(kz_clique_workspace_bytes(g, k), dtype=torch.uint8, device=self.device)
        clique = torch.empty(max(int(k), 1), dtype=torch.int32, device=self.device)
        res = kz_find_clique(self.ctx, g, _dev_ptr(colour), k, _dev_ptr(vmask), ws.data_ptr(), ws.numel(),
                             clique.data_ptr(), _stream_handle(stream, self.device))
        if check and res.status != KZ_OK:
            raise KzError(res.status, "kz_find_clique")
        return clique[:k], res.as_dict()


    def struction(self, rows: torch.Tensor, pivot: int = 0, stream: torch.cuda.Stream | None = None,
                  check: bool = True):
        """G' of Definition 4.1.1 around `pivot` for plain bit rows int64 [n, R]:
        (rows int64 [n', ceil(n'/64)], map int32 [n', 2], result dict)."""
        n, R = int(rows.shape[0]), int(rows.shape[1])
        ws = torch.empty(kz_struction_workspace_bytes(n, R), dtype=torch.uint8, device=self.device)
        sh = _stream_handle(stream, self.device)
        res = kz_struction(self.ctx, n, _dev_ptr(rows), R, pivot, ws.data_ptr(), ws.numel(), None, 0, 0, None, sh)
        if res.status != KZ_OK:
            if check:
                raise KzError(res.status, "kz_struction")
            return None, None, res.as_dict()
        npr, rp = int(res.nodes), max(int(res.row_words), 1)
        out = torch.empty((max(npr, 1), rp), dtype=torch.int64, device=self.device)
        mp = torch.empty((max(npr, 1), 2), dtype=torch.int32, device=self.device)
        res = kz_struction(self.ctx, n, _dev_ptr(rows), R, pivot, ws.data_ptr(), ws.numel(), out.data_ptr(), rp, npr,
                           mp.data_ptr(), sh)
        if check and res.status != KZ_OK:
            raise KzError(res.status, "kz_struction")
        return out[:npr], mp[:npr], res.as_dict()


LINE_WORDS, LINE_VERTICES = 16, 128   # a graph's arena ranges start on a 128-byte line


def _line_up(x: int, q: int) -> int:
    return (x + q - 1) // q * q


class Batch:
    """Arenas, descriptors and results of one batch of bit-row graphs on a device.

    ``graphs`` is a list of (rows uint64 [n, R], colour int32 [n], k) or
    (rows, colour, k, clique) -- clique: the clique size when it is below the
    number of colour classes k (0 = k).  Each graph's ranges start on a
    128-byte line (kz_kernelize_batch requires it).
    """

    def __init__(self, graphs, device):
        self.device = torch.device(device)
        G = len(graphs)
        desc = np.zeros(G, BATCH_GRAPH_DTYPE)
        ro, vo = 0, 0
        for i, gr in enumerate(graphs):
            rows, colour, k = gr[:3]
            clique = int(gr[3]) if len(gr) > 3 else 0
            n, R = (rows.shape[0], rows.shape[1]) if rows.ndim == 2 else (len(colour), 0)
            desc[i] = (n, k, R, clique, ro, vo)
            ro = _line_up(ro + n * R, LINE_WORDS)
            vo = _line_up(vo + n, LINE_VERTICES)
        self.G = G
        self.desc = desc
        rows_all = np.zeros(max(ro, 1), np.uint64)
        col_all = np.zeros(max(vo, 1), np.int32)
        for i, gr in enumerate(graphs):
            rows, colour = gr[0], gr[1]
            n, R = int(desc[i]["n"]), int(desc[i]["row_words"])
            a, b = int(desc[i]["row_offset"]), int(desc[i]["vertex_offset"])
            rows_all[a:a + n * R] = np.asarray(rows, np.uint64).reshape(-1)
            col_all[b:b + n] = colour
        self.rows = torch.from_numpy(rows_all.view(np.int64)).to(self.device)
        self.colour = torch.from_numpy(col_all).to(self.device)
        self.desc_dev = torch.from_numpy(desc.view(np.uint8)).to(self.device)
        self.vmask = torch.empty(max(vo, 1), dtype=torch.uint8, device=self.device)
        self.emask = torch.empty_like(self.rows)
        self.results = torch.zeros(max(G, 1) * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=self.device)

    @classmethod
    def allocate(cls, shapes, device):
        """A batch whose arenas are allocated but not filled: ``shapes`` is a
        list of (n, row_words, k); the caller writes each graph's rows and
        colours at its descriptor's offsets (for example with kz_gen_bitset)."""
        self = cls.__new__(cls)
        self.device = torch.device(device)
        G = len(shapes)
        desc = np.zeros(G, BATCH_GRAPH_DTYPE)
        ro, vo = 0, 0
        for i, (n, R, k) in enumerate(shapes):
            desc[i] = (n, k, R, 0, ro, vo)
            ro = _line_up(ro + n * R, LINE_WORDS)
            vo = _line_up(vo + n, LINE_VERTICES)
        self.G, self.desc = G, desc
        self.rows = torch.zeros(max(ro, 1), dtype=torch.int64, device=self.device)
        self.colour = torch.zeros(max(vo, 1), dtype=torch.int32, device=self.device)
        self.desc_dev = torch.from_numpy(desc.view(np.uint8)).to(self.device)
        self.vmask = torch.empty(max(vo, 1), dtype=torch.uint8, device=self.device)
        self.emask = torch.empty_like(self.rows)
        self.results = torch.zeros(max(G, 1) * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        return self

    def args(self):
        return (self.desc, self.desc_dev.data_ptr(), self.G, self.rows.data_ptr(), self.colour.data_ptr())

    def outputs(self):
        return self.vmask.data_ptr(), self.emask.data_ptr(), self.results.data_ptr()

    def read_results(self) -> np.ndarray:
        return self.results.cpu().numpy()[:self.G * RESULT_DTYPE.itemsize].view(RESULT_DTYPE)

    def masks(self, i):
        """(vmask u8[n], emask uint64 [n, R]) of graph i (host copies)."""
        d = self.desc[i]
        n, R = int(d["n"]), int(d["row_words"])
        a, b = int(d["row_offset"]), int(d["vertex_offset"])
        vm = self.vmask[b:b + n].cpu().numpy()
        em = self.emask[a:a + n * R].cpu().numpy().view(np.uint64).reshape(n, R)
        return vm, em


class BatchKernelizer:
    """kz_kernelize_batch on one device with a reusable workspace."""

    def __init__(self, kz: Kernelizer):
        self.kz = kz
        self._ws = None

    def workspace(self, batch: Batch) -> torch.Tensor:
        need = kz_batch_workspace_bytes(self.kz.ctx, batch.desc)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=batch.device)
        return self._ws

    def run(self, batch: Batch, stream: torch.cuda.Stream | None = None) -> None:
        """Enqueues the batch on the stream (asynchronous)."""
        ws = self.workspace(batch)
        st = kz_kernelize_batch(self.kz.ctx, *batch.args(), ws.data_ptr(), ws.numel(), *batch.outputs(),
                                _stream_handle(stream, batch.device))
        if st != KZ_OK:
            raise KzError(st, "kz_kernelize_batch")

    def autotune(self, batch: Batch) -> dict:
        ws = self.workspace(batch)
        s = torch.cuda.current_stream(batch.device)
        return kz_batch_autotune(self.kz.ctx, *batch.args(), ws.data_ptr(), ws.numel(), *batch.outputs(),
                                 s.cuda_stream)


class Server:
    """A kz_server with its arena allocated by torch on one device."""

    def __init__(self, kz: Kernelizer, arena_bytes: int, max_slots: int = 512,
                 stream: torch.cuda.Stream | None = None):
        self.kz = kz
        self.device = kz.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        fixed = kz_server_fixed_bytes(max_slots)
        self.arena = torch.empty(fixed + int(arena_bytes), dtype=torch.uint8, device=self.device)
        self.srv = kz_server_create(kz.ctx, self.arena.data_ptr(), self.arena.numel(), max_slots,
                                    self.stream.cuda_stream)
        self.keep = {}   # ticket -> tensors that must outlive the request

    @staticmethod
    def request(rows: torch.Tensor, colour: torch.Tensor, k: int, vmask: torch.Tensor,
                emask: torch.Tensor, clique: int = 0) -> kz_request:
        n = int(colour.numel())
        R = int(rows.shape[1]) if rows.dim() == 2 else (int(rows.numel()) // n if n else 0)
        return kz_request(n, int(k), R, int(clique), _dev_ptr(rows), _dev_ptr(colour), _dev_ptr(vmask),
                          _dev_ptr(emask))

    def submit(self, rows, colour, k, vmask, emask, clique: int = 0) -> int | None:
        t = kz_server_submit(self.srv, self.request(rows, colour, k, vmask, emask, clique))
        if t is not None:
            self.keep[t] = (rows, colour, vmask, emask)
        return t

    def configure(self, split_n: int = 0, idle_us: int = 0, resident_limit: int = 0, lease_us: int = 0,
                  session_cus: int = 0, workers: int = 0, partition: int = 0) -> None:
        """Lane split, session idle time and lease, session compute units,
        single-graph workers, compute-unit partition and resident-byte limit
        (0: defaults / no limit); only while no request is admitted."""
        kz_server_configure(self.srv, split_n, idle_us, resident_limit, lease_us, session_cus, workers, partition)

    def progress(self) -> int:
        return kz_server_progress(self.srv)

    def done(self, max_count: int = 256) -> list[tuple[int, dict]]:
        """Finished requests since the last call (retired), oldest first."""
        out = kz_server_done(self.srv, max_count)
        for t, _ in out:
            self.keep.pop(t, None)
        return out

    def poll(self, ticket: int) -> dict | None:
        r = kz_server_poll(self.srv, ticket)
        if r is not None:
            self.keep.pop(ticket, None)
        return r

    def close(self) -> None:
        if self.srv:
            kz_server_destroy(self.srv)
            self.srv = None
            self.keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
