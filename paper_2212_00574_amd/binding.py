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

EXPORTED = ("kz_create", "kz_destroy", "kz_strerror", "kz_workspace_bytes", "kz_kernelize",
            "kz_profile_enable", "kz_profile_read")
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
    lib.kz_profile_enable.restype = C.c_int
    lib.kz_profile_enable.argtypes = [vp, C.c_int]
    lib.kz_profile_read.restype = C.c_int
    lib.kz_profile_read.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
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


def kz_kernelize(ctx: int, graph: kz_graph, colour_ptr: int, k: int, ws_ptr: int, ws_bytes: int,
                 vmask_ptr: int, emask_ptr: int, stream: int) -> kz_result:
    res = kz_result()
    LIB.kz_kernelize(ctx, C.byref(graph), colour_ptr, int(k), ws_ptr, int(ws_bytes), vmask_ptr,
                     emask_ptr, stream, C.byref(res))
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


# ----------------------------------------------------------- tensor helpers
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
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        res = kz_kernelize(self.ctx, graph, _dev_ptr(colour), k, ws.data_ptr(), ws.numel(),
                           _dev_ptr(vmask), _dev_ptr(emask), s.cuda_stream)
        if check and res.status != KZ_OK:
            raise KzError(res.status, "kz_kernelize")
        return res.as_dict()

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
