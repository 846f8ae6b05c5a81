"""Python binding of the MI355X GOVM library (``libdawn.so``, C ABI in
``include/dawn.h``).

Argument marshalling only: every step of the shortest-path computation runs in
the HIP kernels of the library.  PyTorch supplies device memory and streams.
There is no CPU fallback; without the built library every call raises.

    import paper_2306_07872_amd as dawn
    csr = dawn.Csr.from_arrays(rowptr, colidx, weights, device="cuda")
    d = dawn.sssp(csr, source)                 # [n]   uint32 or float32
    D = dawn.msssp(csr, sources)               # [k,n]
    A = dawn.apsp(csr)                         # [n,n]
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdawn.so")

W_U32, W_F32, W_I32, W_UNIT = 0, 1, 2, 3
TILE_K_MAX = 512

_STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "workspace too small",
           4: "HIP error", 5: "run did not converge"}
E_INCOMPLETE = 5
DEVICE_QUERY_LEN = 16


class DawnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class RunInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("frontier_entries", ctypes.c_int64), ("edges_scanned", ctypes.c_int64),
                ("improvements", ctypes.c_int64), ("union_rows", ctypes.c_int64),
                ("union_edges", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in
                ("t_lane", "t_wave", "t_chunk", "wg_threads", "grid", "mode", "step_launches",
                 "tile_k", "tile_t_wave", "tile_t_chunk", "validate", "coop", "tile_t_group",
                 "tile_skip", "small_m", "step_min_m", "tile_sparse", "tile_pull",
                 "tile_pull_src", "ss_skip", "ss_pull", "tile_step_launches", "barrier_ms",
                 "ss_tail_grid")]


INFO_BYTES = ctypes.sizeof(RunInfo)
_lib = None

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t


def load():
    """Load libdawn.so (built by ``python -m paper_2306_07872_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2306_07872_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "dawn_status_str": ([_i32], ctypes.c_char_p),
        "dawn_last_error": ([], ctypes.c_char_p),
        "dawn_build_info": ([], ctypes.c_char_p),
        "dawn_get_tuning": ([ctypes.POINTER(Tuning)], _i32),
        "dawn_set_tuning": ([ctypes.POINTER(Tuning)], _i32),
        "dawn_sssp": ([_vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp], _i32),
        "dawn_sssp_workspace_bytes": ([_i32, _i32], _sz),
        "dawn_sssp_ws": ([_vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _sz, _vp, _vp], _i32),
        "dawn_sssp_noalloc": ([_vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp], _i32),
        "dawn_msssp": ([_vp, _vp, _vp, _i32, _i32, _i32, _vp, _i32, _vp, _vp], _i32),
        "dawn_msssp_workspace_bytes": ([_i32, _i32, _i32], _sz),
        "dawn_msssp_ws": ([_vp, _vp, _vp, _i32, _i32, _i32, _vp, _i32, _vp, _vp, _sz, _vp, _vp],
                          _i32),
        "dawn_apsp": ([_vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp], _i32),
        "dawn_tgraph_bytes": ([_i32, _i32], _sz),
        "dawn_tgraph_build_bytes": ([_i32, _i32], _sz),
        "dawn_tgraph_build": ([_vp, _vp, _vp, _i32, _i32, _vp, _sz, _vp, _sz, _vp], _i32),
        "dawn_msssp_tg_ws": ([_vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _sz, _vp,
                              _vp], _i32),
        "dawn_umsssp_workspace_bytes": ([_i32, _i32, _i32], _sz),
        "dawn_workspace_bytes": ([_i32, _i32, _i32, _i32], _sz),
        "dawn_sssp_tg_ws": ([_vp, _vp, _vp, _i32, _i32, _i32, _vp, _i32, _vp, _vp, _sz, _vp, _vp],
                            _i32),
        "dawn_tile_set_tgraph": ([_vp, _vp], _i32),
        "dawn_umsssp_ws": ([_vp, _vp, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _sz, _vp, _vp], _i32),
        "dawn_batch_create": ([ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp),
                               ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                               ctypes.POINTER(_i32), ctypes.POINTER(_i32), _i32, _vp], _i32),
        "dawn_batch_sizes": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)], _i32),
        "dawn_batch_vertex_offset": ([_vp, _i32], _i64),
        "dawn_batch_run": ([_vp, _vp, _vp, _vp, _vp], _i32),
        "dawn_batch_capture": ([_vp, _vp, _vp, _vp, _vp], _i32),
        "dawn_batch_replay": ([_vp, _vp], _i32),
        "dawn_batch_destroy": ([_vp], None),
        "dawn_tile_bytes": ([_i32, _i32, _i32], _sz),
        "dawn_tile_create": ([ctypes.POINTER(_vp), _vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp,
                              _sz, _vp], _i32),
        "dawn_run_status": ([ctypes.POINTER(_i32), ctypes.POINTER(_i32)], _i32),
        "dawn_tile_admit": ([_vp, _i32, _i32, _vp], _i32),
        "dawn_tile_run": ([_vp, _i32, _vp, _vp], _i32),
        "dawn_tile_capture": ([_vp, _i32, _vp], _i32),
        "dawn_tile_replay": ([_vp, _vp], _i32),
        "dawn_tile_read": ([_vp, _i32, _vp, _vp], _i32),
        "dawn_tile_steps": ([_vp, _vp, _vp], _i32),
        "dawn_tile_evict": ([_vp, _i32, _vp], _i32),
        "dawn_tile_destroy": ([_vp], None),
        "dawn_kernel_timer": ([_i32], _i32),
        "dawn_device_query": ([ctypes.POINTER(_i32)], _i32),
        "dawn_kernel_time": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32)], _i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def exported_symbols() -> list[str]:
    """Names of the C entry points this binding declares."""
    return [
        "dawn_status_str", "dawn_last_error", "dawn_build_info", "dawn_get_tuning",
        "dawn_set_tuning", "dawn_sssp", "dawn_sssp_workspace_bytes", "dawn_sssp_ws",
        "dawn_sssp_tg_ws", "dawn_sssp_noalloc",
        "dawn_msssp", "dawn_msssp_workspace_bytes", "dawn_msssp_ws", "dawn_apsp",
        "dawn_tgraph_bytes", "dawn_tgraph_build_bytes", "dawn_tgraph_build", "dawn_msssp_tg_ws",
        "dawn_umsssp_workspace_bytes", "dawn_umsssp_ws", "dawn_workspace_bytes", "dawn_batch_create", "dawn_batch_sizes", "dawn_batch_vertex_offset", "dawn_batch_run",
        "dawn_batch_capture", "dawn_batch_replay", "dawn_batch_destroy", "dawn_tile_bytes",
        "dawn_tile_create", "dawn_tile_admit", "dawn_tile_run", "dawn_tile_capture",
        "dawn_tile_replay", "dawn_tile_read",
        "dawn_tile_set_tgraph",
        "dawn_tile_steps", "dawn_tile_evict", "dawn_tile_destroy", "dawn_kernel_timer",
        "dawn_kernel_time", "dawn_device_query", "dawn_run_status"]


def _check(status: int):
    if status != 0:
        raise DawnError(status, load().dawn_last_error().decode(errors="replace"))


def _torch():
    import torch
    return torch


def run_status() -> tuple[int, int]:
    """(runs that ended without converging, status of the last one) among the
    runs launched without run info on the current device whose work has
    completed (``dawn_run_status``; synchronise first).  Clears the record."""
    cnt, last = _i32(), _i32()
    st = load().dawn_run_status(ctypes.byref(cnt), ctypes.byref(last))
    if st not in (0, E_INCOMPLETE):
        _check(st)
    return int(cnt.value), int(last.value)


def check_runs(stream=None):
    """Synchronise `stream` and raise DawnError if a run launched without run
    info on this device ended without converging."""
    torch = _torch()
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()
    cnt, last = run_status()
    if cnt:
        raise DawnError(E_INCOMPLETE, f"{cnt} run(s) ended without converging "
                                      f"(last status {last})")


def _check_info(info, stream=None):
    """Synchronise and raise DawnError if the run in `info` did not converge."""
    torch = _torch()
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()
    conv = read_info(info)["converged"]
    if conv != 1:
        raise DawnError(E_INCOMPLETE, f"run ended with status {conv}")


def _finish(info, stream, check):
    if not check:
        return
    if info is None:
        check_runs(stream)
    else:
        _check_info(info, stream)


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def wtype_code(wtype: str) -> int:
    return {"u32": W_U32, "f32": W_F32, "i32": W_I32, "unit": W_UNIT}[wtype]


def dist_dtype(wtype: str):
    torch = _torch()
    return {"u32": torch.uint32, "f32": torch.float32, "i32": torch.int32,
            "unit": torch.uint32}[wtype]


# ---------------------------------------------------------------------------
# graph residency
# ---------------------------------------------------------------------------

@dataclass
class Csr:
    """A CSR graph resident in device memory (torch tensors)."""
    rowptr: object   # int32 [n+1]
    colidx: object   # int32 [m]
    w: object        # uint32, float32 or int32 [m]
    n: int
    m: int
    wtype: str

    @staticmethod
    def from_arrays(rowptr, colidx, w, wtype: str | None = None, device="cuda") -> "Csr":
        torch = _torch()
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        colidx = np.ascontiguousarray(colidx, dtype=np.int32)
        w = np.ascontiguousarray(w)
        if wtype is None:
            wtype = "f32" if np.issubdtype(w.dtype, np.floating) else "u32"
        # unit weights are never read: keep a one-word placeholder
        if wtype == "unit":
            w = np.zeros(1, np.uint32)
        w = w.astype({"f32": np.float32, "u32": np.uint32, "i32": np.int32,
                      "unit": np.uint32}[wtype], copy=False)
        n = int(rowptr.shape[0]) - 1
        m = int(colidx.shape[0])
        # keep at least one element so every pointer is valid even when m == 0
        ci = colidx if m else np.zeros(1, np.int32)
        ww = w if (m and wtype != "unit") else np.zeros(1, w.dtype)
        return Csr(torch.from_numpy(rowptr).to(device), torch.from_numpy(ci).to(device),
                   torch.from_numpy(ww).to(device), n, m, wtype)

    @staticmethod
    def from_graph(g, device="cuda", wtype: str | None = None) -> "Csr":
        """wtype overrides the graph's ("unit": hop counts, weights dropped)."""
        return Csr.from_arrays(g.rowptr, g.colidx, g.w, wtype or g.wtype, device)

    @property
    def code(self) -> int:
        return wtype_code(self.wtype)

    def nbytes(self) -> int:
        return 4 * (self.n + 1) + 8 * self.m


def _csr_args(c: Csr):
    return (_ptr(c.rowptr), _ptr(c.colidx), _ptr(c.w), c.code, c.n, c.m)


def info_tensor(device="cuda"):
    torch = _torch()
    return torch.zeros(INFO_BYTES, dtype=torch.uint8, device=device)


def read_info(t) -> dict:
    raw = bytes(t.cpu().numpy().tobytes())
    ri = RunInfo.from_buffer_copy(raw)
    return {k: getattr(ri, k) for k, _ in RunInfo._fields_}


# ---------------------------------------------------------------------------
# tuning
# ---------------------------------------------------------------------------

def get_tuning() -> dict:
    t = Tuning()
    _check(load().dawn_get_tuning(ctypes.byref(t)))
    return {k: getattr(t, k) for k, _ in Tuning._fields_}


def set_tuning(**kw) -> dict:
    """Update tuning fields (see dawn_tuning); returns the previous settings.
    ``set_tuning(reset=True)`` restores the defaults."""
    prev = get_tuning()
    if kw.pop("reset", False):
        _check(load().dawn_set_tuning(None))
        if not kw:
            return prev
    cur = get_tuning()
    for k, v in kw.items():
        if k not in cur:
            raise KeyError(k)
        cur[k] = int(v)
    t = Tuning(**cur)
    _check(load().dawn_set_tuning(ctypes.byref(t)))
    return prev


# ---------------------------------------------------------------------------
# single / multi source, all pairs
# ---------------------------------------------------------------------------

def sssp_workspace_bytes(n: int, m: int) -> int:
    return int(load().dawn_sssp_workspace_bytes(n, m))


def workspace(nbytes: int, device="cuda"):
    """A device buffer usable as a caller workspace (256-byte aligned)."""
    torch = _torch()
    return torch.empty(max(nbytes, 256) + 256, dtype=torch.uint8, device=device)


def _aligned(buf):
    p = buf.data_ptr()
    return ctypes.c_void_p((p + 255) & ~255), buf.numel() - (((p + 255) & ~255) - p)


def sssp(csr: Csr, source: int, out=None, stream=None, ws=None, info=None, tgraph=None,
         check: bool = True):
    """Distances from `source` (tensor of length n, of the graph's distance type).
    With `ws` (a buffer from ``workspace``) and/or `info` (from
    ``info_tensor``) the ``dawn_sssp_ws`` entry point is used; with `tgraph`
    (from ``tgraph(csr)``) ``dawn_sssp_tg_ws``, whose dense steps may pull
    (tuning field ss_pull).  check=True synchronises the stream and raises
    DawnError if the run did not converge (from `info`, or from
    ``dawn_run_status`` when no info is given); check=False leaves the call
    asynchronous."""
    torch = _torch()
    if out is None:
        out = torch.empty(csr.n, dtype=dist_dtype(csr.wtype), device=csr.rowptr.device)
    L = load()
    if tgraph is not None:
        if ws is None:
            ws = workspace(sssp_workspace_bytes(csr.n, csr.m), csr.rowptr.device)
        p, nb = _aligned(ws)
        _check(L.dawn_sssp_tg_ws(*_csr_args(csr), _aligned(tgraph)[0], int(source), _ptr(out), p,
                                 nb, _ptr(info), _stream(stream)))
    elif ws is None and info is None:
        _check(L.dawn_sssp(*_csr_args(csr), int(source), _ptr(out), _stream(stream)))
    else:
        if ws is None:
            ws = workspace(sssp_workspace_bytes(csr.n, csr.m), csr.rowptr.device)
        p, nb = _aligned(ws)
        _check(L.dawn_sssp_ws(*_csr_args(csr), int(source), _ptr(out), p, nb,
                              _ptr(info), _stream(stream)))
    _finish(info, stream, check)
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def sssp_noalloc(csr: Csr, source: int, out, stream=None, check: bool = True):
    """``dawn_sssp_noalloc``: distances from `source` into the caller's `out`
    (length n, the graph's distance type), with the library's fixed per-device
    scratch array as workspace, so the call allocates no device memory.  Graphs
    needing more than NOALLOC_SCRATCH_BYTES of workspace raise DawnError
    (workspace too small).  Calls on one device share the array: order them on
    one stream.  check=True synchronises and raises if the run did not
    converge (``dawn_run_status``)."""
    if out.numel() < csr.n or out.element_size() != 4 or not out.is_contiguous():
        raise ValueError("out must be a contiguous 4-byte tensor of at least n elements")
    L = load()
    _check(L.dawn_sssp_noalloc(*_csr_args(csr), int(source), _ptr(out), _stream(stream)))
    _finish(None, stream, check)
    return out


def msssp_workspace_bytes(n: int, m: int, k: int) -> int:
    return int(load().dawn_msssp_workspace_bytes(n, m, k))


def tgraph(csr: Csr, stream=None):
    """The reverse graph of `csr` for pull steps (``dawn_tgraph_build``), as a
    device byte buffer; built once and kept on the Csr object."""
    cached = getattr(csr, "_tgraph", None)
    if cached is not None:
        return cached
    dev = csr.rowptr.device
    L = load()
    buf = workspace(int(L.dawn_tgraph_bytes(csr.n, csr.m)), dev)
    scratch = workspace(int(L.dawn_tgraph_build_bytes(csr.n, csr.m)), dev)
    bp, bn = _aligned(buf)
    sp, sn = _aligned(scratch)
    w = None if csr.wtype == "unit" else _ptr(csr.w)  # unit graphs have no weight array
    _check(L.dawn_tgraph_build(_ptr(csr.rowptr), _ptr(csr.colidx), w, csr.n, csr.m,
                               bp, bn, sp, sn, _stream(stream)))
    _torch().cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    csr._tgraph = buf
    return buf


def umsssp_workspace_bytes(n: int, m: int, k: int) -> int:
    return int(load().dawn_umsssp_workspace_bytes(n, m, k))


def workspace_bytes(n: int, m: int, k: int, wtype: str = "u32") -> int:
    """Scratch bytes of the workspace-taking call for k sources of this weight
    type (``dawn_workspace_bytes``); 0 when no such call accepts them."""
    return int(load().dawn_workspace_bytes(n, m, k, wtype_code(wtype)))


def umsssp(csr: Csr, sources, out=None, stream=None, ws=None, info=None, tgraph=None,
           check: bool = True):
    """Hop counts from each source, every edge weight taken as 1
    (``dawn_umsssp_ws``): uint32 [k, n] tensor, row j = sources[j],
    0xFFFFFFFF where unreachable.  The weights of `csr` are not read.  With
    `tgraph` (from ``tgraph(csr)``) dense steps run as pull steps.  `check`
    as in ``sssp``."""
    torch = _torch()
    dev = csr.rowptr.device
    if not torch.is_tensor(sources):
        sources = torch.as_tensor(np.asarray(sources, dtype=np.int32), device=dev)
    sources = sources.to(device=dev, dtype=torch.int32).contiguous()
    k = int(sources.numel())
    if out is None:
        out = torch.empty((k, csr.n), dtype=torch.uint32, device=dev)
    if ws is None:
        ws = workspace(umsssp_workspace_bytes(csr.n, csr.m, k), dev)
    p, nb = _aligned(ws)
    tp = _aligned(tgraph)[0] if tgraph is not None else None
    L = load()
    _check(L.dawn_umsssp_ws(_ptr(csr.rowptr), _ptr(csr.colidx), csr.n, csr.m, tp, _ptr(sources),
                            k, _ptr(out), p, nb, _ptr(info), _stream(stream)))
    _finish(info, stream, check)
    return out


def msssp(csr: Csr, sources, out=None, stream=None, ws=None, info=None, tgraph=None,
          check: bool = True):
    """Distances from each source: [k, n] tensor, row j = sources[j].  With
    `tgraph` (from ``tgraph(csr)``) dense steps run as pull steps.  `check` as
    in ``sssp``."""
    torch = _torch()
    dev = csr.rowptr.device
    if not torch.is_tensor(sources):
        sources = torch.as_tensor(np.asarray(sources, dtype=np.int32), device=dev)
    sources = sources.to(device=dev, dtype=torch.int32).contiguous()
    k = int(sources.numel())
    if out is None:
        out = torch.empty((k, csr.n), dtype=dist_dtype(csr.wtype), device=dev)
    L = load()
    if tgraph is not None:
        if ws is None:
            ws = workspace(msssp_workspace_bytes(csr.n, csr.m, k), dev)
        p, nb = _aligned(ws)
        tp, _ = _aligned(tgraph)
        _check(L.dawn_msssp_tg_ws(*_csr_args(csr), tp, _ptr(sources), k, _ptr(out), p, nb,
                                  _ptr(info), _stream(stream)))
    elif ws is None and info is None:
        _check(L.dawn_msssp(*_csr_args(csr), _ptr(sources), k, _ptr(out), _stream(stream)))
    else:
        if ws is None:
            ws = workspace(msssp_workspace_bytes(csr.n, csr.m, k), dev)
        p, nb = _aligned(ws)
        _check(L.dawn_msssp_ws(*_csr_args(csr), _ptr(sources), k, _ptr(out), p, nb, _ptr(info),
                               _stream(stream)))
    _finish(info, stream, check)
    return out


def apsp(csr: Csr, out=None, stream=None, check: bool = True):
    """All pairs: [n, n] tensor, row s = distances from s.  `check` as in
    ``sssp``."""
    torch = _torch()
    if out is None:
        out = torch.empty((csr.n, csr.n), dtype=dist_dtype(csr.wtype), device=csr.rowptr.device)
    _check(load().dawn_apsp(*_csr_args(csr), _ptr(out), _stream(stream)))
    _finish(None, stream, check)
    return out


# ---------------------------------------------------------------------------
# many graphs in one launch
# ---------------------------------------------------------------------------

class Batch:
    """A disjoint union of CSR graphs of one weight type, solved in one launch."""

    def __init__(self, graphs: list[Csr], stream=None):
        if not graphs:
            raise ValueError("empty batch")
        wt = {g.wtype for g in graphs}
        if len(wt) != 1:
            raise DawnError(2, "mixed weight types in one batch")
        self.wtype = graphs[0].wtype
        self.count = len(graphs)
        L = load()
        arr = lambda vals, t: (t * len(vals))(*vals)
        rp = arr([g.rowptr.data_ptr() for g in graphs], _vp)
        ci = arr([g.colidx.data_ptr() for g in graphs], _vp)
        ww = arr([g.w.data_ptr() for g in graphs], _vp)
        ns = arr([g.n for g in graphs], _i32)
        ms = arr([g.m for g in graphs], _i32)
        h = _vp()
        _check(L.dawn_batch_create(ctypes.byref(h), self.count, rp, ci, ww, ns, ms,
                                   wtype_code(self.wtype), _stream(stream)))
        self._h = h
        tn, tm = _i64(), _i64()
        _check(L.dawn_batch_sizes(h, ctypes.byref(tn), ctypes.byref(tm)))
        self.total_n, self.total_m = int(tn.value), int(tm.value)
        self.offsets = [int(L.dawn_batch_vertex_offset(h, i)) for i in range(self.count)]
        self.sizes = [g.n for g in graphs]
        self.device = graphs[0].rowptr.device

    def run(self, sources, out=None, info=None, stream=None):
        """sources: int32 device tensor [count] of local source ids.
        Returns the concatenated distances [total_n]."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.total_n, dtype=dist_dtype(self.wtype), device=self.device)
        _check(load().dawn_batch_run(self._h, _ptr(sources), _ptr(out), _ptr(info),
                                     _stream(stream)))
        return out

    def capture(self, sources, out, info=None, stream=None):
        _check(load().dawn_batch_capture(self._h, _ptr(sources), _ptr(out), _ptr(info),
                                         _stream(stream)))

    def replay(self, stream=None):
        _check(load().dawn_batch_replay(self._h, _stream(stream)))

    def split(self, dist):
        return [dist[o:o + n] for o, n in zip(self.offsets, self.sizes)]

    def close(self):
        if getattr(self, "_h", None):
            load().dawn_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# tile sessions (continuous batching)
# ---------------------------------------------------------------------------

def tile_bytes(n: int, m: int, k: int) -> int:
    return int(load().dawn_tile_bytes(n, m, k))


class Tile:
    """Per-query distance state for up to k queries on one resident graph."""

    def __init__(self, csr: Csr, k: int, stream=None, ws=None):
        """ws: the session's device memory (a buffer from ``workspace`` of at
        least ``tile_bytes(n, m, k)``); allocated here when None.  The buffer is
        kept referenced while the session lives."""
        self.csr = csr
        self.k = int(k)
        if ws is None:
            ws = workspace(tile_bytes(csr.n, csr.m, self.k), csr.rowptr.device)
        self.ws = ws
        p, nb = _aligned(ws)
        h = _vp()
        _check(load().dawn_tile_create(ctypes.byref(h), *_csr_args(csr), self.k, p, nb,
                                       _stream(stream)))
        self._h = h
        torch = _torch()
        # zeroed on the session's stream, ordered before its first run
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            self.done_buf = torch.zeros((self.k + 31) // 32, dtype=torch.int32,
                                        device=csr.rowptr.device)

    def set_tgraph(self, tgraph):
        """Attach the reverse graph (``tgraph(csr)``) for pull steps, or None."""
        self._tgraph = tgraph  # kept alive while attached
        _check(load().dawn_tile_set_tgraph(self._h, _aligned(tgraph)[0] if tgraph is not None
                                           else None))

    def admit(self, col: int, source: int, stream=None):
        _check(load().dawn_tile_admit(self._h, int(col), int(source), _stream(stream)))

    def run(self, max_steps: int, stream=None):
        """Enqueue up to max_steps steps; the done bits land in self.done_buf."""
        _check(load().dawn_tile_run(self._h, int(max_steps), _ptr(self.done_buf),
                                    _stream(stream)))
        return self.done_buf

    def capture(self, max_steps: int):
        """Capture run(max_steps) once as a HIP graph (done bits to self.done_buf)."""
        _check(load().dawn_tile_capture(self._h, int(max_steps), _ptr(self.done_buf)))

    def replay(self, stream=None):
        """Enqueue the captured run; returns self.done_buf."""
        _check(load().dawn_tile_replay(self._h, _stream(stream)))
        return self.done_buf

    def read(self, col: int, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.csr.n, dtype=dist_dtype(self.csr.wtype),
                              device=self.csr.rowptr.device)
        _check(load().dawn_tile_read(self._h, int(col), _ptr(out), _stream(stream)))
        return out

    def steps(self, stream=None):
        torch = _torch()
        out = torch.empty(self.k, dtype=torch.int32, device=self.csr.rowptr.device)
        _check(load().dawn_tile_steps(self._h, _ptr(out), _stream(stream)))
        return out

    def evict(self, col: int, stream=None):
        _check(load().dawn_tile_evict(self._h, int(col), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            load().dawn_tile_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_query() -> dict:
    """Compute units, cooperative-launch support and persistent-kernel
    occupancy of the current device (see dawn_device_query)."""
    out = (_i32 * DEVICE_QUERY_LEN)()
    _check(load().dawn_device_query(out))
    keys = ("cus", "coop", "ss_blocks_per_cu", "tile_blocks_per_cu", "ss_grid", "tile_grid",
            "device", "wg_threads", "ss_vgprs", "ss_lds", "ss_api_blocks_per_cu", "tile_vgprs",
            "tile_lds", "tile_api_blocks_per_cu", "utile_blocks_per_cu", "utile_vgprs")
    return dict(zip(keys, list(out)))


def kernel_timer(enable: bool):
    """Start (clearing earlier records) or stop the library's kernel timer."""
    _check(load().dawn_kernel_timer(1 if enable else 0))


def kernel_time() -> tuple[float, int]:
    """(summed milliseconds, launches) of the main GOVM launches recorded."""
    ms = ctypes.c_double()
    n = _i32()
    _check(load().dawn_kernel_time(ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


def done_columns(done_words, k: int) -> list[int]:
    """Decode done bits (int32 words) into column indices."""
    w = np.asarray(done_words, dtype=np.int64) & 0xFFFFFFFF
    return [j for j in range(k) if (int(w[j >> 5]) >> (j & 31)) & 1]
