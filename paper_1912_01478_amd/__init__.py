"""IPGC graph coloring on MI355X (gfx950): Python binding of the C-ABI library ``libipgc.so``.

The method is Section II-C of Rai, M P, Pai, "A Hybrid Graph Coloring Algorithm for GPUs"
(arXiv 1912.01478), run under the hybrid schedule of Section IV.  Every step of the coloring
runs in the library's HIP kernels; this module only checks and marshals arguments.  PyTorch
supplies device memory and streams.  There is no CPU fallback: if the library is missing the
import of :func:`library` raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
# The library this package loads: the in-tree build, unless IPGC_LIBRARY names another build of the
# same sources (for comparing builds side by side).
LIB_PATH = os.environ.get("IPGC_LIBRARY") or os.path.join(HERE, "libipgc.so")

MODE_TOPOLOGY = 0
MODE_DATA = 1
MODE_HYBRID = 2
MODE_REBUILD = 3
MODES = {"topology": MODE_TOPOLOGY, "data": MODE_DATA, "hybrid": MODE_HYBRID, "rebuild": MODE_REBUILD}

VALIDATE_DEFAULT = 0
VALIDATE_NONE = 1
VALIDATE_RANGES = 2
VALIDATE_FULL = 3

# Size of the static device array that ipgc_color_graph_noalloc carves its workspace from
# (IPGC_NOALLOC_SCRATCH_BYTES in include/ipgc.h).
NOALLOC_SCRATCH_BYTES = 256 << 20

OK, EINVAL, ETOOBIG, EBADCSR, ENOMEM, EHIP, ELIMIT, ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7
STATUS = {0: "IPGC_OK", -1: "IPGC_EINVAL", -2: "IPGC_ETOOBIG", -3: "IPGC_EBADCSR", -4: "IPGC_ENOMEM",
          -5: "IPGC_EHIP", -6: "IPGC_ELIMIT", -7: "IPGC_ECANCELED"}

# Every symbol the header declares; the tests check that the library exports all of them.
EXPORTS = ("ipgc_color_graph", "ipgc_color_graph_ex", "ipgc_color_graph_noalloc", "ipgc_color_graphs_batched",
           "ipgc_last_error",
           "ipgc_kernel_name", "ipgc_unit_name", "ipgc_version", "ipgc_release_workspaces", "ipgc_server_create",
           "ipgc_server_submit", "ipgc_server_step", "ipgc_server_poll", "ipgc_server_stats_get",
           "ipgc_server_destroy", "ipgc_server_wait", "ipgc_server_cancel", "ipgc_set_allocator",
           "ipgc_push_microbench", "ipgc_bfs")
FLAG_STEPPED = 1
FLAG_LIGHT_PULL = 2
FLAG_LIGHT_PUSH = 4
FLAG_RACY = 8
FLAG_PER_GRAPH = 16
LIGHT = {"auto": 0, "pull": FLAG_LIGHT_PULL, "push": FLAG_LIGHT_PUSH}
PROFILE_KINDS = 16


class IpgcError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, message))
        self.code = code


class Profile(ctypes.Structure):
    """Mirror of ``ipgc_profile``."""
    _fields_ = [("mask", ctypes.c_uint32), ("kinds", ctypes.c_int32),
                ("ms", ctypes.c_double * PROFILE_KINDS), ("launches", ctypes.c_int64 * PROFILE_KINDS),
                ("unit_kinds", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("units", ctypes.c_int64 * PROFILE_KINDS), ("phase_ticks", ctypes.POINTER(ctypes.c_uint64)),
                ("phase_capacity", ctypes.c_int64), ("phase_recorded", ctypes.c_int64),
                ("tick_khz", ctypes.c_int64)]

    def as_dict(self) -> dict:
        lib = library()
        kernels = {lib.ipgc_kernel_name(k).decode(): {"ms": self.ms[k], "launches": self.launches[k]}
                   for k in range(self.kinds)}
        units = {lib.ipgc_unit_name(k).decode(): self.units[k] for k in range(self.unit_kinds)}
        out = {"kernels": kernels, "units": units}
        if self.phase_recorded:
            out["phase_ticks"] = [self.phase_ticks[i] for i in range(self.phase_recorded)]
            out["tick_khz"] = self.tick_khz
        return out


class Options(ctypes.Structure):
    """Mirror of ``ipgc_options``."""
    _fields_ = [("threshold", ctypes.c_int64), ("light_max_degree", ctypes.c_int32),
                ("hub_min_degree", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("profile", ctypes.POINTER(Profile)), ("workgroups", ctypes.c_int32),
                ("tail_workgroups", ctypes.c_int32), ("barrier_timeout_ms", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    """Mirror of ``ipgc_server_config``."""
    _fields_ = [("node_capacity", ctypes.c_int64), ("edge_capacity", ctypes.c_int64), ("max_jobs", ctypes.c_int32),
                ("rounds_per_step", ctypes.c_int32), ("mode", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("options", Options)]


class JobResult(ctypes.Structure):
    """Mirror of ``ipgc_job_result``."""
    _fields_ = [("job_id", ctypes.c_int64), ("status", ctypes.c_int32), ("rounds", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    """Mirror of ``ipgc_server_stats``."""
    _fields_ = [(k, ctypes.c_int64) for k in ("steps", "cancelled", "rounds", "submitted", "admitted", "completed",
                                              "resident",
                                              "queued", "resident_nodes", "resident_edges", "peak_resident",
                                              "arena_bytes")] + [("units", ctypes.c_int64 * 16)]


class Trace(ctypes.Structure):
    """Mirror of ``ipgc_trace``."""
    _fields_ = [("capacity", ctypes.c_int64), ("wl_size", ctypes.POINTER(ctypes.c_int32)),
                ("wl_degree", ctypes.POINTER(ctypes.c_int64)),
                ("topology", ctypes.POINTER(ctypes.c_int8)), ("recorded", ctypes.c_int64),
                ("topo_graphs", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def library() -> ctypes.CDLL:
    """Load ``libipgc.so`` (built by ``build.py``); raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("HIP library %s is missing: run __graft_entry__.build() first" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.ipgc_color_graph.restype = i32
        lib.ipgc_color_graph.argtypes = [vp, vp, i64, i64, i32, vp, ctypes.POINTER(ctypes.c_int32)]
        lib.ipgc_color_graph_ex.restype = i32
        lib.ipgc_color_graph_ex.argtypes = [vp, vp, i64, i64, i32, ctypes.POINTER(Options), vp, vp,
                                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Trace)]
        lib.ipgc_color_graph_noalloc.restype = i32
        lib.ipgc_color_graph_noalloc.argtypes = [vp, vp, i64, i64, i32, ctypes.POINTER(Options), vp, vp,
                                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Trace)]
        lib.ipgc_color_graphs_batched.restype = i32
        lib.ipgc_color_graphs_batched.argtypes = [i64, vp, vp, vp, vp, i32, ctypes.POINTER(Options), vp, vp, vp,
                                                  ctypes.POINTER(Trace)]
        srv = ctypes.c_void_p
        lib.ipgc_server_create.restype = i32
        lib.ipgc_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(srv)]
        lib.ipgc_server_submit.restype = i32
        lib.ipgc_server_submit.argtypes = [srv, vp, vp, i64, i64, vp, ctypes.POINTER(ctypes.c_int64)]
        lib.ipgc_server_step.restype = i32
        lib.ipgc_server_step.argtypes = [srv]
        lib.ipgc_server_poll.restype = i32
        lib.ipgc_server_poll.argtypes = [srv, ctypes.POINTER(JobResult), i64, ctypes.POINTER(ctypes.c_int64)]
        lib.ipgc_server_stats_get.restype = i32
        lib.ipgc_server_stats_get.argtypes = [srv, ctypes.POINTER(ServerStats)]
        lib.ipgc_server_destroy.restype = None
        lib.ipgc_server_destroy.argtypes = [srv]
        lib.ipgc_server_wait.restype = i32
        lib.ipgc_server_wait.argtypes = [srv, i64, ctypes.POINTER(JobResult)]
        lib.ipgc_server_cancel.restype = i32
        lib.ipgc_server_cancel.argtypes = [srv, i64]
        lib.ipgc_set_allocator.restype = i32
        lib.ipgc_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
        lib.ipgc_bfs.restype = i32
        lib.ipgc_bfs.argtypes = [vp, vp, i64, i64, i64, i32, ctypes.POINTER(Options), vp, vp,
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Trace)]
        lib.ipgc_push_microbench.restype = i32
        lib.ipgc_push_microbench.argtypes = [i64, i32, i32, i32, vp, vp, i64, ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_int64)]
        lib.ipgc_last_error.restype = ctypes.c_char_p
        lib.ipgc_last_error.argtypes = []
        lib.ipgc_kernel_name.restype = ctypes.c_char_p
        lib.ipgc_kernel_name.argtypes = [i32]
        lib.ipgc_unit_name.restype = ctypes.c_char_p
        lib.ipgc_unit_name.argtypes = [i32]
        lib.ipgc_version.restype = i32
        lib.ipgc_version.argtypes = []
        lib.ipgc_release_workspaces.restype = None
        lib.ipgc_release_workspaces.argtypes = []
        _lib = lib
        atexit.register(_release_at_exit)
    return _lib


# Device memory hook (ipgc_set_allocator): alloc(bytes, device, user) -> pointer or NULL,
# free(ptr, bytes, device, user).
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p)
_hooks = []  # every callback pair ever installed stays alive: memory it gave is returned through it


def set_allocator(alloc=None, free=None) -> None:
    """Route the library's device allocations (workspaces, server arenas) through Python
    callables: ``alloc(nbytes, device) -> int`` returns a device pointer (0 for failure, which
    the library reports as IPGC_ENOMEM); ``free(ptr, nbytes, device)`` takes one back.  Both
    None restores hipMalloc / hipFree.  Memory goes back to the pair that gave it."""
    lib = library()
    if (alloc is None) != (free is None):
        raise ValueError("set_allocator takes both callables or neither")
    if alloc is None:
        _check(lib.ipgc_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return

    def _alloc(nbytes, device, _user):
        try:
            return int(alloc(int(nbytes), int(device)) or 0) or None
        except Exception:
            return None

    def _free(ptr, nbytes, device, _user):
        try:
            free(int(ptr), int(nbytes), int(device))
        except Exception:
            pass

    pair = (ALLOC_FN(_alloc), FREE_FN(_free))
    _hooks.append(pair)
    _check(lib.ipgc_set_allocator(pair[0], pair[1], None))


def torch_allocator():
    """(alloc, free) callables that take the library's device memory from PyTorch's caching
    allocator, for ``set_allocator``."""
    import torch

    def alloc(nbytes, device):
        return torch.cuda.caching_allocator_alloc(nbytes, device)

    def free(ptr, nbytes, device):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


_servers = weakref.WeakSet()  # open servers, closed before the process exits


def _release_at_exit():
    """Returns the device memory, pinned host memory and events the library holds before the
    interpreter, the HIP runtime and any profiler loaded into the process shut down."""
    for srv in list(_servers):
        try:
            srv.close()
        except Exception:
            pass
    if _lib is not None:
        try:
            _lib.ipgc_release_workspaces()
            _lib.ipgc_set_allocator(ALLOC_FN(), FREE_FN(), None)
        except Exception:
            pass


def _check(rc: int):
    if rc != 0:
        raise IpgcError(rc, library().ipgc_last_error().decode(errors="replace"))


@dataclass
class Coloring:
    colors: "object"   # torch.int32 tensor on the device, 1-based colors
    rounds: int
    wl_sizes: list | None = None    # |WL_r| per round, when requested
    wl_degrees: list | None = None  # degree sum over WL_r per round, when requested
    topology: list | None = None    # 1 for topology-driven rounds, when requested
    profile: dict | None = None     # per-kernel-kind event times and work units, when requested

    @property
    def num_colors(self) -> int:
        return int(self.colors.max().item()) if self.colors.numel() else 0


def _mode(mode) -> int:
    if isinstance(mode, str):
        return MODES[mode.lower()]
    return int(mode)


TRACE_CAPACITY = 1 << 20  # rounds recorded at most per traced call


class _Call:
    """Marshalled options, optional profile and optional trace of one library call."""

    def __init__(self, threshold, light_max_degree, hub_min_degree, validate, stepped, trace, trace_cap,
                 profile_mask, timeline, workgroups=0, light="auto", racy=False, tail_workgroups=0,
                 barrier_timeout_ms=0, per_graph=False):
        self.prof = None
        if profile_mask or timeline:
            self.prof = Profile(int(profile_mask))
            if timeline:
                self._ticks = (ctypes.c_uint64 * int(timeline))()
                self.prof.phase_ticks = ctypes.cast(self._ticks, ctypes.POINTER(ctypes.c_uint64))
                self.prof.phase_capacity = int(timeline)
        self.opts = Options(int(threshold), int(light_max_degree), int(hub_min_degree), int(validate),
                            (FLAG_STEPPED if stepped else 0) | LIGHT[light] | (FLAG_RACY if racy else 0) |
                            (FLAG_PER_GRAPH if per_graph else 0),
                            ctypes.pointer(self.prof) if self.prof is not None else None, int(workgroups),
                            int(tail_workgroups), int(barrier_timeout_ms), 0)
        self.tr = None
        if trace:
            cap = max(1, min(int(trace_cap), TRACE_CAPACITY))
            self._wl = (ctypes.c_int32 * cap)()
            self._wd = (ctypes.c_int64 * cap)()
            self._topo = (ctypes.c_int8 * cap)()
            self._tg = (ctypes.c_int32 * cap)() if per_graph else None
            self.tr = Trace(cap, ctypes.cast(self._wl, ctypes.POINTER(ctypes.c_int32)),
                            ctypes.cast(self._wd, ctypes.POINTER(ctypes.c_int64)),
                            ctypes.cast(self._topo, ctypes.POINTER(ctypes.c_int8)), 0,
                            ctypes.cast(self._tg, ctypes.POINTER(ctypes.c_int32)) if per_graph else None)

    def trace_ref(self):
        return ctypes.byref(self.tr) if self.tr is not None else None

    def finish(self, res):
        if self.tr is not None:
            k = self.tr.recorded
            res.wl_sizes = list(self._wl[:k])
            res.wl_degrees = list(self._wd[:k])
            res.topology = list(self._topo[:k])
            if self._tg is not None:
                res.topo_graphs = list(self._tg[:k])
        if self.prof is not None:
            res.profile = self.prof.as_dict()
        return res


def color_graph(rowptr, colidx, mode="hybrid", *, threshold: int = 0, light_max_degree: int = 0,
                hub_min_degree: int = 0, validate: int = VALIDATE_DEFAULT, stepped: bool = False, out=None,
                stream=None, trace: bool = False, profile_mask: int = 0, timeline: int = 0,
                workgroups: int = 0, light: str = "auto", racy: bool = False,
                tail_workgroups: int = 0, barrier_timeout_ms: int = 0) -> Coloring:
    """Color the symmetric CSR graph (``rowptr``: int32[n+1], ``colidx``: int32[m], both on the
    HIP device) and return the 1-based colors and round count.  ``mode`` is "topology", "data"
    or "hybrid"; ``threshold`` is H for hybrid rounds (0: floor(6n/10)).  ``stepped`` runs one
    launch per round step instead of one cooperative launch.  Options only change the time,
    never the result.  ``trace`` returns the per-round worklist sizes and degree sums;
    ``profile_mask`` times the selected kernel kinds with HIP events (bit k = kind k); ``timeline``
    > 0 records that many device wall-clock ticks at the round-step boundaries; ``workgroups`` sets
    the round kernels' workgroup count (0: automatic) and ``tail_workgroups`` how many of them stay
    for the small data-driven rounds at the end (0: default, negative: all); ``light`` is "pull",
    "push" or "auto" (how nodes of degree <= light_max_degree learn their neighbours' colors);
    ``racy`` selects the in-place mode (a proper coloring that depends on timing, not the
    synchronous one); ``barrier_timeout_ms`` bounds every grid-barrier wait (0: 60 s; -1: give up
    at once, which exercises the error path).  ``validate`` is VALIDATE_NONE, _RANGES (default) or
    _FULL (also a simple symmetric graph)."""
    import torch

    if rowptr.dtype != torch.int32 or colidx.dtype != torch.int32:
        raise TypeError("rowptr and colidx must be int32")
    if not (rowptr.is_cuda and colidx.is_cuda):
        raise ValueError("rowptr and colidx must be device tensors")
    rowptr = rowptr.contiguous()
    colidx = colidx.contiguous()
    n = rowptr.numel() - 1
    m = colidx.numel()
    if n < 0:
        raise ValueError("rowptr needs n+1 >= 1 entries")
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=rowptr.device)
    elif out.dtype != torch.int32 or out.numel() != n or not out.is_contiguous() or out.device != rowptr.device:
        raise ValueError("out must be a contiguous int32 tensor of n entries on the graph's device")
    call = _Call(threshold, light_max_degree, hub_min_degree, validate, stepped, trace, n, profile_mask, timeline,
                 workgroups, light, racy, tail_workgroups, barrier_timeout_ms)
    rounds = ctypes.c_int32(-1)
    if stream is None:
        stream = torch.cuda.current_stream(rowptr.device)
    with torch.cuda.device(rowptr.device):
        rc = library().ipgc_color_graph_ex(
            ctypes.c_void_p(rowptr.data_ptr()), ctypes.c_void_p(colidx.data_ptr() if m else 0), n, m,
            _mode(mode), ctypes.byref(call.opts), ctypes.c_void_p(stream.cuda_stream),
            ctypes.c_void_p(out.data_ptr() if n else 0), ctypes.byref(rounds), call.trace_ref())
    _check(rc)
    return call.finish(Coloring(out, rounds.value))


def color_graph_raw(rowptr_ptr: int, colidx_ptr: int, n: int, m: int, mode: int, out_ptr: int) -> int:
    """The plain entry point ``ipgc_color_graph`` on raw device pointers; returns the round count."""
    rounds = ctypes.c_int32(-1)
    rc = library().ipgc_color_graph(ctypes.c_void_p(rowptr_ptr), ctypes.c_void_p(colidx_ptr), n, m, int(mode),
                                    ctypes.c_void_p(out_ptr), ctypes.byref(rounds))
    _check(rc)
    return rounds.value


def color_graph_noalloc(rowptr, colidx, mode="hybrid", *, out, stream=None, threshold: int = 0,
                        light_max_degree: int = 0, hub_min_degree: int = 0, validate: int = VALIDATE_DEFAULT,
                        stepped: bool = False, trace: bool = False, workgroups: int = 0, light: str = "auto",
                        racy: bool = False, tail_workgroups: int = 0) -> Coloring:
    """``color_graph`` through ``ipgc_color_graph_noalloc``: the library allocates no device memory
    (its workspace is a static array of NOALLOC_SCRATCH_BYTES per GPU), so ``out`` (int32[n] on
    the graph's device) must be given.  A graph whose workspace does not fit raises IPGC_ETOOBIG.
    No profile; other arguments as for ``color_graph``."""
    import torch

    if rowptr.dtype != torch.int32 or colidx.dtype != torch.int32:
        raise TypeError("rowptr and colidx must be int32")
    if not (rowptr.is_cuda and colidx.is_cuda):
        raise ValueError("rowptr and colidx must be device tensors")
    if not (rowptr.is_contiguous() and colidx.is_contiguous()):
        raise ValueError("rowptr and colidx must be contiguous (a copy would allocate)")
    n = rowptr.numel() - 1
    m = colidx.numel()
    if n < 0:
        raise ValueError("rowptr needs n+1 >= 1 entries")
    if out.dtype != torch.int32 or out.numel() != n or not out.is_contiguous() or out.device != rowptr.device:
        raise ValueError("out must be a contiguous int32 tensor of n entries on the graph's device")
    call = _Call(threshold, light_max_degree, hub_min_degree, validate, stepped, trace, n, 0, 0, workgroups, light,
                 racy, tail_workgroups)
    rounds = ctypes.c_int32(-1)
    if stream is None:
        stream = torch.cuda.current_stream(rowptr.device)
    with torch.cuda.device(rowptr.device):
        rc = library().ipgc_color_graph_noalloc(
            ctypes.c_void_p(rowptr.data_ptr()), ctypes.c_void_p(colidx.data_ptr() if m else 0), n, m,
            _mode(mode), ctypes.byref(call.opts), ctypes.c_void_p(stream.cuda_stream),
            ctypes.c_void_p(out.data_ptr() if n else 0), ctypes.byref(rounds), call.trace_ref())
    _check(rc)
    return call.finish(Coloring(out, rounds.value))


def pack_graphs(graphs):
    """Pack host CSR graphs [(rowptr int32[n+1], colidx int32[m]), ...] into the batched layout:
    returns (node_off int64[G+1], edge_off int64[G+1], rowptr_packed int32[N+G],
    colidx_packed int32[M]) as numpy arrays."""
    import numpy as np

    ns = np.array([len(rp) - 1 for rp, _ in graphs], dtype=np.int64)
    ms = np.array([len(ci) for _, ci in graphs], dtype=np.int64)
    node_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    edge_off = np.concatenate([[0], np.cumsum(ms)]).astype(np.int64)
    rowptr_packed = np.concatenate([np.asarray(rp, dtype=np.int32) for rp, _ in graphs]) if graphs else \
        np.zeros(0, dtype=np.int32)
    colidx_packed = np.concatenate([np.asarray(ci, dtype=np.int32) for _, ci in graphs]) if graphs else \
        np.zeros(0, dtype=np.int32)
    return node_off, edge_off, rowptr_packed, colidx_packed


@dataclass
class BatchColoring:
    colors: "object"   # torch.int32 tensor on the device: graph g's colors at node_off[g]:node_off[g+1]
    rounds: list       # rounds per graph
    node_off: "object"
    wl_sizes: list | None = None    # per round of the batch: size of the union of the worklists
    wl_degrees: list | None = None  # per round of the batch: degree sum over that union
    topology: list | None = None
    profile: dict | None = None
    topo_graphs: list | None = None  # per-graph schedules: graphs run topology-driven per round

    def graph(self, g: int):
        return self.colors[int(self.node_off[g]):int(self.node_off[g + 1])]


def color_graphs_batched(rowptr_packed, colidx_packed, node_off, edge_off, mode="hybrid", *, threshold: int = 0,
                         light_max_degree: int = 0, hub_min_degree: int = 0, validate: int = VALIDATE_DEFAULT,
                         stepped: bool = False, out=None, stream=None, trace: bool = False,
                         profile_mask: int = 0, workgroups: int = 0, light: str = "auto",
                         racy: bool = False, tail_workgroups: int = 0, barrier_timeout_ms: int = 0,
                         timeline: int = 0, per_graph: bool = False) -> BatchColoring:
    """Color many graphs in one launch.  ``rowptr_packed`` (int32[N+G]) and ``colidx_packed``
    (int32[M]) are device tensors in the layout of ``pack_graphs``; ``node_off`` and ``edge_off``
    (G+1 int64 each) are host arrays.  Each graph gets the coloring and round count it gets alone.
    ``trace``, ``profile_mask`` and ``timeline`` are as for ``color_graph``, over the rounds of the
    whole batch.  ``per_graph`` lets every graph take its own schedule decision (H_g, the
    ``threshold`` scaled to its node count; ``IPGC_FLAG_PER_GRAPH``); with ``trace`` the result
    then also holds the number of graphs that ran each round topology-driven."""
    import numpy as np
    import torch

    node_off = np.ascontiguousarray(node_off, dtype=np.int64)
    edge_off = np.ascontiguousarray(edge_off, dtype=np.int64)
    G = len(node_off) - 1
    N = int(node_off[-1]) if G >= 0 else 0
    if rowptr_packed.dtype != torch.int32 or colidx_packed.dtype != torch.int32:
        raise TypeError("rowptr_packed and colidx_packed must be int32")
    if not (rowptr_packed.is_cuda and colidx_packed.is_cuda):
        raise ValueError("rowptr_packed and colidx_packed must be device tensors")
    if rowptr_packed.numel() != N + G:
        raise ValueError("rowptr_packed needs N + G = %d entries" % (N + G))
    if colidx_packed.numel() != int(edge_off[-1]):
        raise ValueError("colidx_packed needs edge_off[G] entries")
    rowptr_packed = rowptr_packed.contiguous()
    colidx_packed = colidx_packed.contiguous()
    dev = rowptr_packed.device
    if out is None:
        out = torch.empty(N, dtype=torch.int32, device=dev)
    elif out.dtype != torch.int32 or out.numel() != N or not out.is_contiguous() or out.device != dev:
        raise ValueError("out must be a contiguous int32 tensor of N entries on the batch's device")
    call = _Call(threshold, light_max_degree, hub_min_degree, validate, stepped, trace, N, profile_mask, timeline,
                 workgroups, light, racy, tail_workgroups, barrier_timeout_ms, per_graph)
    rounds = np.full(max(G, 1), -1, dtype=np.int32)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        rc = library().ipgc_color_graphs_batched(
            G, node_off.ctypes.data_as(ctypes.c_void_p), edge_off.ctypes.data_as(ctypes.c_void_p),
            ctypes.c_void_p(rowptr_packed.data_ptr()), ctypes.c_void_p(colidx_packed.data_ptr()),
            _mode(mode), ctypes.byref(call.opts), ctypes.c_void_p(stream.cuda_stream),
            ctypes.c_void_p(out.data_ptr() if N else 0), rounds.ctypes.data_as(ctypes.c_void_p), call.trace_ref())
    _check(rc)
    return call.finish(BatchColoring(out, rounds[:G].tolist(), node_off))


@dataclass
class BfsResult:
    dist: "object"      # torch.int32 tensor on the device: hops from the source, -1 if unreachable
    levels: int         # non-empty frontiers
    frontier_sizes: list | None = None
    topology: list | None = None


def bfs(rowptr, colidx, source: int, mode="hybrid", *, threshold: int = 0, workgroups: int = 0,
        validate: int = VALIDATE_DEFAULT, out=None, stream=None, trace: bool = False,
        barrier_timeout_ms: int = 0) -> BfsResult:
    """Breadth-first search from `source` on the device CSR under the keep-the-worklist hybrid
    schedule (``ipgc_bfs``)."""
    import torch

    if rowptr.dtype != torch.int32 or colidx.dtype != torch.int32:
        raise TypeError("rowptr and colidx must be int32")
    n, m = rowptr.numel() - 1, colidx.numel()
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=rowptr.device)
    call = _Call(threshold, 0, 0, validate, False, trace, max(n, 1), 0, 0, workgroups,
                 barrier_timeout_ms=barrier_timeout_ms)
    levels = ctypes.c_int32(-1)
    if stream is None:
        stream = torch.cuda.current_stream(rowptr.device)
    with torch.cuda.device(rowptr.device):
        rc = library().ipgc_bfs(ctypes.c_void_p(rowptr.data_ptr()), ctypes.c_void_p(colidx.data_ptr() if m else 0),
                                n, m, int(source), _mode(mode), ctypes.byref(call.opts),
                                ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(out.data_ptr() if n else 0),
                                ctypes.byref(levels), call.trace_ref())
    _check(rc)
    res = BfsResult(out, levels.value)
    if call.tr is not None:
        k = call.tr.recorded
        res.frontier_sizes = list(call._wl[:k])
        res.topology = list(call._topo[:k])
    return res


def push_microbench(n: int, count: int = 1000, nowl: bool = False, atomic: bool = False):
    """Worklist push micro-benchmark (``ipgc_push_microbench``) on the current device.  Returns
    (tti_us, sizes): the time of every non-empty iteration in microseconds and the worklist size
    at its start."""
    import numpy as np
    import torch  # noqa: F401  (the device context belongs to torch's current device)

    cap = (n + count - 1) // count + 2
    ticks = np.zeros(cap, dtype=np.uint64)
    sizes = np.zeros(cap, dtype=np.int32)
    iters = ctypes.c_int64(0)
    khz = ctypes.c_int64(0)
    _check(library().ipgc_push_microbench(int(n), int(count), int(bool(nowl)), int(bool(atomic)),
                                          ticks.ctypes.data_as(ctypes.c_void_p), sizes.ctypes.data_as(ctypes.c_void_p),
                                          cap, ctypes.byref(iters), ctypes.byref(khz)))
    k = iters.value
    tti = np.diff(ticks[:k + 1].astype(np.float64)) / khz.value * 1000.0
    return tti, sizes[:k].copy()


# ---------------------------------------------------------------- serving

# Device bytes per arena node slot and per CSR entry slot of a server (see ipgc_server_create):
# per node: row start 8, graph base/index 8, state 4, color mask 8, pending positions 4, class 1,
# ring start/length 8, static list 4, staging 4, both segmented lists 24; per entry: column id 4,
# ring 4, byte map 1.
SERVER_NODE_BYTES = 73
SERVER_ENTRY_BYTES = 9


@dataclass
class JobDone:
    job_id: int
    status: int        # 0, or a negative ipgc_status
    rounds: int
    colors: "object"   # numpy int32 array of the job's colors (None on error)


class Server:
    """A device-resident job server with continuous batching (``ipgc_server_*``).  Jobs are host
    CSR arrays; ``step()`` admits queued jobs that fit, runs ``rounds_per_step`` rounds over every
    resident job and retires finished ones; ``poll()`` returns the finished jobs."""

    def __init__(self, node_capacity: int, edge_capacity: int, max_jobs: int = 4096, rounds_per_step: int = 0,
                 mode="hybrid", threshold: int = 0, light_max_degree: int = 0, hub_min_degree: int = 0,
                 workgroups: int = 0, light: str = "auto", racy: bool = False, tail_workgroups: int = 0,
                 validate: int = VALIDATE_DEFAULT, barrier_timeout_ms: int = 0):
        opts = Options(int(threshold), int(light_max_degree), int(hub_min_degree), int(validate),
                       LIGHT[light] | (FLAG_RACY if racy else 0), None, int(workgroups), int(tail_workgroups),
                       int(barrier_timeout_ms), 0)
        cfg = ServerConfig(int(node_capacity), int(edge_capacity), int(max_jobs), int(rounds_per_step), _mode(mode),
                           0, opts)
        self._h = ctypes.c_void_p()
        _check(library().ipgc_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._jobs = {}  # job id -> (rowptr, colidx, out) kept alive until the job is polled
        _servers.add(self)

    @staticmethod
    def capacity_for(budget_bytes: int, avg_degree: float):
        """Node and entry capacities that fill about budget_bytes for jobs of the given average degree."""
        nodes = int(budget_bytes / (SERVER_NODE_BYTES + SERVER_ENTRY_BYTES * avg_degree))
        return nodes, int(nodes * avg_degree)

    def submit(self, rowptr, colidx) -> int:
        import numpy as np
        rp = np.ascontiguousarray(rowptr, dtype=np.int32)
        ci = np.ascontiguousarray(colidx, dtype=np.int32)
        n = rp.size - 1
        out = np.empty(max(n, 0), dtype=np.int32)
        jid = ctypes.c_int64(-1)
        _check(library().ipgc_server_submit(self._h, rp.ctypes.data_as(ctypes.c_void_p),
                                            ci.ctypes.data_as(ctypes.c_void_p), n, ci.size,
                                            out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(jid)))
        self._jobs[jid.value] = (rp, ci, out)
        return jid.value

    def step(self) -> None:
        _check(library().ipgc_server_step(self._h))

    def poll(self) -> list:
        res = (JobResult * 256)()
        out = []
        while True:
            cnt = ctypes.c_int64(0)
            _check(library().ipgc_server_poll(self._h, res, 256, ctypes.byref(cnt)))
            for i in range(cnt.value):
                r = res[i]
                _, _, colors = self._jobs.pop(r.job_id)
                out.append(JobDone(r.job_id, r.status, r.rounds, colors if r.status == 0 else None))
            if cnt.value < 256:
                return out

    def wait(self, job_id: int) -> JobDone:
        """Runs steps until job ``job_id`` finishes and returns its result (which poll() then
        no longer reports)."""
        r = JobResult()
        _check(library().ipgc_server_wait(self._h, int(job_id), ctypes.byref(r)))
        _, _, colors = self._jobs.pop(r.job_id)
        return JobDone(r.job_id, r.status, r.rounds, colors if r.status == 0 else None)

    def cancel(self, job_id: int) -> None:
        """Cancels an unfinished job; it is reported with status ECANCELED."""
        _check(library().ipgc_server_cancel(self._h, int(job_id)))

    def stats(self) -> dict:
        st = ServerStats()
        _check(library().ipgc_server_stats_get(self._h, ctypes.byref(st)))
        d = {k: getattr(st, k) for k, _ in ServerStats._fields_ if k != "units"}
        d["units"] = {library().ipgc_unit_name(k).decode(): st.units[k] for k in range(16)
                      if library().ipgc_unit_name(k)}
        return d

    def close(self) -> None:
        if self._h:
            library().ipgc_server_destroy(self._h)
            self._h = ctypes.c_void_p()
        _servers.discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


from . import autotune  # noqa: E402  (options search; imports nothing heavy at load time)
