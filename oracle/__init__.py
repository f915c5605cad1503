"""CPU oracle for IPGC -- test infrastructure only.

Plain single-threaded C (``ipgc_oracle.c``) that defines the coloring the GPU library must
reproduce bit for bit: Section II-C of Rai, M P, Pai, "A Hybrid Graph Coloring Algorithm for
GPUs" (arXiv 1912.01478), with the readings stated at the top of the C file.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import this package; the product path
(``paper_1912_01478_amd``) never imports it and shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ipgc_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "bfs_oracle.c")]
_LIB = os.path.join(_HERE, "libipgc_oracle.so")
_lib = None

_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, no OpenMP: it is single-threaded by design)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.ipgc_oracle_color.restype = ctypes.c_int
        lib.ipgc_oracle_color.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, vp, vp, vp,
                                          ctypes.c_int64, vp, vp, vp, ctypes.c_int64]
        lib.ipgc_oracle_bfs.restype = ctypes.c_int
        lib.ipgc_oracle_bfs.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int64, vp, vp, ctypes.c_int64, vp]
        lib.ipgc_oracle_first_free_color.restype = ctypes.c_int32
        lib.ipgc_oracle_first_free_color.argtypes = [_I32P, _I32P, ctypes.c_int64, _I32P, ctypes.c_int64]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class OracleResult:
    colors: np.ndarray          # int32[n], 1-based
    rounds: int
    commit_round: np.ndarray    # int32[n], round in which each node kept its color
    wl_sizes: np.ndarray        # int64[rounds], |WL_r|
    wl_degree_sums: np.ndarray  # int64[rounds], sum of degrees over WL_r
    topology: np.ndarray        # int32[rounds], 1 if round r is topology-driven under H

    @property
    def num_colors(self) -> int:
        return int(self.colors.max()) if self.colors.size else 0


def color_graph(rowptr, colidx, threshold: int = -1, trace_cap: int | None = None,
                max_rounds: int = 0) -> OracleResult:
    """Synchronous IPGC on the host.  ``threshold`` is H (negative: floor(6n/10)); it only labels
    rounds as topology- or data-driven and never changes the colors.  ``max_rounds`` > 0 stops
    early (an incomplete coloring, for timing a bounded sample only)."""
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    n = rowptr.shape[0] - 1
    col = np.zeros(max(n, 0), dtype=np.int32)
    cr = np.zeros(max(n, 0), dtype=np.int32)
    cap = int(trace_cap) if trace_cap is not None else max(n, 1)
    twl = np.zeros(cap, dtype=np.int64)
    tdeg = np.zeros(cap, dtype=np.int64)
    ttopo = np.zeros(cap, dtype=np.int32)
    rounds = ctypes.c_int32(0)
    rc = lib.ipgc_oracle_color(_ptr(rowptr), _ptr(colidx), n, int(threshold), _ptr(col),
                               ctypes.byref(rounds), _ptr(cr), cap, _ptr(twl), _ptr(tdeg), _ptr(ttopo),
                               int(max_rounds))
    if rc != 0:
        raise ValueError("oracle rejected the input (code %d)" % rc)
    r = rounds.value
    k = min(r, cap)
    return OracleResult(col, r, cr, twl[:k].copy(), tdeg[:k].copy(), ttopo[:k].copy())


def first_free_color(rowptr, colidx, col, v: int) -> int:
    """The oracle's assignment rule alone: the color v takes given committed colors ``col``."""
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    return int(lib.ipgc_oracle_first_free_color(rowptr, colidx, rowptr.shape[0] - 1, col, int(v)))


def algorithmic_bytes(res: OracleResult) -> int:
    """Bytes the method must move, summed over rounds: per round 36*|WL_r| + 16*D_r.

    Per active node: worklist entry 4 + row bounds 8 + tentative write 4 (assign) and
    worklist entry 4 + row bounds 8 + own tentative 4 + commit-or-push 4 (conflict) = 36.
    Per neighbour visit: column index 4 + neighbour color 4, once in each step = 16."""
    return int(36 * res.wl_sizes.sum() + 16 * res.wl_degree_sums.sum())


@dataclass
class BfsResult:
    dist: np.ndarray      # int32[n]: hops from the source, -1 if unreachable
    levels: int           # non-empty frontiers (largest finite distance + 1)
    frontier_sizes: np.ndarray  # int64[levels]: nodes at each distance


def bfs(rowptr, colidx, source: int) -> BfsResult:
    """Breadth-first search by its definition (FIFO queue): hop distances from `source`."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    n = rowptr.size - 1
    dist = np.empty(max(n, 0), dtype=np.int32)
    sizes = np.zeros(max(n, 1), dtype=np.int64)
    levels = ctypes.c_int32(0)
    rc = _load().ipgc_oracle_bfs(rowptr.ctypes.data, colidx.ctypes.data, n, int(source), dist.ctypes.data,
                                 sizes.ctypes.data, sizes.size, ctypes.byref(levels))
    if rc != 0:
        raise ValueError("oracle bfs failed (%d)" % rc)
    return BfsResult(dist, levels.value, sizes[:levels.value].copy())
