"""Seeded synthetic inputs shared by the device path and the CPU oracle.

Everything here draws numbers; nothing here computes connectivity.  The heavy
generators live in ``gen.c`` (OpenMP), compiled to ``libccinputs.so`` next to
this file by ``build()``.  All draws are splitmix64 outputs in counter mode,
so a workload is fully named by (family, sizes, seed).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libccinputs.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)


def build(verbose: bool = False) -> str:
    """Compile gen.c into libccinputs.so (gcc -O3 -fopenmp)."""
    src = os.path.join(_HERE, "gen.c")
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(_SO)
        lib.gen_er.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, _i32p, _i32p]
        lib.gen_pairs.argtypes = lib.gen_er.argtypes
        lib.gen_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint64, _i32p, _i32p]
        lib.gen_grid.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                 _i32p, _i32p]
        lib.gen_grid.restype = ctypes.c_int64
        lib.gen_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, _i32p]
        lib.gen_shuffle_pairs.argtypes = [ctypes.c_int64, ctypes.c_uint64, _i32p, _i32p]
        lib.gen_orient_drop_loops.argtypes = [ctypes.c_int64, _i32p, _i32p]
        lib.gen_orient_drop_loops.restype = ctypes.c_int64
        lib.gen_splitmix_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.gen_splitmix_draw.restype = ctypes.c_uint64
        lib.gen_pair_weights.argtypes = [ctypes.c_int64, ctypes.c_int64, _i32p, _i32p, ctypes.c_double,
                                         ctypes.c_uint64, ctypes.POINTER(ctypes.c_float)]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_i32p)


class Graph:
    """An undirected multigraph given as a pair list on vertices [0, n)."""

    __slots__ = ("n", "u", "v", "name")

    def __init__(self, n: int, u: np.ndarray, v: np.ndarray, name: str = ""):
        self.n = int(n)
        self.u = np.ascontiguousarray(u, dtype=np.int32)
        self.v = np.ascontiguousarray(v, dtype=np.int32)
        self.name = name

    @property
    def num_pairs(self) -> int:
        return int(self.u.shape[0])

    def __repr__(self):
        return f"Graph({self.name or '?'}, n={self.n}, pairs={self.num_pairs})"


def splitmix_draw(seed: int, stream: int, i: int) -> int:
    return int(_load().gen_splitmix_draw(seed, stream, i))


def er(n: int, num_pairs: int, seed: int) -> Graph:
    lib = _load()
    u = np.empty(num_pairs, np.int32)
    v = np.empty(num_pairs, np.int32)
    if num_pairs:
        lib.gen_er(n, num_pairs, seed, _p(u), _p(v))
    return Graph(n, u, v, f"er(n={n},pairs={num_pairs},seed={seed})")


def query_pairs(n: int, count: int, seed: int):
    lib = _load()
    a = np.empty(count, np.int32)
    b = np.empty(count, np.int32)
    if count:
        lib.gen_pairs(n, count, seed, _p(a), _p(b))
    return a, b


def rmat(scale: int, num_tuples: int, a: float, b: float, c: float, seed: int) -> Graph:
    lib = _load()
    u = np.empty(num_tuples, np.int32)
    v = np.empty(num_tuples, np.int32)
    if num_tuples:
        lib.gen_rmat(scale, num_tuples, a, b, c, seed, _p(u), _p(v))
    return Graph(1 << scale, u, v, f"rmat(scale={scale},tuples={num_tuples},a={a},b={b},c={c},seed={seed})")


def grid(dims: int, side: int, p: float, seed: int) -> Graph:
    lib = _load()
    cnt = lib.gen_grid(dims, side, p, seed, None, None)
    u = np.empty(cnt, np.int32)
    v = np.empty(cnt, np.int32)
    if cnt:
        lib.gen_grid(dims, side, p, seed, _p(u), _p(v))
    return Graph(side ** dims, u, v, f"grid{dims}d(side={side},p={p},seed={seed})")


def permutation(n: int, seed: int) -> np.ndarray:
    perm = np.empty(n, np.int32)
    if n:
        _load().gen_permutation(n, seed, _p(perm))
    return perm


def shuffle_pairs(u: np.ndarray, v: np.ndarray, seed: int):
    u = np.array(u, dtype=np.int32, copy=True)
    v = np.array(v, dtype=np.int32, copy=True)
    if u.shape[0]:
        _load().gen_shuffle_pairs(u.shape[0], seed, _p(u), _p(v))
    return u, v


def orient_drop_loops(u: np.ndarray, v: np.ndarray):
    u = np.array(u, dtype=np.int32, copy=True)
    v = np.array(v, dtype=np.int32, copy=True)
    k = int(_load().gen_orient_drop_loops(u.shape[0], _p(u), _p(v))) if u.shape[0] else 0
    return u[:k].copy(), v[:k].copy()


# ---- small structured families (numpy; sizes are modest) --------------------

def empty(n: int) -> Graph:
    z = np.zeros(0, np.int32)
    return Graph(n, z, z, f"empty(n={n})")


def path(n: int, perm: np.ndarray | None = None) -> Graph:
    ids = np.arange(n, dtype=np.int32) if perm is None else np.asarray(perm, np.int32)
    return Graph(n, ids[:-1], ids[1:], f"path(n={n})")


def chain(n: int, seed: int) -> Graph:
    """A path visiting the vertices in a seeded random order."""
    g = path(n, permutation(n, seed))
    g.name = f"chain(n={n},seed={seed})"
    return g


def star(n: int, center: int = 0) -> Graph:
    leaves = np.array([i for i in range(n) if i != center], dtype=np.int32)
    return Graph(n, np.full(leaves.shape, center, np.int32), leaves, f"star(n={n},c={center})")


def clique(n: int) -> Graph:
    iu, iv = np.triu_indices(n, k=1)
    return Graph(n, iu.astype(np.int32), iv.astype(np.int32), f"clique(n={n})")


def disjoint_union(parts) -> Graph:
    us, vs, off = [], [], 0
    for g in parts:
        us.append(g.u.astype(np.int64) + off)
        vs.append(g.v.astype(np.int64) + off)
        off += g.n
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    return Graph(off, u.astype(np.int32), v.astype(np.int32), "union(" + ",".join(g.name for g in parts) + ")")


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    perm = np.asarray(perm, np.int32)
    return Graph(g.n, perm[g.u], perm[g.v], g.name + "+perm")


def all_graphs_on(k: int) -> Graph:
    """Disjoint union of every labelled simple graph on k vertices.

    Graph number g (0 <= g < 2^(k(k-1)/2)) occupies vertices [g*k, (g+1)*k) and
    contains vertex-pair number b (in row-major upper-triangle order) iff bit b
    of g is set."""
    iu, iv = np.triu_indices(k, k=1)
    nb = iu.shape[0]
    ng = 1 << nb
    gs = np.arange(ng, dtype=np.int64)
    bits = ((gs[:, None] >> np.arange(nb)[None, :]) & 1).astype(bool)
    gi, bi = np.nonzero(bits)
    u = gi * k + iu[bi]
    v = gi * k + iv[bi]
    return Graph(ng * k, u.astype(np.int32), v.astype(np.int32), f"all_graphs_on({k})")


# ---- the benchmark workloads --------------------------------------------------

def workload_er_2_16() -> Graph:
    """Erdos-Renyi: n = 2^16, 2^19 uniform pairs, seed 1."""
    return er(1 << 16, 1 << 19, seed=1)


def workload_rmat(scale: int = 24, edge_factor: int = 8, seed: int = 2,
                  abc=(0.57, 0.19, 0.19)) -> Graph:
    """R-MAT with edge_factor * n tuples (16n directed edges nominal)."""
    a, b, c = abc
    return rmat(scale, edge_factor << scale, a, b, c, seed)


def workload_grid3d(side: int = 256, p: float = 0.35, seed: int = 3) -> Graph:
    return grid(3, side, p, seed)


def log_uniform_int(lo: float, hi: float, u: float) -> int:
    return int(math.floor(10 ** (math.log10(lo) + u * (math.log10(hi) - math.log10(lo)))))


def pair_weights(n: int, a, b, seed: int, mean: float = 1.0) -> np.ndarray:
    """Float32 weight of each undirected pair (a[i], b[i]): exponential with
    the given mean, a function of the unordered pair (so both orientations
    and repeated copies agree).  Also gives the weight of every adjacency
    entry of a CSR: pass the row ids and the adjacency."""
    a = np.ascontiguousarray(a, np.int32)
    b = np.ascontiguousarray(b, np.int32)
    w = np.empty(a.shape[0], np.float32)
    if a.size:
        _load().gen_pair_weights(n, a.shape[0], _p(a), _p(b), float(mean), seed,
                                 w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return w
