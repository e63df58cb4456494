"""Plain CPU oracle for epsilon-cost sharded VFunc / VFilter (arXiv 2503.18397).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product path
(the HIP library in ``paper_2503_18397_amd``) never imports this package and
shares no code with it.

This module only marshals numpy arrays into the plain C oracle in
``vf_oracle.c``; every step of the method (signatures, geometry, fuse edges,
round-synchronous peeling, the lexicographically smallest GF(2) solution of
the 2-core, reverse-order assignment, queries) is computed there.  The
readings of the paper that the oracle implements are listed in its header.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")


def build_lib(force: bool = False) -> str:
    """Compile the oracle with the host C compiler (plain C99, -O2)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Geom(C.Structure):
    _fields_ = [
        ("M", C.c_uint32),
        ("h", C.c_int32),
        ("c_num", C.c_uint32),
        ("c_den", C.c_uint32),
        ("sigma", C.c_int32),
        ("l", C.c_uint32),
        ("V", C.c_uint64),
        ("mwhc", C.c_uint32),
        ("part", C.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Fail(C.Structure):
    _fields_ = [
        ("shard", C.c_uint32),
        ("attempt", C.c_uint32),
        ("kind", C.c_uint32),
        ("core_edges", C.c_uint32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build_lib())
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C")
        L.orc_mix64.restype = C.c_uint64
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_seed_words.argtypes = [C.c_uint64, u64p]
        L.orc_fingerprint.restype = C.c_uint64
        L.orc_fingerprint.argtypes = [C.c_uint64, C.c_uint64, u64p, C.c_int32]
        L.orc_shard_ids.argtypes = [u64p, C.c_uint64, C.c_int32, C.c_uint64, u32p]
        L.orc_pack.argtypes = [u64p, C.c_uint64, C.c_int32, u64p]
        L.orc_unpack.restype = C.c_uint64
        L.orc_unpack.argtypes = [u64p, C.c_uint64, C.c_int32]
        L.orc_shard_of.restype = C.c_uint32
        L.orc_shard_of.argtypes = [C.c_uint64, C.c_int32]
        L.orc_edge.argtypes = [C.c_uint64, C.c_uint64, C.c_int32, C.c_uint32,
                               C.c_int32, C.c_uint32, u32p]
        L.orc_edge_mwhc.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, u32p]
        L.orc_geometry_mwhc.argtypes = [C.c_uint32, C.c_int32, C.c_uint32, C.c_uint32,
                                        C.c_void_p]
        L.orc_lambert_w0.restype = C.c_double
        L.orc_lambert_w0.argtypes = [C.c_double]
        L.orc_shard_bits_eps.restype = C.c_int32
        L.orc_shard_bits_eps.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_shard_bits_exact.restype = C.c_double
        L.orc_shard_bits_exact.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_dupmwhc_bits.restype = C.c_int32
        L.orc_dupmwhc_bits.argtypes = [C.c_double, C.c_double, C.c_double]
        for fn in (L.orc_logdupfuse, L.orc_dupfuse):
            fn.restype = C.c_double
            fn.argtypes = [C.c_double] * 5
        L.orc_geometry.argtypes = [C.c_uint32, C.c_int32, C.c_uint32, C.c_uint32,
                                   C.c_int32, C.POINTER(Geom)]
        L.orc_peel.restype = C.c_int32
        L.orc_peel.argtypes = [C.c_uint64, C.c_uint32, u32p, i32p, i8p]
        L.orc_core_lexmin.restype = C.c_int32
        L.orc_core_lexmin.argtypes = [C.c_uint64, C.c_uint32, u32p, u64p, u64p]
        L.orc_solve.restype = C.c_int32
        L.orc_solve.argtypes = [C.c_uint64, C.c_uint32, u32p, u64p, u64p,
                                C.POINTER(C.c_uint32)]
        L.orc_plan.restype = C.c_int32
        L.orc_plan.argtypes = [u64p, C.c_uint64, C.c_int32, C.c_uint64, C.c_uint32,
                               C.c_uint32, C.c_int32, C.POINTER(Geom), u32p]
        L.orc_build.restype = C.c_int32
        L.orc_build.argtypes = [u64p, C.c_void_p, C.c_uint64, C.c_int32, C.c_int32,
                                C.c_uint64, C.c_uint32, C.POINTER(Geom), C.c_void_p,
                                C.c_uint32, u32p, u64p, C.c_void_p, C.c_uint32,
                                C.POINTER(C.c_uint32)]
        L.orc_query.argtypes = [u64p, C.c_uint64, C.c_uint64, C.c_int32, C.c_int32,
                                C.POINTER(Geom), u32p, C.c_void_p, u64p, u64p]
        _lib = L
    return _lib


def _u64(a) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype == np.int64:
        a = a.view(np.uint64)
    return np.ascontiguousarray(a, dtype=np.uint64)


# ------------------------------------------------------------------ hashing

def mix64(x: int) -> int:
    return int(lib().orc_mix64(x))


def seed_words(seed: int) -> np.ndarray:
    out = np.zeros(3, np.uint64)
    lib().orc_seed_words(seed, out)
    return out


def shard_of(hi: int, h: int) -> int:
    """Shard of a signature whose first word is hi (R2)."""
    return int(lib().orc_shard_of(hi, h))


def edge(hi: int, lo: int, h: int, l: int, sigma: int, t: int) -> tuple:
    v = np.zeros(3, np.uint32)
    lib().orc_edge(hi, lo, h, l, sigma, t, v)
    return tuple(int(x) for x in v)


def edge_mwhc(lo: int, part: int, t: int) -> tuple:
    v = np.zeros(3, np.uint32)
    lib().orc_edge_mwhc(lo, part, t, v)
    return tuple(int(x) for x in v)


def fingerprint(hi: int, lo: int, seed: int, b: int) -> int:
    return int(lib().orc_fingerprint(hi, lo, seed_words(seed), b))


# ----------------------------------------------------------- parameter math

def lambert_w0(x: float) -> float:
    return lib().orc_lambert_w0(x)


def shard_bits_eps(n: float, eps: float, alpha: float = 1.0) -> int:
    return lib().orc_shard_bits_eps(n, eps, alpha)


def shard_bits_exact(n: float, eps: float, alpha: float = 1.0) -> float:
    return lib().orc_shard_bits_exact(n, eps, alpha)


def dupmwhc_bits(n: float, c: float, eta: float) -> int:
    return lib().orc_dupmwhc_bits(n, c, eta)


def logdupfuse(n, c, eta, alpha=0.41, beta=-3.0) -> float:
    return lib().orc_logdupfuse(n, c, eta, alpha, beta)


def dupfuse(n, c, eta, alpha=0.41, beta=-3.0) -> float:
    return lib().orc_dupfuse(n, c, eta, alpha, beta)


def geometry(M: int, h: int, c: tuple | None = None, sigma: int = -1,
             mwhc: bool = False) -> dict:
    g = Geom()
    cn, cd = c if c else (0, 0)
    if mwhc:
        lib().orc_geometry_mwhc(M, h, cn, cd, C.byref(g))
    else:
        lib().orc_geometry(M, h, cn, cd, sigma, C.byref(g))
    return g.as_dict()


# ------------------------------------------------------------------ solvers

def peel(nv: int, edges) -> tuple[np.ndarray, np.ndarray, int]:
    e = np.ascontiguousarray(np.asarray(edges, np.uint32).reshape(-1))
    m = e.size // 3
    rnd = np.zeros(max(m, 1), np.int32)
    side = np.zeros(max(m, 1), np.int8)
    nr = lib().orc_peel(nv, m, e if m else np.zeros(3, np.uint32), rnd, side)
    return rnd[:m], side[:m], nr


def core_lexmin(nv: int, rows3, rhs) -> tuple[int, np.ndarray]:
    r = np.ascontiguousarray(np.asarray(rows3, np.uint32).reshape(-1))
    k = r.size // 3
    x = np.zeros(max(nv, 1), np.uint64)
    bad = lib().orc_core_lexmin(nv, k, r if k else np.zeros(3, np.uint32),
                                _u64(rhs) if k else np.zeros(1, np.uint64), x)
    return bad, x[:nv]


def solve(nv: int, edges, rhs) -> tuple[int, np.ndarray, int]:
    e = np.ascontiguousarray(np.asarray(edges, np.uint32).reshape(-1))
    m = e.size // 3
    w = np.zeros(max(nv, 1), np.uint64)
    core = C.c_uint32(0)
    bad = lib().orc_solve(nv, m, e if m else np.zeros(3, np.uint32),
                          _u64(rhs) if m else np.zeros(1, np.uint64), w, C.byref(core))
    return bad, w[:nv], core.value


# ----------------------------------------------------- construction, query

@dataclass
class Built:
    geom: dict
    geom_c: Geom
    seed: int
    b: int
    is_filter: bool
    counts: np.ndarray        # keys per shard
    shards: np.ndarray        # shards that were built
    t: np.ndarray             # local seed per built shard (tmax = failed)
    w: np.ndarray             # (len(shards), V) uint64 cells
    failures: list            # (shard, attempt, kind, core_edges), sorted
    status: int               # 0 ok, 1 some built shard failed


def plan(keys, h: int, seed: int, c: tuple | None = None, sigma: int = -1,
         mwhc: bool = False):
    keys = _u64(keys)
    g = Geom()
    counts = np.zeros(1 << h, np.uint32)
    cn, cd = c if c else (0, 0)
    rc = lib().orc_plan(keys, keys.size, h, seed, cn, cd, sigma, C.byref(g), counts)
    if rc != 0:
        raise ValueError("bad shard bits")
    if mwhc:  # same largest shard, MWHC geometry (R11)
        gm = Geom()
        lib().orc_geometry_mwhc(g.M, h, cn, cd, C.byref(gm))
        g = gm
    return g, counts


def shard_ids(keys, h: int, seed: int) -> np.ndarray:
    """Shard of every key (R2), as uint32."""
    keys = _u64(keys)
    out = np.zeros(max(keys.size, 1), np.uint32)
    lib().orc_shard_ids(keys, keys.size, h, seed, out)
    return out[: keys.size]


def build(keys, values=None, *, b: int, is_filter: bool, h: int, seed: int,
          tmax: int = 255, c: tuple | None = None, sigma: int = -1,
          shards=None, mwhc: bool = False, geom: Geom | None = None) -> Built:
    """Build the listed shards (all if None) of a VFunc / VFilter (fuse
    graphs, or MWHC 3-partite hypergraphs with mwhc=True).  With geom (the
    geometry plan() gives for the whole key set) the keys may be just those
    of the listed shards."""
    keys = _u64(keys)
    if geom is None:
        g, counts = plan(keys, h, seed, c, sigma, mwhc)
    else:
        g, counts = geom, None
    S = 1 << h
    sh = np.arange(S, dtype=np.uint32) if shards is None else \
        np.ascontiguousarray(np.asarray(shards, np.uint32))
    w = np.zeros((max(sh.size, 1), g.V), np.uint64)
    t = np.zeros(max(sh.size, 1), np.uint32)
    cap = 4 * sh.size + 1024
    rec = (Fail * cap)()
    nrec = C.c_uint32(0)
    vals = None
    if not is_filter:
        vals = _u64(values)
    status = lib().orc_build(
        keys, vals.ctypes.data if vals is not None else None, keys.size, b,
        1 if is_filter else 0, seed, tmax, C.byref(g),
        sh.ctypes.data if shards is not None else None, sh.size, t, w,
        C.cast(rec, C.c_void_p), cap, C.byref(nrec))
    fails = sorted((r.shard, r.attempt, r.kind, r.core_edges)
                   for r in rec[: min(nrec.value, cap)])
    return Built(g.as_dict(), g, seed, b, is_filter, counts, sh, t[: sh.size],
                 w[: sh.size], fails, status)


def build_threaded(keys, values=None, *, b: int, is_filter: bool, h: int, seed: int,
                   threads: int, tmax: int = 255, c: tuple | None = None, sigma: int = -1,
                   mwhc: bool = False) -> Built:
    """build() of every shard with the shards split over host threads (the
    C oracle runs with the interpreter lock released): thread k builds the
    shards j with j % threads == k from just their keys.  The result equals
    build() of all shards."""
    import concurrent.futures as cf
    keys = _u64(keys)
    vals = None if is_filter else _u64(values)
    g, counts = plan(keys, h, seed, c, sigma, mwhc)
    sid = shard_ids(keys, h, seed)
    S = 1 << h
    threads = max(1, min(threads, S))

    def one(k):
        sel = (sid % threads) == k
        sh = np.arange(k, S, threads, dtype=np.uint32)
        return build(keys[sel], None if vals is None else vals[sel], b=b, is_filter=is_filter,
                     h=h, seed=seed, tmax=tmax, shards=sh, mwhc=mwhc, geom=g)

    with cf.ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(one, range(threads)))
    w = np.zeros((S, g.V), np.uint64)
    t = np.zeros(S, np.uint32)
    fails = []
    status = 0
    for p in parts:
        w[p.shards] = p.w
        t[p.shards] = p.t
        fails += p.failures
        status |= p.status
    return Built(g.as_dict(), g, seed, b, is_filter, counts, np.arange(S, dtype=np.uint32), t, w,
                 sorted(fails), status)


def pack(w, b: int) -> np.ndarray:
    """Cells w (uint64, b bits used) as a packed bit string of 64-bit words."""
    w = np.ascontiguousarray(np.asarray(w, np.uint64).reshape(-1))
    out = np.zeros(max((w.size * b + 63) // 64, 1), np.uint64)
    lib().orc_pack(w, w.size, b, out)
    return out[: (w.size * b + 63) // 64]


def unpack(words, i: int, b: int) -> int:
    words = np.ascontiguousarray(np.asarray(words, np.uint64))
    return int(lib().orc_unpack(words, i, b))


def query(built: Built, keys) -> np.ndarray:
    """Answers for `keys`; keys of shards that were not built get all ones."""
    keys = _u64(keys)
    S = 1 << built.geom["h"]
    t_full = np.zeros(S, np.uint32)
    slot = np.full(S, -1, np.int32)
    t_full[built.shards] = built.t
    slot[built.shards] = np.arange(built.shards.size, dtype=np.int32)
    out = np.zeros(max(keys.size, 1), np.uint64)
    lib().orc_query(keys, keys.size, built.seed, built.b, 1 if built.is_filter else 0,
                    C.byref(built.geom_c), t_full, slot.ctypes.data,
                    np.ascontiguousarray(built.w.reshape(-1)), out)
    return out[: keys.size]
