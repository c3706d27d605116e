"""ctypes front end of the FP64 reference library (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this module.  It loads `liboracle.so` built from `oracle.c` by `make -C oracle`.
"""
from __future__ import annotations

import ctypes as C
import multiprocessing
import os
import subprocess
from concurrent.futures import ProcessPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

NBAL = 6
NCOUNT = 32
BAL_NAMES = ("E_src", "E_csda", "E_local", "E_esc", "E_miss", "track_e")
COUNT_NAMES = ("histories", "flights", "virtual", "compton", "photo", "pair", "segments",
               "seg_E", "seg_h", "seg_k", "seg_b", "seg_f", "hinges", "moller", "brems",
               "spawns", "philox", "flushes", "escapes", "misses", "local", "void",
               "compton_tries", "moller_tries", "max_stack", "rayleigh", "bhabha")


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double)]


class Source(C.Structure):
    _fields_ = [("particle", C.c_int32), ("energy_kind", C.c_int32), ("beam_kind", C.c_int32),
                ("n_bins", C.c_int32), ("e0", C.c_double), ("pos", C.c_double * 3),
                ("field", C.c_double * 4), ("edges", C.c_double * 65),
                ("weights", C.c_double * 64)]


class History(C.Structure):
    _fields_ = [("edep", C.c_double), ("track_e", C.c_double), ("hash", C.c_uint64),
                ("n_particles", C.c_uint32), ("escaped", C.c_uint32)]


HISTORY_DTYPE = np.dtype([("edep", "<f8"), ("track_e", "<f8"), ("hash", "<u8"),
                          ("n_particles", "<u4"), ("escaped", "<u4")])

_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(["make", "-s"] + (["-B"] if force else []) + ["-C", _HERE],
                       check=True, capture_output=True)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB_PATH)
        vp, sz, dp, u8p, f32p = C.c_void_p, C.c_size_t, C.POINTER(C.c_double), C.c_void_p, C.c_void_p
        L.orc_philox.argtypes = [C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_blob_check.argtypes = [vp, sz]
        L.orc_interp.argtypes = [vp, sz, C.c_int, C.c_int, C.c_double, dp]
        L.orc_range_inverse.argtypes = [vp, sz, C.c_int, C.c_double, dp]
        L.orc_majorant.argtypes = [vp, sz, C.POINTER(Grid), u8p, f32p, dp]
        L.orc_philox_n.argtypes = [C.c_uint32, C.c_uint32, vp, sz, vp]
        L.orc_interp_n.argtypes = [vp, sz, C.c_int, C.c_int, dp, sz, dp]
        L.orc_range_inverse_n.argtypes = [vp, sz, C.c_int, C.c_int, dp, sz, dp]
        L.orc_simulate.argtypes = [vp, sz, C.POINTER(Grid), u8p, f32p, C.POINTER(Source),
                                   C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, dp, dp, dp,
                                   C.POINTER(C.c_uint64), vp, vp]
        L.orc_first_interaction.argtypes = [vp, sz, C.POINTER(Grid), u8p, f32p, C.POINTER(Source),
                                            C.c_uint64, C.c_uint32, C.c_uint32, dp, vp]
        L.orc_sample.argtypes = [vp, sz, C.c_int, C.c_double, C.c_uint64, C.c_uint32, dp]
        L.orc_finalize.argtypes = [C.POINTER(Grid), f32p, dp, dp, C.c_uint64, dp, dp, dp, dp]
        L.orc_finalize_groups.argtypes = [C.POINTER(Grid), f32p, dp, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_grid(ph) -> Grid:
    return Grid(ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, ph.x0, ph.y0, ph.z0)


def make_source(src) -> Source:
    s = Source()
    s.particle, s.energy_kind, s.beam_kind = src.particle, src.energy_kind, src.beam_kind
    s.n_bins = src.n_bins if src.energy_kind == 1 else 0
    s.e0 = src.e0
    for i in range(3):
        s.pos[i] = src.pos[i]
    for i in range(4):
        s.field[i] = src.field_rect[i]
    if src.energy_kind == 1:
        for i, v in enumerate(src.edges):
            s.edges[i] = v
        for i, v in enumerate(src.weights):
            s.weights[i] = v
    return s


def philox(k0: int, k1: int, ctr) -> tuple:
    c = (C.c_uint32 * 4)(*ctr)
    o = (C.c_uint32 * 4)()
    lib().orc_philox(k0, k1, c, o)
    return tuple(o)


def uniform(x: int) -> float:
    return lib().orc_uniform(x)


def blob_check(blob: bytes) -> int:
    return lib().orc_blob_check(blob, len(blob))


def interp(blob: bytes, m: int, q: int, e: float) -> float:
    out = C.c_double()
    if lib().orc_interp(blob, len(blob), m, q, e, C.byref(out)):
        raise ValueError("orc_interp rejected its input")
    return out.value


def range_inverse(blob: bytes, m: int, r: float) -> float:
    out = C.c_double()
    if lib().orc_range_inverse(blob, len(blob), m, r, C.byref(out)):
        raise ValueError("orc_range_inverse rejected its input")
    return out.value


def philox_n(k0: int, k1: int, ctr: np.ndarray) -> np.ndarray:
    """Philox4x32-10 of an (n, 4) uint32 array of counters."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.empty_like(c)
    lib().orc_philox_n(k0, k1, c.ctypes.data, c.shape[0], out.ctypes.data)
    return out


def interp_n(blob: bytes, m: int, q: int, e) -> np.ndarray:
    e = np.ascontiguousarray(e, dtype=np.float64)
    out = np.empty_like(e)
    if lib().orc_interp_n(blob, len(blob), m, q, _dp(e), e.size, _dp(out)):
        raise ValueError("orc_interp_n rejected its input")
    return out


def range_inverse_n(blob: bytes, m: int, q: int, r) -> np.ndarray:
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.empty_like(r)
    if lib().orc_range_inverse_n(blob, len(blob), m, q, _dp(r), r.size, _dp(out)):
        raise ValueError("orc_range_inverse_n rejected its input")
    return out


def _phantom_arrays(ph):
    mat = np.ascontiguousarray(ph.mat, dtype=np.uint8)
    rho = np.ascontiguousarray(ph.rho, dtype=np.float32)
    return mat, rho


def majorant(blob: bytes, ph) -> np.ndarray:
    mat, rho = _phantom_arrays(ph)
    out = np.zeros(512)
    g = make_grid(ph)
    if lib().orc_majorant(blob, len(blob), C.byref(g), mat.ctypes.data, rho.ctypes.data, _dp(out)):
        raise ValueError("orc_majorant rejected its input")
    return out


def simulate(blob: bytes, ph, src, n: int, seed: int, key: int = 0, first: int = 0,
             history: bool = False, S=None, Q=None, groups: bool = False) -> dict:
    """Runs histories [first, first + n); returns S, Q, balance, counters (and the
    per-history records if `history`)."""
    mat, rho = _phantom_arrays(ph)
    nv = ph.n_vox
    S = np.zeros(nv) if S is None else S
    Q = np.zeros(nv) if Q is None else Q
    bal = np.zeros(NBAL)
    cnt = np.zeros(NCOUNT, dtype=np.uint64)
    hist = np.zeros(n, dtype=HISTORY_DTYPE) if history else None
    Sb = np.zeros((16, nv)) if groups else None
    g = make_grid(ph)
    s = make_source(src)
    rc = lib().orc_simulate(blob, len(blob), C.byref(g), mat.ctypes.data, rho.ctypes.data,
                            C.byref(s), first, n, seed, key, _dp(S), _dp(Q), _dp(bal),
                            cnt.ctypes.data_as(C.POINTER(C.c_uint64)),
                            hist.ctypes.data if hist is not None else None,
                            Sb.ctypes.data if Sb is not None else None)
    if rc:
        raise ValueError(f"orc_simulate failed ({rc})")
    out = {"S": S, "Q": Q, "bal": dict(zip(BAL_NAMES, bal)), "bal_raw": bal,
           "cnt": dict(zip(COUNT_NAMES, (int(x) for x in cnt))), "cnt_raw": cnt, "n": n}
    if history:
        out["hist"] = hist
    if groups:
        out["Sb"] = Sb
        out["nb"] = np.array([len(range(first + ((b - first) % 16), first + n, 16)) for b in range(16)],
                             dtype=np.float64)
    return out


def _sim_chunk(args):
    import time
    blob, ph, src, first, n, seed, key = args
    t0 = time.perf_counter()
    r = simulate(blob, ph, src, n, seed, key, first=first)
    return r["S"], r["Q"], r["bal_raw"], r["cnt_raw"], time.perf_counter() - t0


def simulate_parallel(blob, ph, src, n, seed, key=0, first=0, procs=None) -> dict:
    """Disjoint history ranges in independent single-threaded processes, merged
    in FP64 (identical to one sequential run up to summation order)."""
    procs = procs or min(8, os.cpu_count() or 1)
    bounds = np.linspace(first, first + n, procs + 1).astype(np.int64)
    jobs = [(blob, ph, src, int(a), int(b - a), seed, key) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    S = np.zeros(ph.n_vox)
    Q = np.zeros(ph.n_vox)
    bal = np.zeros(NBAL)
    cnt = np.zeros(NCOUNT, dtype=np.uint64)
    busy = 0.0
    # fresh interpreters, not forks: a caller that has opened a GPU keeps its
    # device handles to itself
    with ProcessPoolExecutor(len(jobs), mp_context=multiprocessing.get_context("spawn")) as ex:
        for s_, q_, b_, c_, t_ in ex.map(_sim_chunk, jobs):
            busy += t_
            S += s_
            Q += q_
            bal += b_
            cnt[:24] += c_[:24]
            cnt[24] = max(cnt[24], c_[24])
            cnt[25:] += c_[25:]
    return {"S": S, "Q": Q, "bal": dict(zip(BAL_NAMES, bal)), "bal_raw": bal,
            "cnt": dict(zip(COUNT_NAMES, (int(x) for x in cnt))), "cnt_raw": cnt, "n": n,
            "procs": len(jobs), "busy_s": busy}


def first_interaction(blob, ph, src, n, seed, key=0, kinds=False):
    mat, rho = _phantom_arrays(ph)
    z = np.zeros(n)
    kind = np.zeros(n, dtype=np.int32)
    g = make_grid(ph)
    s = make_source(src)
    if lib().orc_first_interaction(blob, len(blob), C.byref(g), mat.ctypes.data, rho.ctypes.data,
                                   C.byref(s), n, seed, key, _dp(z), kind.ctypes.data):
        raise ValueError("orc_first_interaction rejected its input")
    return (z, kind) if kinds else z


def sample(blob, which: int, e: float, n: int, seed: int = 1) -> np.ndarray:
    """n x 8 sampler outputs (see orc_sample)."""
    out = np.zeros((n, 8))
    if lib().orc_sample(blob, len(blob), which, e, n, seed, _dp(out)):
        raise ValueError("orc_sample rejected its input")
    return out


def finalize(ph, S, Q, n):
    rho = np.ascontiguousarray(ph.rho, dtype=np.float32)
    dose = np.zeros(ph.n_vox)
    sigma = np.zeros(ph.n_vox)
    dmax = C.c_double()
    sbar = C.c_double()
    g = make_grid(ph)
    if lib().orc_finalize(C.byref(g), rho.ctypes.data, _dp(np.ascontiguousarray(S)),
                          _dp(np.ascontiguousarray(Q)), n, _dp(dose), _dp(sigma),
                          C.byref(dmax), C.byref(sbar)):
        raise ValueError("orc_finalize rejected its input")
    return dose, sigma, dmax.value, sbar.value


def finalize_groups(ph, Sb, nb):
    rho = np.ascontiguousarray(ph.rho, dtype=np.float32)
    dose = np.zeros(ph.n_vox)
    sigma = np.zeros(ph.n_vox)
    dmax = C.c_double()
    sbar = C.c_double()
    g = make_grid(ph)
    if lib().orc_finalize_groups(C.byref(g), rho.ctypes.data, _dp(np.ascontiguousarray(Sb)),
                                 _dp(np.ascontiguousarray(nb, dtype=np.float64)), _dp(dose),
                                 _dp(sigma), C.byref(dmax), C.byref(sbar)):
        raise ValueError("orc_finalize_groups rejected its input")
    return dose, sigma, dmax.value, sbar.value
