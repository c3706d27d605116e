"""Python binding of libmcdose (the C ABI declared in include/mcdose.h).

Argument marshalling only: every step of the transport, tally and
finalisation runs in the HIP library.  PyTorch provides device memory and the
stream the library runs on.  The library must have been built
(`python -m paper_0910_0329_amd.build`); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmcdose.so")

OK, E_INVAL, E_NOMEM, E_NOTFOUND, E_OVERFLOW, E_DEVICE, E_BUSY, E_CANCELED = 0, -1, -2, -3, -4, -5, -6, -7
NCOUNT = 40
COUNT_NAMES = ("histories", "flights", "virtual", "compton", "photo", "pair", "segments",
               "seg_E", "seg_h", "seg_k", "seg_b", "seg_f", "hinges", "moller", "brems",
               "spawns", "philox", "flushes", "escapes", "misses", "local", "void",
               "compton_tries", "moller_tries", "max_stack", "iters", "live", "it_fetch", "it_photon",
               "it_electron", "it_hard", "ln_fetch", "ln_photon", "ln_electron", "ln_hard",
               "rayleigh", "bhabha")


class McdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double)]


class Source(C.Structure):
    _fields_ = [("particle", C.c_int32), ("energy_kind", C.c_int32), ("beam_kind", C.c_int32),
                ("n_bins", C.c_int32), ("e0", C.c_double), ("pos", C.c_double * 3),
                ("field", C.c_double * 4), ("edges", C.c_double * 65),
                ("weights", C.c_double * 64)]


class EnergyBalance(C.Structure):
    _fields_ = [("e_src", C.c_double), ("e_csda", C.c_double), ("e_local", C.c_double),
                ("e_esc", C.c_double), ("e_miss", C.c_double), ("track_e", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("first_history", C.c_uint64), ("block_size", C.c_int32),
                ("grid_blocks", C.c_int32), ("stack_depth", C.c_int32),
                ("tally_slots", C.c_int32), ("diagnostics", C.c_int32),
                ("accumulate", C.c_int32), ("history_records", C.c_void_p),
                ("lockstep", C.c_int32), ("kernel", C.c_int32), ("tally_fp32", C.c_int32),
                ("chunk_per_lane", C.c_int32), ("use_graph", C.c_int32), ("regroup", C.c_int32),
                ("sched_fetch_div", C.c_int32), ("sched_hard_div", C.c_int32),
                ("sched_photon_div", C.c_int32), ("refined_build", C.c_int32),
                ("table_placement", C.c_int32), ("sched_fetch_photon_div", C.c_int32),
                ("sched_segments", C.c_int32)]


KERNEL_REGROUPED, KERNEL_PLAIN = 0, 1
TABLES_AUTO, TABLES_LDS, TABLES_GLOBAL = 0, 1, 2          # mcd_opts.table_placement
# mcd_measure_valu kinds
(VALU_FMA_F32, VALU_ADD_F32, VALU_MUL_F32, VALU_XAD_U32, VALU_MAD_U64, VALU_FMAMK_F32, VALU_RCP_F32,
 VALU_EXP_F32) = range(8)


class Result(C.Structure):
    _fields_ = [("dose", C.c_void_p), ("sigma", C.c_void_p), ("S", C.c_void_p), ("Q", C.c_void_p),
                ("on_device", C.c_int32), ("eb", EnergyBalance),
                ("counters", C.c_uint64 * NCOUNT), ("dmax", C.c_double),
                ("sigma_bar", C.c_double), ("kernel_ms", C.c_double), ("total_ms", C.c_double),
                ("launches", C.c_int32), ("reserved", C.c_int32), ("n_histories", C.c_uint64)]


class BatchItem(C.Structure):
    _fields_ = [("src", Source), ("n_histories", C.c_uint64), ("request_key", C.c_uint32),
                ("reserved", C.c_uint32), ("out", C.POINTER(Result))]


QUEUED, ADMITTED, RUNNING, DONE, FAILED, CANCELED = range(6)
PHANTOMS_SHORTEST, PHANTOMS_IN_TURN = 0, 1               # mcd_serve_config.phantom_order
STATE_NAMES = ("queued", "admitted", "running", "done", "failed", "canceled")


class ServeConfig(C.Structure):
    _fields_ = [("opts", Opts), ("epoch_histories", C.c_uint64), ("max_active", C.c_int32),
                ("phantom_order", C.c_int32), ("memory_limit", C.c_uint64)]


class ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("canceled", C.c_uint64), ("queued", C.c_uint64), ("active", C.c_uint64),
                ("request_bytes", C.c_uint64), ("hbm_used", C.c_uint64), ("hbm_budget", C.c_uint64),
                ("histories", C.c_uint64), ("epochs", C.c_uint64), ("busy_ms", C.c_double),
                ("kernel_ms", C.c_double), ("eb", EnergyBalance), ("counters", C.c_uint64 * NCOUNT)]


HISTORY_DTYPE = np.dtype([("edep", "<f8"), ("track_e", "<f8"), ("hash", "<u8"),
                          ("n_particles", "<u4"), ("escaped", "<u4")])

_lib = None


def lib():
    """Loads libmcdose.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_0910_0329_amd.build`")
        # Load torch's HIP runtime first so that the library binds to the same
        # one (two runtimes in one process do not share devices).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        L.mcd_create.argtypes = [C.c_int, C.c_uint64, C.POINTER(vp)]
        L.mcd_destroy.argtypes = [vp]
        L.mcd_load_materials.argtypes = [vp, vp, C.c_size_t, C.POINTER(i32)]
        L.mcd_unload_materials.argtypes = [vp, i32]
        L.mcd_load_phantom.argtypes = [vp, C.POINTER(Grid), vp, vp, i32, C.POINTER(i32)]
        L.mcd_unload_phantom.argtypes = [vp, i32]
        L.mcd_simulate.argtypes = [vp, i32, C.POINTER(Source), C.c_uint64, C.c_uint64, C.c_uint32,
                                   C.POINTER(Opts), C.POINTER(Result), vp]
        L.mcd_simulate_batch.argtypes = [vp, i32, C.POINTER(BatchItem), i32, C.c_uint64,
                                         C.POINTER(Opts), C.POINTER(Result), vp]
        L.mcd_serve_configure.argtypes = [vp, C.POINTER(ServeConfig)]
        L.mcd_submit.argtypes = [vp, i32, C.POINTER(Source), C.c_uint64, C.c_uint64, C.c_uint32,
                                 C.POINTER(C.c_uint64)]
        L.mcd_submit_adaptive.argtypes = [vp, i32, C.POINTER(Source), C.c_double, C.c_uint64, C.c_uint64,
                                          C.c_uint32, C.POINTER(C.c_uint64)]
        L.mcd_poll.argtypes = [vp, C.c_uint64, C.POINTER(i32), C.POINTER(C.c_uint64)]
        L.mcd_wait.argtypes = [vp, C.c_uint64, C.POINTER(Result), C.c_int64]
        L.mcd_cancel.argtypes = [vp, C.c_uint64]
        L.mcd_serve_stats_get.argtypes = [vp, C.POINTER(ServeStats)]
        L.mcd_simulate_noalloc.argtypes = [vp, i32, C.POINTER(Source), C.c_uint64, C.c_uint64, C.c_uint32,
                                           C.POINTER(Opts), C.POINTER(Result), vp]
        L.mcd_measure_atomics.argtypes = [vp, vp, C.c_uint64, vp, C.c_uint64, i32, C.POINTER(C.c_double), vp]
        L.mcd_check_philox.argtypes = [vp, C.c_uint32, C.c_uint32, vp, C.c_uint64, vp, vp]
        pi32 = C.POINTER(C.c_int32)
        L.mcd_launch_shape.argtypes = [vp, i32, C.POINTER(Opts), pi32, pi32, pi32, pi32, pi32]
        L.mcd_measure_valu.argtypes = [vp, i32, i32, vp, C.POINTER(C.c_double), vp]
        L.mcd_check_tables.argtypes = [vp, i32, i32, i32, vp, C.c_uint64, vp, vp]
        L.mcd_status_string.argtypes = [C.c_int]
        L.mcd_status_string.restype = C.c_char_p
        L.mcd_last_error.argtypes = [vp]
        L.mcd_last_error.restype = C.c_char_p
        _lib = L
    return _lib


EXPORTED = ("mcd_create", "mcd_destroy", "mcd_load_materials", "mcd_unload_materials",
            "mcd_load_phantom", "mcd_unload_phantom", "mcd_simulate", "mcd_simulate_noalloc", "mcd_simulate_batch",
            "mcd_serve_configure", "mcd_submit", "mcd_submit_adaptive", "mcd_poll", "mcd_wait", "mcd_cancel",
            "mcd_serve_stats_get", "mcd_check_philox", "mcd_check_tables", "mcd_measure_atomics", "mcd_measure_valu",
            "mcd_launch_shape", "mcd_status_string", "mcd_last_error")

# Quantities of mcd_check_tables (include/mcdose.h).
Q_MU_C, Q_MU_PE, Q_MU_PP, Q_RANGE, Q_LAMBDA1_INV, Q_SIGMA_M, Q_SIGMA_B = range(7)
Q_MU_R, Q_RANGE_POS, Q_SIGMA_BH = 8, 10, 11
Q_MAJORANT, Q_RANGE_INV, Q_RANGE_POS_INV = 100, 101, 102


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


def make_opts(**kw) -> Opts:
    """mcd_opts from keyword arguments named after its fields; an unknown name
    is an error (a ctypes structure would otherwise take it silently)."""
    o = Opts()
    names = {f[0] for f in Opts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown option {k!r}; mcd_opts has {sorted(names)}")
        setattr(o, k, v)
    return o


def _stream_ptr(stream):
    if stream is None:
        return None
    return getattr(stream, "cuda_stream", stream)


class Engine:
    """One mcdose context on one GPU."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self._h = C.c_void_p()
        self._check(lib().mcd_create(device, hbm_budget, C.byref(self._h)), "mcd_create")
        self.device = device

    def _check(self, rc, what):
        if rc != OK:
            msg = lib().mcd_last_error(self._h).decode() if self._h else lib().mcd_status_string(rc).decode()
            raise McdError(rc, f"{what}: {msg}")

    def close(self):
        if self._h:
            lib().mcd_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def load_materials(self, blob: bytes) -> int:
        out = C.c_int32()
        self._check(lib().mcd_load_materials(self._h, blob, len(blob), C.byref(out)), "mcd_load_materials")
        return out.value

    def unload_materials(self, t: int):
        self._check(lib().mcd_unload_materials(self._h, t), "mcd_unload_materials")

    def load_phantom(self, ph, tables: int) -> int:
        g = Grid(ph.nx, ph.ny, ph.nz, ph.dx, ph.dy, ph.dz, ph.x0, ph.y0, ph.z0)
        mat = np.ascontiguousarray(ph.mat, dtype=np.uint8)
        rho = np.ascontiguousarray(ph.rho, dtype=np.float32)
        out = C.c_int32()
        self._check(lib().mcd_load_phantom(self._h, C.byref(g), mat.ctypes.data, rho.ctypes.data,
                                           tables, C.byref(out)), "mcd_load_phantom")
        return out.value

    def unload_phantom(self, p: int):
        self._check(lib().mcd_unload_phantom(self._h, p), "mcd_unload_phantom")

    def simulate(self, phantom: int, src, n: int, seed: int, key: int = 0, *, n_vox: int = None,
                 device_out: bool = True, want_dose: bool = True, want_tallies: bool = False,
                 stream=None, history_records=None, **opts) -> dict:
        """Runs histories and returns dose, sigma (torch CUDA tensors when
        device_out, numpy otherwise), the raw tallies if asked, the energy
        balance, counters, Dmax, sigma-bar and device timings."""
        s = make_source(src)
        o = make_opts(**opts)
        if history_records is not None:
            o.history_records = history_records.data_ptr()
            o.diagnostics = 1
        if n_vox is None and (want_dose or want_tallies):
            raise ValueError("n_vox is required for dose or tally outputs")
        tallies = ("S", "Q") if o.kernel == KERNEL_PLAIN else ("S",)
        names = (("dose", "sigma") if want_dose else ()) + (tallies if want_tallies else ())
        r, bufs, stream = self._outputs(names, n_vox, device_out, stream)
        rc = lib().mcd_simulate(self._h, phantom, C.byref(s), n, seed, key, C.byref(o), C.byref(r),
                                _stream_ptr(stream))
        self._check(rc, "mcd_simulate")
        out = dict(bufs)
        out.update(_scalars(r))
        out["n"] = n
        return out

    def simulate_noalloc(self, phantom: int, src, n: int, seed: int, key: int = 0, *, dose, sigma, S=None,
                         stream=None, history_records=None, **opts) -> dict:
        """mcd_simulate_noalloc: the regrouped run into caller-owned device
        tensors (float64 dose, sigma and optional S of n_vox each); the library
        allocates nothing.  Returns the scalar results."""
        import torch
        s = make_source(src)
        o = make_opts(**opts)
        if history_records is not None:
            o.history_records = history_records.data_ptr()
            o.diagnostics = 1
        r = Result()
        r.dose = dose.data_ptr()
        r.sigma = sigma.data_ptr()
        if S is not None:
            r.S = S.data_ptr()
        r.on_device = 1
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        rc = lib().mcd_simulate_noalloc(self._h, phantom, C.byref(s), n, seed, key, C.byref(o), C.byref(r),
                                        _stream_ptr(stream))
        self._check(rc, "mcd_simulate_noalloc")
        out = _scalars(r)
        out["n"] = n
        return out

    def _outputs(self, names, n_vox, device_out, stream):
        r = Result()
        bufs = {}
        if device_out:
            import torch
            for nm in names:
                bufs[nm] = torch.empty(n_vox, dtype=torch.float64, device=f"cuda:{self.device}")
                setattr(r, nm, bufs[nm].data_ptr())
            r.on_device = 1
            if stream is None:
                stream = torch.cuda.current_stream(self.device)
        else:
            for nm in names:
                bufs[nm] = np.empty(n_vox, dtype=np.float64)
                setattr(r, nm, bufs[nm].ctypes.data)
            r.on_device = 0
        return r, bufs, stream

    def simulate_batch(self, phantom: int, items, seed: int, *, n_vox: int, device_out: bool = True,
                       want_dose: bool = True, want_tallies: bool = False, stream=None, **opts):
        """items: sequence of (source, n_histories, request_key).  Returns the
        per-item outputs (dose, sigma[, S], dmax, sigma_bar) and the batch totals."""
        o = make_opts(**opts)
        n = len(items)
        arr = (BatchItem * n)()
        results = [None] * n
        per = []
        names = (("dose", "sigma") if want_dose else ()) + (("S",) if want_tallies else ())
        for i, (src, nh, key) in enumerate(items):
            r, bufs, stream = self._outputs(names, n_vox, device_out, stream)
            results[i] = r
            per.append(bufs)
            arr[i].src = make_source(src)
            arr[i].n_histories = nh
            arr[i].request_key = key
            arr[i].out = C.pointer(r)
        tot = Result()
        rc = lib().mcd_simulate_batch(self._h, phantom, arr, n, seed, C.byref(o), C.byref(tot),
                                      _stream_ptr(stream))
        self._check(rc, "mcd_simulate_batch")
        outs = []
        for r, bufs in zip(results, per):
            d = dict(bufs)
            d["dmax"] = r.dmax
            d["sigma_bar"] = r.sigma_bar
            outs.append(d)
        return outs, _scalars(tot)

    # ------------------------------------------------------- verification

    def check_philox(self, seed: int, key: int, counters, stream=None):
        """Philox4x32-10 blocks of the device generator for a (n, 4) uint32
        CUDA tensor of counters; returns a tensor of the same shape."""
        import torch
        ctr = counters.contiguous()
        out = torch.empty_like(ctr)
        self._check(lib().mcd_check_philox(self._h, seed, key, ctr.data_ptr(), ctr.shape[0], out.data_ptr(),
                                           _stream_ptr(stream)), "mcd_check_philox")
        return out

    def check_tables(self, phantom: int, material: int, quantity: int, x, stream=None):
        """A table quantity as the transport kernels evaluate it, at the points
        of a float32 CUDA tensor x; returns a float32 tensor."""
        import torch
        xs = x.contiguous()
        out = torch.empty_like(xs)
        self._check(lib().mcd_check_tables(self._h, phantom, material, quantity, xs.data_ptr(), xs.numel(),
                                           out.data_ptr(), _stream_ptr(stream)), "mcd_check_tables")
        return out

    def launch_shape(self, phantom: int, **opts) -> dict:
        """mcd_launch_shape: the launch a run with these options takes
        (grid_blocks, block_size), the CU count, the workgroups one CU holds
        at once (wave-stack kernel; 0 for the others) and the table placement
        (TABLES_LDS or TABLES_GLOBAL) that TABLES_AUTO resolves to."""
        o = make_opts(**opts)
        v = [C.c_int32() for _ in range(5)]
        self._check(lib().mcd_launch_shape(self._h, phantom, C.byref(o), *(C.byref(x) for x in v)),
                    "mcd_launch_shape")
        return dict(zip(("grid_blocks", "block_size", "cu_count", "resident_per_cu", "table_placement"),
                        (x.value for x in v)))

    def measure_valu(self, kind: int, iters: int = 200, stream=None) -> float:
        """mcd_measure_valu: SIMD cycles per wave-wide operation of one VALU
        instruction kind (VALU_* constants) at the peak engine clock."""
        import torch
        sink = torch.zeros(1, dtype=torch.float32, device=f"cuda:{self.device}")
        cyc = C.c_double()
        self._check(lib().mcd_measure_valu(self._h, kind, iters, sink.data_ptr(), C.byref(cyc),
                                           _stream_ptr(stream)), "mcd_measure_valu")
        return cyc.value

    def measure_atomics(self, target, idx, reps: int = 1, stream=None) -> float:
        """Device milliseconds for reps x idx.numel() FP64 atomic adds at
        target[idx] (float64 and int32/uint32 CUDA tensors)."""
        ms = C.c_double()
        self._check(lib().mcd_measure_atomics(self._h, target.data_ptr(), target.numel(), idx.data_ptr(),
                                              idx.numel(), reps, C.byref(ms), _stream_ptr(stream)),
                    "mcd_measure_atomics")
        return ms.value

    # ------------------------------------------------------------ serving

    def serve_configure(self, epoch_histories: int = 0, max_active: int = 0, memory_limit: int = 0,
                        phantom_order: int = 0, **opts):
        cfg = ServeConfig()
        cfg.opts = make_opts(**opts)
        cfg.epoch_histories = epoch_histories
        cfg.max_active = max_active
        cfg.phantom_order = phantom_order
        cfg.memory_limit = memory_limit
        self._check(lib().mcd_serve_configure(self._h, C.byref(cfg)), "mcd_serve_configure")

    def submit(self, phantom: int, src, n: int, seed: int, key: int = 0, *, sigma_target: float = None) -> int:
        """Queues a request; returns its ticket without waiting for the device.
        With sigma_target the request stops once sigma-bar reaches it (n is
        then the most histories it may run)."""
        s = make_source(src)
        t = C.c_uint64()
        if sigma_target is None:
            self._check(lib().mcd_submit(self._h, phantom, C.byref(s), n, seed, key, C.byref(t)), "mcd_submit")
        else:
            self._check(lib().mcd_submit_adaptive(self._h, phantom, C.byref(s), sigma_target, n, seed, key,
                                                  C.byref(t)), "mcd_submit_adaptive")
        return t.value

    def poll(self, ticket: int):
        """(state, histories done) of a ticket."""
        st, done = C.c_int32(), C.c_uint64()
        self._check(lib().mcd_poll(self._h, ticket, C.byref(st), C.byref(done)), "mcd_poll")
        return st.value, done.value

    def cancel(self, ticket: int):
        self._check(lib().mcd_cancel(self._h, ticket), "mcd_cancel")

    def wait(self, ticket: int, *, n_vox: int = None, device_out: bool = True, want_dose: bool = True,
             timeout_ms: int = -1) -> dict:
        """Waits for a request and collects dose, sigma, Dmax, sigma-bar,
        its device time and its latency (submit to completion, ms)."""
        if want_dose and n_vox is None:
            raise ValueError("n_vox is required for dose outputs")
        names = ("dose", "sigma") if want_dose else ()
        r, bufs, _ = self._outputs(names, n_vox, device_out, None)
        rc = lib().mcd_wait(self._h, ticket, C.byref(r), timeout_ms)
        self._check(rc, "mcd_wait")
        out = dict(bufs)
        out.update({"dmax": r.dmax, "sigma_bar": r.sigma_bar, "kernel_ms": r.kernel_ms,
                    "latency_ms": r.total_ms, "n_histories": r.n_histories})
        return out

    def serve_stats(self) -> dict:
        st = ServeStats()
        self._check(lib().mcd_serve_stats_get(self._h, C.byref(st)), "mcd_serve_stats_get")
        d = {k: getattr(st, k) for k, _ in ServeStats._fields_ if k not in ("eb", "counters")}
        eb = st.eb
        d["bal"] = {"E_src": eb.e_src, "E_csda": eb.e_csda, "E_local": eb.e_local,
                    "E_esc": eb.e_esc, "E_miss": eb.e_miss, "track_e": eb.track_e}
        d["cnt"] = dict(zip(COUNT_NAMES, (int(x) for x in st.counters)))
        return d


def _scalars(r: Result) -> dict:
    eb = r.eb
    return {
        "bal": {"E_src": eb.e_src, "E_csda": eb.e_csda, "E_local": eb.e_local,
                "E_esc": eb.e_esc, "E_miss": eb.e_miss, "track_e": eb.track_e},
        "cnt": dict(zip(COUNT_NAMES, (int(x) for x in r.counters))),
        "dmax": r.dmax, "sigma_bar": r.sigma_bar, "kernel_ms": r.kernel_ms,
        "total_ms": r.total_ms, "launches": r.launches, "n_histories": r.n_histories,
    }
