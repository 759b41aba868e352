"""Replica-exchange Wang-Landau (arXiv:1407.5140) on MI355X: Python binding.

This module only marshals arguments to librewl.so (include/rewl.h); every step
of the method runs in the library's HIP kernels.  The library must have been
built in-tree (``python -m paper_1407_5140_amd.build``); importing without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librewl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1407_5140_amd.build` "
                      "(hipcc, gfx950); the REWL path has no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

REWL_OK = 0
REWL_E_INVALID = -1
_STATUS = {0: "OK", -1: "INVALID", -2: "EMPTY_WINDOW", -3: "NOMEM", -4: "DEVICE", -5: "OVERFLOW",
           -6: "INIT_STUCK", -7: "STATE"}


class RewlError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.rewl_last_error().decode(errors="replace")
        super().__init__(f"{where}: REWL_E_{_STATUS.get(status, status)} ({status}): {msg}")
        self.status = status


class rewl_config(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("q", ctypes.c_int32), ("L", ctypes.c_int32),
                ("n_windows", ctypes.c_int32), ("overlap_num", ctypes.c_int32),
                ("overlap_den", ctypes.c_int32), ("walkers_per_window", ctypes.c_int32),
                ("flat_num", ctypes.c_int32), ("flat_den", ctypes.c_int32),
                ("lnf_k0", ctypes.c_int32), ("lnf_kfinal", ctypes.c_int32),
                ("exchange_enabled", ctypes.c_int32), ("exchange_interval", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("flat_rule", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("window_lo", ctypes.c_void_p), ("window_hi", ctypes.c_void_p)]


REWL_SWEEP_AUTO, REWL_SWEEP_LANE, REWL_SWEEP_WAVE = 0, 1, 2


class rewl_tune(ctypes.Structure):
    _fields_ = [("walkers_per_block", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("poll_every", ctypes.c_int32), ("sweep_kind", ctypes.c_int32),
                ("lds_target_kb", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("guard_band_log2", ctypes.c_int32), ("table_placement", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("map_log2", ctypes.c_int32)]


PLACEMENTS = {"auto": 0, "lds": 1, "device": 2}


def make_tune(kind="auto", walkers_per_block=0, use_graph=0, poll_every=8, lds_target_kb=0,
              autotune=0, guard_band_log2=0, table_placement="auto", persistent=0,
              map_log2=0) -> rewl_tune:
    """guard_band_log2: 0 keeps the library's 2^-40 guard band of the fast acceptance
    test; -40..-2 widen it (identical results, more exact slow-path decisions).
    table_placement: where the wave sweep keeps the counts ("lds", "device", "auto");
    persistent: 1 runs the lane sweep as a persistent grid over a tile queue;
    map_log2: the wave sweep's site map holds at most 2^map_log2 entries per walker
    (6..12; 0 = the library's choice)."""
    return rewl_tune(walkers_per_block, use_graph, poll_every,
                     {"auto": 0, "lane": 1, "wave": 2}[kind], lds_target_kb, autotune, guard_band_log2,
                     PLACEMENTS[table_placement], persistent, map_log2)


class rewl_stats(ctypes.Structure):
    _fields_ = [("intervals", ctypes.c_int64), ("attempts", ctypes.c_int64),
                ("windows_done", ctypes.c_int32), ("min_k", ctypes.c_int32),
                ("sweep_ms", ctypes.c_double), ("interval_ms", ctypes.c_double),
                ("round_trips", ctypes.c_int64), ("slow_decisions", ctypes.c_int64)]


_vp = ctypes.c_void_p
_P = ctypes.POINTER
_sigs = {
    "rewl_last_error": ([], ctypes.c_char_p),
    "rewl_layout": ([_P(rewl_config), _vp, _vp, _vp, _vp], ctypes.c_int),
    "rewl_mask": ([_P(rewl_config), _vp], ctypes.c_int),
    "rewl_balanced_layout": ([_P(rewl_config), _vp, _vp, _vp], ctypes.c_int),
    "rewl_tilt_density": ([_P(rewl_config), _vp], ctypes.c_int),
    "rewl_create": ([_P(rewl_config), _vp, _P(_vp)], ctypes.c_int),
    "rewl_batch_create": ([_P(rewl_config), ctypes.c_int32, _vp, _P(rewl_tune), _P(_vp)], ctypes.c_int),
    "rewl_set_initial_lng": ([_vp, ctypes.c_int32, _vp], ctypes.c_int),
    "rewl_run": ([_vp, ctypes.c_int64, _P(ctypes.c_int32)], ctypes.c_int),
    "rewl_run_exact": ([_vp, ctypes.c_int64], ctypes.c_int),
    "rewl_get_window_lng": ([_vp, ctypes.c_int32, ctypes.c_int32, _vp], ctypes.c_int),
    "rewl_concat": ([_vp, ctypes.c_int32, _vp, _vp], ctypes.c_int),
    "rewl_concat_noalloc": ([_vp, ctypes.c_int32, _vp, _vp], ctypes.c_int),
    "rewl_ensemble": ([_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, _vp, _vp], ctypes.c_int),
    "rewl_thermo": ([ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp,
                     _vp], ctypes.c_int),
    "rewl_get_state": ([_vp, ctypes.c_int32] + [_vp] * 9, ctypes.c_int),
    "rewl_get_stats": ([_vp, ctypes.c_int32, _P(rewl_stats), _vp, _vp, _vp, _vp], ctypes.c_int),
    "rewl_set_timing": ([_vp, ctypes.c_int32], ctypes.c_int),
    "rewl_checkpoint": ([_vp, _vp, _P(ctypes.c_size_t)], ctypes.c_int),
    "rewl_restore": ([_vp, _vp, ctypes.c_size_t], ctypes.c_int),
    "rewl_destroy": ([_vp], None),
    "rewl_info": ([_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "rewl_wave_plan": ([_P(rewl_config), _P(rewl_tune), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                        _vp, _vp, _vp, _vp], ctypes.c_int),
    "rewl_get_tune": ([_vp, _P(rewl_tune)], ctypes.c_int),
    "rewl_probe_accept": ([_vp, _vp, ctypes.c_int32, _vp], ctypes.c_int),
    "rewl_probe_philox": ([_vp, ctypes.c_int32, _vp], ctypes.c_int),
    # density-of-states network (include/rewl_mlp.h)
    "mlp_last_error": ([], ctypes.c_char_p),
    "mlp_create": ([_vp, _vp, _P(_vp)], ctypes.c_int),
    "mlp_destroy": ([_vp], None),
    "mlp_n_params": ([_vp, _P(ctypes.c_int64)], ctypes.c_int),
    "mlp_get_params": ([_vp, _vp, ctypes.c_size_t], ctypes.c_int),
    "mlp_set_params": ([_vp, _vp, ctypes.c_size_t], ctypes.c_int),
    "mlp_infer": ([_vp, _vp, _vp, ctypes.c_int32], ctypes.c_int),
    "mlp_grad": ([_vp, _vp, _vp, ctypes.c_int32, _vp, _vp], ctypes.c_int),
    "mlp_fit": ([_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                 ctypes.c_uint32, _vp], ctypes.c_int),
    "mlp_warm_table": ([_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp], ctypes.c_int),
    "mlp_probe_gemm": ([_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp], ctypes.c_int),
}
for _name, (_args, _res) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_sigs)


def _check(status: int, where: str) -> None:
    if status != REWL_OK:
        raise RewlError(status, where)


class MlpError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.mlp_last_error().decode(errors="replace")
        super().__init__(f"{where}: REWL_E_{_STATUS.get(status, status)} ({status}): {msg}")
        self.status = status


def _mcheck(status: int, where: str) -> None:
    if status != REWL_OK:
        raise MlpError(status, where)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_vp)


REWL_FLAT_MEAN, REWL_FLAT_VISITS = 0, 1


def make_config(model="ising", q=2, L=8, n_windows=4, overlap=(3, 4), m=1, flat=(4, 5), k0=0,
                kfinal=20, X=10000, seed=1, exchange=True, flat_rule="mean", windows=None) -> rewl_config:
    """Problem statement of Sec. II.A / IV: model, L, h windows with overlap o,
    m walkers per window, flatness num/den (rule "mean": min H >= num/den of the
    mean; rule "visits": H >= (num/den)/sqrt(ln f), Eq. (8)), ln f = 2^-k0 ..
    2^-kfinal, X attempts per walker between exchanges, Philox seed; windows:
    optional (lo, hi) inclusive global bins of unequal windows (kept alive by
    the returned config)."""
    c = rewl_config(0 if model == "ising" else 1, q, L, n_windows, overlap[0], overlap[1], m,
                    flat[0], flat[1], k0, kfinal, 1 if exchange else 0, X, seed,
                    {"mean": REWL_FLAT_MEAN, "visits": REWL_FLAT_VISITS}[flat_rule], 0, None, None)
    if windows is not None:
        c._wlo = np.ascontiguousarray(windows[0], dtype=np.int32)
        c._whi = np.ascontiguousarray(windows[1], dtype=np.int32)
        c.window_lo = c._wlo.ctypes.data
        c.window_hi = c._whi.ctypes.data
    return c


# ------------------------------------------------------------ C-ABI mirrors
def rewl_layout(cfg: rewl_config):
    nb, wb = ctypes.c_int32(), ctypes.c_int32()
    lo = np.zeros(cfg.n_windows, np.int32)
    hi = np.zeros(cfg.n_windows, np.int32)
    _check(_lib.rewl_layout(ctypes.byref(cfg), ctypes.byref(nb), ctypes.byref(wb), _p(lo), _p(hi)),
           "rewl_layout")
    return nb.value, wb.value, lo, hi


def rewl_balanced_layout(cfg: rewl_config, rho) -> tuple[np.ndarray, np.ndarray]:
    """Unequal windows of equal total difficulty rho[W] (pure host)."""
    r = np.ascontiguousarray(rho, dtype=np.float64)
    lo = np.zeros(cfg.n_windows, np.int32)
    hi = np.zeros(cfg.n_windows, np.int32)
    _check(_lib.rewl_balanced_layout(ctypes.byref(cfg), _p(r), _p(lo), _p(hi)), "rewl_balanced_layout")
    return lo, hi


def rewl_tilt_density(cfg: rewl_config) -> np.ndarray:
    """Difficulty density near the ground levels, for rewl_balanced_layout (pure host)."""
    rho = np.zeros(rewl_layout(cfg)[0], np.float64)
    _check(_lib.rewl_tilt_density(ctypes.byref(cfg), _p(rho)), "rewl_tilt_density")
    return rho


def tilted_layout(cfg: rewl_config) -> tuple[np.ndarray, np.ndarray]:
    """Windows narrowed towards the slow ground levels (pure host)."""
    return rewl_balanced_layout(cfg, rewl_tilt_density(cfg))


def rewl_mask(cfg: rewl_config) -> np.ndarray:
    W = rewl_layout(cfg)[0]
    m = np.zeros(W, np.uint8)
    _check(_lib.rewl_mask(ctypes.byref(cfg), _p(m)), "rewl_mask")
    return m


def rewl_create(cfg: rewl_config, stream=None):
    h = _vp()
    _check(_lib.rewl_create(ctypes.byref(cfg), stream, ctypes.byref(h)), "rewl_create")
    return h


def rewl_batch_create(cfgs, stream=None, tune: rewl_tune | None = None):
    arr = (rewl_config * len(cfgs))(*cfgs)
    h = _vp()
    _check(_lib.rewl_batch_create(arr, len(cfgs), stream, ctypes.byref(tune) if tune else None,
                                  ctypes.byref(h)), "rewl_batch_create")
    return h


def rewl_set_initial_lng(h, instance: int, lng: np.ndarray) -> None:
    a = np.ascontiguousarray(lng, dtype=np.float64)
    _check(_lib.rewl_set_initial_lng(h, instance, _p(a)), "rewl_set_initial_lng")


def rewl_run(h, max_intervals: int) -> bool:
    done = ctypes.c_int32(0)
    _check(_lib.rewl_run(h, int(max_intervals), ctypes.byref(done)), "rewl_run")
    return bool(done.value)


def rewl_run_exact(h, n: int) -> None:
    _check(_lib.rewl_run_exact(h, int(n)), "rewl_run_exact")


def rewl_get_window_lng(h, instance: int, window: int, WB: int) -> np.ndarray:
    out = np.empty(WB, np.float64)
    _check(_lib.rewl_get_window_lng(h, instance, window, _p(out)), "rewl_get_window_lng")
    return out


def rewl_concat(h, instance: int, W: int, n_windows: int):
    out = np.empty(W, np.float64)
    join = np.zeros(max(n_windows - 1, 1), np.int32)
    _check(_lib.rewl_concat(h, instance, _p(out), _p(join)), "rewl_concat")
    return out, join[: max(n_windows - 1, 0)]


def rewl_concat_noalloc(h, instance: int, W: int, n_windows: int):
    """rewl_concat staged in the library's fixed device array (no allocation)."""
    out = np.empty(W, np.float64)
    join = np.zeros(max(n_windows - 1, 1), np.int32)
    _check(_lib.rewl_concat_noalloc(h, instance, _p(out), _p(join)), "rewl_concat_noalloc")
    return out, join[: max(n_windows - 1, 0)]


def rewl_ensemble(h, runs, R: int, seed: int, W: int, n_windows: int):
    r = np.ascontiguousarray(runs, np.int32)
    out = np.empty((R + 1, W), np.float64)
    join = np.zeros((R + 1, max(n_windows - 1, 1)), np.int32)
    _check(_lib.rewl_ensemble(h, _p(r), int(r.size), int(R), int(seed), _p(out), _p(join)), "rewl_ensemble")
    return out, join[:, : max(n_windows - 1, 0)]


def rewl_thermo(model, L: int, lng, T):
    """u, c, f per spin, shape (rows, len(T)), for ln g rows over the model's bins."""
    m = {"ising": 0, "potts": 1}.get(model, model)
    x = np.ascontiguousarray(np.atleast_2d(lng), np.float64)
    t = np.ascontiguousarray(np.atleast_1d(T), np.float64)
    S, nT = x.shape[0], t.size
    W = L * L + 1 if m == 0 else 2 * L * L + 1
    if m in (0, 1) and x.shape[1] != W:
        raise ValueError(f"ln g rows have {x.shape[1]} bins, the model needs {W}")
    u, c, f = (np.empty((S, nT), np.float64) for _ in range(3))
    _check(_lib.rewl_thermo(int(m), int(L), _p(x), int(S), _p(t), int(nT), _p(u), _p(c), _p(f)),
           "rewl_thermo")
    return u, c, f


def rewl_get_state(h, instance: int, cfg: rewl_config) -> dict:
    W, WB, _, _ = rewl_layout(cfg)
    S, N, nw = cfg.n_windows * cfg.walkers_per_window, cfg.L * cfg.L, cfg.n_windows
    st = dict(spins=np.empty((S, N), np.uint8), bins=np.empty(S, np.int32),
              H=np.empty((S, WB), np.int64), lng=np.empty((S, WB), np.float64),
              flat=np.empty(S, np.uint8), k=np.empty(nw, np.int32), done=np.empty(nw, np.uint8),
              swaps=np.empty(S, np.int8))
    t = ctypes.c_int64(0)
    _check(_lib.rewl_get_state(h, instance, *[_p(st[n]) for n in
                                              ("spins", "bins", "H", "lng", "flat", "k", "done",
                                               "swaps")], ctypes.byref(t)), "rewl_get_state")
    st["t"] = t.value
    return st


def rewl_get_stats(h, instance: int, n_windows: int, n_slots: int) -> dict:
    s = rewl_stats()
    p = np.zeros(n_windows, np.int64)
    a = np.zeros(n_windows, np.int64)
    k = np.zeros(n_windows, np.int32)
    rt = np.zeros(n_slots, np.int32)
    _check(_lib.rewl_get_stats(h, instance, ctypes.byref(s), _p(p), _p(a), _p(k), _p(rt)), "rewl_get_stats")
    return dict(intervals=s.intervals, attempts=s.attempts, windows_done=s.windows_done,
                min_k=s.min_k, sweep_ms=s.sweep_ms, interval_ms=s.interval_ms, ex_prop=p, ex_acc=a,
                k=k, round_trips=rt, round_trips_total=s.round_trips, slow_decisions=s.slow_decisions)


def rewl_set_timing(h, on: bool) -> None:
    _check(_lib.rewl_set_timing(h, 1 if on else 0), "rewl_set_timing")


def rewl_checkpoint(h) -> bytes:
    n = ctypes.c_size_t(0)
    _check(_lib.rewl_checkpoint(h, None, ctypes.byref(n)), "rewl_checkpoint")
    buf = ctypes.create_string_buffer(n.value)
    _check(_lib.rewl_checkpoint(h, buf, ctypes.byref(n)), "rewl_checkpoint")
    return buf.raw[: n.value]


def rewl_restore(h, blob: bytes) -> None:
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(_lib.rewl_restore(h, buf, len(blob)), "rewl_restore")


def rewl_destroy(h) -> None:
    _lib.rewl_destroy(h)


def rewl_info(h, instance: int = 0) -> dict:
    n, kind, w, lds = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
    pl, mp = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.rewl_info(h, instance, ctypes.byref(n), ctypes.byref(kind), ctypes.byref(w),
                          ctypes.byref(lds), ctypes.byref(pl), ctypes.byref(mp)), "rewl_info")
    return dict(n_instances=n.value, sweep_kind={1: "lane", 2: "wave"}[kind.value],
                walkers_per_block=w.value, lds_bytes=lds.value,
                table_placement={1: "lds", 2: "device"}[pl.value], map_entries=mp.value)


def rewl_wave_plan(cfg: rewl_config, tune: rewl_tune | None = None, lds_per_block: int = 163840,
                   n_cu: int = 256, waves_per_cu: int = 16) -> dict:
    """Pure host: the wave sweep's plan for one instance (defaults: MI355X's 160 KiB of
    LDS, 256 CUs and 16 waves of the sweep kernel per CU)."""
    g, pl, mp, lds = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
    _check(_lib.rewl_wave_plan(ctypes.byref(cfg), ctypes.byref(tune) if tune is not None else None,
                               lds_per_block, n_cu, waves_per_cu, ctypes.byref(g), ctypes.byref(pl),
                               ctypes.byref(mp), ctypes.byref(lds)), "rewl_wave_plan")
    return dict(walkers_per_block=g.value, table_placement={1: "lds", 2: "device"}[pl.value],
                map_entries=mp.value, lds_bytes=lds.value)


def rewl_get_tune(h) -> dict:
    t = rewl_tune()
    _check(_lib.rewl_get_tune(h, ctypes.byref(t)), "rewl_get_tune")
    return {f: getattr(t, f) for f, _ in rewl_tune._fields_}


def rewl_probe_accept(delta, u53) -> np.ndarray:
    d = np.ascontiguousarray(delta, dtype=np.float64)
    u = np.ascontiguousarray(u53, dtype=np.uint64)
    out = np.empty(len(d), np.int32)
    _check(_lib.rewl_probe_accept(_p(d), _p(u), len(d), _p(out)), "rewl_probe_accept")
    return out


def rewl_probe_philox(ctr_key: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(ctr_key, dtype=np.uint32).reshape(-1, 6)
    out = np.empty((len(a), 4), np.uint32)
    _check(_lib.rewl_probe_philox(_p(a), len(a), _p(out)), "rewl_probe_philox")
    return out


# ------------------------------------------------------------ convenience
class Rewl:
    """One handle (a batch of instances) with the C-ABI calls as methods."""

    def __init__(self, cfgs, stream=None, tune: rewl_tune | None = None):
        self.cfgs = list(cfgs) if isinstance(cfgs, (list, tuple)) else [cfgs]
        self.h = rewl_batch_create(self.cfgs, stream, tune)
        self.layouts = [rewl_layout(c) for c in self.cfgs]

    def close(self):
        if self.h:
            rewl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, max_intervals: int) -> bool:
        return rewl_run(self.h, max_intervals)

    def run_exact(self, n: int) -> None:
        rewl_run_exact(self.h, n)

    def state(self, i: int = 0) -> dict:
        return rewl_get_state(self.h, i, self.cfgs[i])

    def stats(self, i: int = 0) -> dict:
        c = self.cfgs[i]
        return rewl_get_stats(self.h, i, c.n_windows, c.n_windows * c.walkers_per_window)

    def pieces(self, i: int = 0) -> np.ndarray:
        W, WB, lo, hi = self.layouts[i]
        return np.stack([rewl_get_window_lng(self.h, i, a, WB) for a in range(len(lo))])

    def concat(self, i: int = 0):
        W = self.layouts[i][0]
        return rewl_concat(self.h, i, W, self.cfgs[i].n_windows)

    def ensemble(self, runs, R: int = 0, seed: int = 1):
        """Mean global ln g of the listed instances (row 0) and R bootstrap resamples."""
        i = int(runs[0])
        return rewl_ensemble(self.h, runs, R, seed, self.layouts[i][0], self.cfgs[i].n_windows)

    def set_initial_lng(self, lng, i: int = 0) -> None:
        rewl_set_initial_lng(self.h, i, lng)

    def info(self, i: int = 0) -> dict:
        return rewl_info(self.h, i)

    def tune(self) -> dict:
        return rewl_get_tune(self.h)


# ------------------------------------------------------------ DOS network
class mlp_config(ctypes.Structure):
    _fields_ = [("in_dim", ctypes.c_int32), ("hidden", ctypes.c_int32), ("layers", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("seed", ctypes.c_uint64)]


MODELS = {"ising": 0, "potts": 1}


def _rows(a, width: int) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32).reshape(-1, width)


def mlp_probe_gemm(A, B) -> np.ndarray:
    a = np.ascontiguousarray(A, dtype=np.float32)
    b = np.ascontiguousarray(B, dtype=np.float32)
    M_, K = a.shape
    K2, N_ = b.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    c = np.empty((M_, N_), np.float32)
    _mcheck(_lib.mlp_probe_gemm(_p(a), _p(b), M_, N_, K, _p(c)), "mlp_probe_gemm")
    return c


class Mlp:
    """The density-of-states network: parameters, training and inference live on
    the device (include/rewl_mlp.h); rows and results cross as numpy arrays."""

    def __init__(self, in_dim=3, hidden=256, layers=3, max_batch=4096, seed=1, stream=None):
        self.cfg = mlp_config(in_dim, hidden, layers, max_batch, seed)
        h = _vp()
        _mcheck(_lib.mlp_create(ctypes.byref(self.cfg), stream, ctypes.byref(h)), "mlp_create")
        self.h = h
        n = ctypes.c_int64()
        _mcheck(_lib.mlp_n_params(self.h, ctypes.byref(n)), "mlp_n_params")
        self.n_params = n.value

    def close(self):
        if getattr(self, "h", None):
            _lib.mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _mcheck(_lib.mlp_get_params(self.h, _p(out), out.size), "mlp_get_params")
        return out

    def set_params(self, p) -> None:
        a = np.ascontiguousarray(p, dtype=np.float32)
        _mcheck(_lib.mlp_set_params(self.h, _p(a), a.size), "mlp_set_params")

    def infer(self, x) -> np.ndarray:
        xr = _rows(x, self.cfg.in_dim)
        y = np.empty(xr.shape[0], np.float32)
        _mcheck(_lib.mlp_infer(self.h, _p(xr), _p(y), xr.shape[0]), "mlp_infer")
        return y

    def grad(self, x, t):
        xr = _rows(x, self.cfg.in_dim)
        tr = np.ascontiguousarray(t, dtype=np.float32).reshape(-1)
        g = np.empty(self.n_params, np.float32)
        loss = ctypes.c_float()
        _mcheck(_lib.mlp_grad(self.h, _p(xr), _p(tr), xr.shape[0], _p(g), ctypes.byref(loss)), "mlp_grad")
        return g, loss.value

    def fit(self, x, t, steps: int, batch: int = 4096, lr: float = 1e-3, seed: int = 1) -> float:
        """Adam steps on minibatches drawn from the rows (x, t); returns the last batch loss."""
        xr = _rows(x, self.cfg.in_dim)
        tr = np.ascontiguousarray(t, dtype=np.float32).reshape(-1)
        loss = ctypes.c_float()
        _mcheck(_lib.mlp_fit(self.h, _p(xr), _p(tr), xr.shape[0], batch, steps, lr, seed,
                             ctypes.byref(loss)), "mlp_fit")
        return loss.value

    def warm_table(self, model: str, q: int, L: int) -> np.ndarray:
        W = L * L + 1 if model == "ising" else 2 * L * L + 1
        out = np.empty(W, np.float64)
        _mcheck(_lib.mlp_warm_table(self.h, MODELS[model], q, L, _p(out)), "mlp_warm_table")
        return out
