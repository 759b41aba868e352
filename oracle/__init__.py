"""Plain CPU reference for replica-exchange Wang-Landau (arXiv:1407.5140).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path never does.
Nothing here is shared with the GPU library (`paper_1407_5140_amd`).

* ``rewl_oracle.c``  -- the REWL algorithm of Sec. II.A/II.B in plain C
  (per-walker ln g and H kept literally, OpenMP over walkers between sync points).
* ``exact_dos.py``   -- exact densities of states used to pin the oracle
  (brute force, transfer matrix, Kaufman's torus partition function).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rewl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle into oracle/liboracle.so (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp,
                               "-lquadmath", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Config(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("q", ctypes.c_int32), ("L", ctypes.c_int32),
                ("n_windows", ctypes.c_int32), ("overlap_num", ctypes.c_int32),
                ("overlap_den", ctypes.c_int32), ("walkers_per_window", ctypes.c_int32),
                ("flat_num", ctypes.c_int32), ("flat_den", ctypes.c_int32),
                ("lnf_k0", ctypes.c_int32), ("lnf_kfinal", ctypes.c_int32),
                ("exchange_enabled", ctypes.c_int32), ("exchange_interval", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("flat_rule", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("window_lo", ctypes.c_void_p), ("window_hi", ctypes.c_void_p)]


def make_config(model="ising", q=2, L=8, n_windows=4, overlap=(3, 4), m=1, flat=(4, 5),
                k0=0, kfinal=20, X=10000, seed=1, exchange=True, flat_rule="mean",
                windows=None) -> Config:
    """flat_rule "mean": min H >= num/den of the mean (Sec. II.A); "visits":
    H(E) >= (num/den)/sqrt(ln f) for every E, Eq. (8).  windows: optional
    (lo, hi) sequences of inclusive global bins (unequal widths); the config
    keeps the arrays alive."""
    c = Config(0 if model == "ising" else 1, q, L, n_windows, overlap[0], overlap[1], m,
               flat[0], flat[1], k0, kfinal, 1 if exchange else 0, X, seed,
               {"mean": 0, "visits": 1}[flat_rule], 0, None, None)
    if windows is not None:
        c._wlo = np.ascontiguousarray(windows[0], dtype=np.int32)
        c._whi = np.ascontiguousarray(windows[1], dtype=np.int32)
        c.window_lo = c._wlo.ctypes.data
        c.window_hi = c._whi.ctypes.data
    return c


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        L.orc_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.orc_accept.argtypes = [ctypes.c_double, ctypes.c_uint64]
        L.orc_accept.restype = ctypes.c_int
        L.orc_n_bins.argtypes = [P(Config)]
        L.orc_n_bins.restype = ctypes.c_int32
        L.orc_layout.argtypes = [P(Config), P(ctypes.c_int32), P(ctypes.c_int32)]
        L.orc_mask_rule.argtypes = [P(Config), P(ctypes.c_uint8)]
        L.orc_energy.argtypes = [P(Config), P(ctypes.c_uint8)]
        L.orc_energy.restype = ctypes.c_int64
        L.orc_create.argtypes = [P(Config), ctypes.c_void_p, ctypes.c_void_p, P(ctypes.c_int)]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_run.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        L.orc_run.restype = ctypes.c_int
        L.orc_interval.argtypes = [ctypes.c_void_p]
        L.orc_interval.restype = ctypes.c_int64
        L.orc_window_bins.argtypes = [ctypes.c_void_p]
        L.orc_window_bins.restype = ctypes.c_int32
        L.orc_get_state.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 8
        L.orc_window_lng.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        L.orc_set_window_lng.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        L.orc_stats.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 3
        L.orc_init_attempts_max.argtypes = [ctypes.c_void_p]
        L.orc_init_attempts_max.restype = ctypes.c_int
        L.orc_concat.argtypes = [P(Config), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p]
        L.orc_concat.restype = ctypes.c_int
        L.orc_boot_picks.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_void_p]
        L.orc_boot_picks.restype = ctypes.c_int
        L.orc_replicas.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_set_tables.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_test_exchange_mutation.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(o)


def accept(delta: float, u53: int) -> bool:
    return bool(lib().orc_accept(float(delta), int(u53)))


def n_bins(cfg: Config) -> int:
    return lib().orc_n_bins(ctypes.byref(cfg))


def layout(cfg: Config):
    h = cfg.n_windows
    lo = (ctypes.c_int32 * h)()
    hi = (ctypes.c_int32 * h)()
    if lib().orc_layout(ctypes.byref(cfg), lo, hi) != 0:
        raise ValueError("invalid layout")
    return np.array(lo, dtype=np.int64), np.array(hi, dtype=np.int64)


def mask_rule(cfg: Config) -> np.ndarray:
    m = np.zeros(n_bins(cfg), dtype=np.uint8)
    lib().orc_mask_rule(ctypes.byref(cfg), m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return m


def energy(cfg: Config, spins) -> int:
    s = np.ascontiguousarray(spins, dtype=np.uint8)
    return int(lib().orc_energy(ctypes.byref(cfg), s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))


def concat(cfg: Config, mask: np.ndarray, pieces: np.ndarray):
    W = n_bins(cfg)
    out = np.empty(W, dtype=np.float64)
    join = np.zeros(max(cfg.n_windows - 1, 1), dtype=np.int32)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    p = np.ascontiguousarray(pieces, dtype=np.float64)
    rc = lib().orc_concat(ctypes.byref(cfg), _ptr(m), _ptr(p), _ptr(out), _ptr(join))
    if rc != 0:
        raise ValueError(f"concatenation failed ({rc})")
    return out, join[: max(cfg.n_windows - 1, 0)]


def boot_picks(seed: int, R: int, h: int, n: int) -> np.ndarray:
    """Run index of every draw, shape (R + 1, h, n); resample 0 is the ensemble itself."""
    out = np.zeros((R + 1, h, n), dtype=np.int32)
    if lib().orc_boot_picks(int(seed), int(R), int(h), int(n), _ptr(out)) != 0:
        raise ValueError("invalid bootstrap size")
    return out


class Sim:
    """One REWL run of the oracle (state kept in host memory)."""

    def __init__(self, cfg: Config, mask=None, init_lng=None):
        self.cfg = cfg
        self._mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        self._init = None if init_lng is None else np.ascontiguousarray(init_lng, dtype=np.float64)
        st = ctypes.c_int(0)
        h = lib().orc_create(ctypes.byref(cfg),
                             None if self._mask is None else _ptr(self._mask),
                             None if self._init is None else _ptr(self._init), ctypes.byref(st))
        if not h:
            raise ValueError(f"oracle create failed (status {st.value})")
        self.h = h
        self.N = cfg.L * cfg.L
        self.S = cfg.n_windows * cfg.walkers_per_window
        self.WB = lib().orc_window_bins(h)
        self.lo, self.hi = layout(cfg)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def run(self, n_intervals: int, threads: int = 0) -> bool:
        rc = lib().orc_run(self.h, int(n_intervals), int(threads))
        if rc < 0:
            raise RuntimeError(f"oracle run failed ({rc})")
        return bool(rc)

    @property
    def t(self) -> int:
        return int(lib().orc_interval(self.h))

    def state(self) -> dict:
        S, N, WB, h = self.S, self.N, self.WB, self.cfg.n_windows
        st = dict(spins=np.empty((S, N), np.uint8), bins=np.empty(S, np.int32),
                  H=np.empty((S, WB), np.int64), lng=np.empty((S, WB), np.float64),
                  flat=np.empty(S, np.uint8), k=np.empty(h, np.int32),
                  done=np.empty(h, np.uint8), swaps=np.empty(S, np.int8))
        lib().orc_get_state(self.h, *[_ptr(st[n]) for n in
                                      ("spins", "bins", "H", "lng", "flat", "k", "done", "swaps")])
        st["t"] = self.t
        return st

    def window_lng(self, a: int) -> np.ndarray:
        out = np.empty(self.WB, np.float64)
        lib().orc_window_lng(self.h, int(a), _ptr(out))
        return out

    def set_window_lng(self, a: int, tab) -> None:
        t = np.ascontiguousarray(tab, dtype=np.float64)
        assert t.shape == (self.WB,)
        lib().orc_set_window_lng(self.h, int(a), _ptr(t))

    def pieces(self) -> np.ndarray:
        return np.stack([self.window_lng(a) for a in range(self.cfg.n_windows)])

    def stats(self) -> dict:
        h = self.cfg.n_windows
        att = ctypes.c_int64(0)
        p = np.zeros(h, np.int64)
        a = np.zeros(h, np.int64)
        lib().orc_stats(self.h, ctypes.byref(att), _ptr(p), _ptr(a))
        return dict(attempts=att.value, ex_prop=p, ex_acc=a)

    def init_attempts_max(self) -> int:
        return int(lib().orc_init_attempts_max(self.h))

    def replicas(self) -> dict:
        """rid[S]: replica held by each slot; round_trips[S]: completed round trips
        0 -> h-1 -> 0 of each replica (Sec. IV.A)."""
        rid = np.empty(self.S, np.int32)
        rt = np.empty(self.S, np.int32)
        lib().orc_replicas(self.h, _ptr(rid), _ptr(rt))
        return dict(rid=rid, round_trips=rt)

    def set_tables(self, H=None, lng=None) -> None:
        """Replace every walker's counts and ln g (S x WB each)."""
        h = None if H is None else np.ascontiguousarray(H, dtype=np.int64)
        g = None if lng is None else np.ascontiguousarray(lng, dtype=np.float64)
        for a in (h, g):
            assert a is None or a.shape == (self.S, self.WB)
        lib().orc_set_tables(self.h, None if h is None else _ptr(h), None if g is None else _ptr(g))


def exchange_mutation(mode: int) -> None:
    """Test hook: plant a mistake in the oracle's exchange rule (0 restores Eq. (1))."""
    lib().orc_test_exchange_mutation(int(mode))
