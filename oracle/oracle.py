"""ctypes view of the C oracle -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads oracle/libmgfwa_oracle.so (built by oracle/build.py)
and exposes the plain CPU MGFWA: an independent Philox4x32-10, binary64 MLP
fitness, and the binary32 state path of one generation, phase by phase.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

ACT = {"identity": 0, "relu": 1, "tanh": 2, "gelu": 3}
LOSS = {"mse": 0, "ce": 1}
TAG = {"init": 0, "expl": 1, "expl_map": 2, "guide_map": 3, "reinit": 4}
MAX_LAYERS = 12
KIND = {"train": 0, "input": 1}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _build.up_to_date():
            _build.build()
        L = C.CDLL(_build.LIB)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_word.argtypes = [C.c_uint64, C.c_int, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_word.restype = C.c_uint32
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_float
        L.orc_dim.argtypes = [C.c_void_p]
        L.orc_n_params.argtypes = [C.c_void_p]
        L.orc_net_output.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_net_output.restype = C.c_double
        L.orc_loss.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_loss.restype = C.c_double
        L.orc_loss_rows.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        L.orc_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
        L.orc_threads.argtypes = [C.c_int]
        L.orc_threads.restype = C.c_int
        L.orc_init_row.argtypes = [C.c_void_p, C.c_int, C.c_uint32, C.c_uint32, C.c_int, C.c_void_p]
        L.orc_explosion_row.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_float, C.c_uint32,
                                        C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_population_range.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_population_range.restype = None
        L.orc_guide_group.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_float, C.c_float, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p]
        L.orc_create.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_error.restype = C.c_char_p
        for name in ("orc_init_positions", "orc_eval_init", "orc_explode", "orc_eval_explosion",
                     "orc_guide", "orc_eval_guiding", "orc_select"):
            getattr(L, name).argtypes = [C.c_void_p]
        for name in ("orc_tell_init", "orc_tell_explosion", "orc_tell_guiding"):
            getattr(L, name).argtypes = [C.c_void_p, C.c_void_p]
        L.orc_run.argtypes = [C.c_void_p, C.c_int]
        L.orc_get_view.argtypes = [C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


class _Problem(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("widths", C.c_int * (MAX_LAYERS + 1)),
                ("acts", C.c_int * MAX_LAYERS), ("loss", C.c_int), ("n_samples", C.c_int),
                ("x", C.c_void_p), ("y", C.c_void_p), ("labels", C.c_void_p),
                ("kind", C.c_int), ("net", C.c_void_p)]


class _Config(C.Structure):
    _fields_ = [("B", C.c_int), ("N", C.c_int), ("lam", C.c_int), ("G", C.c_int),
                ("sigma", C.c_float), ("boost", C.c_float), ("amp_up", C.c_float),
                ("amp_down", C.c_float), ("amp_init", C.c_float), ("lb", C.c_float),
                ("ub", C.c_float), ("T", C.c_int), ("seed", C.c_uint64),
                ("loser_out", C.c_int), ("use_target", C.c_int), ("target_loss", C.c_float),
                ("lag_guiding", C.c_int), ("map_range", C.c_int)]


class _View(C.Structure):
    _fields_ = [("D", C.c_int), ("m", C.c_int), ("k", C.c_int), ("t", C.c_int),
                ("done", C.c_int), ("inv_k", C.c_float)] + [
        (n, C.c_void_p) for n in ("F", "A", "Y", "Yprev", "fresh", "SE", "SG", "Yc", "Yc64",
                                  "top", "bottom", "tie", "cstar", "improved", "reinit",
                                  "best_f", "best_x", "best_y", "best_gen")]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Problem:
    """MLP loss problem (the spark is the MLP's parameters), or with net= the
    paper's testbed (the spark is the input of the fixed MLP whose parameters
    are `net`; the fitness is its scalar output).  Holds references to the
    arrays it points at."""

    def __init__(self, widths, acts, loss="mse", x=None, y=None, labels=None, net=None):
        widths = [int(w) for w in widths]
        L = len(widths) - 1
        if not 1 <= L <= MAX_LAYERS:
            raise ValueError("layers")
        self.widths, self.acts, self.loss = widths, list(acts), loss
        self.x = None if x is None else np.ascontiguousarray(x, dtype=np.float32)
        self.y = None if y is None else np.ascontiguousarray(y, dtype=np.float32)
        self.labels = None if labels is None else np.ascontiguousarray(labels, dtype=np.int32)
        s = _Problem()
        s.n_layers = L
        for i, w in enumerate(widths):
            s.widths[i] = w
        for i, a in enumerate(self.acts):
            s.acts[i] = ACT[a]
        s.loss = LOSS[loss]
        s.n_samples = 0 if self.x is None else self.x.shape[0]
        s.x, s.y, s.labels = _ptr(self.x), _ptr(self.y), _ptr(self.labels)
        self.net = None if net is None else np.ascontiguousarray(net, dtype=np.float32)
        s.kind = KIND["input" if net is not None else "train"]
        s.net = _ptr(self.net)
        if net is not None and self.net.size != lib().orc_n_params(C.byref(s)):
            raise ValueError("net parameter count does not match the widths")
        self.s = s

    @classmethod
    def from_workload(cls, wl):
        if getattr(wl, "net", None) is not None:
            return cls(wl.widths, wl.acts, net=wl.net)
        return cls(wl.widths, wl.acts, wl.loss, wl.x, wl.y, wl.labels)

    @property
    def n_params(self) -> int:
        return lib().orc_n_params(C.byref(self.s))

    def output(self, x) -> float:
        """The fixed network's output at input x (input problems)."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        return lib().orc_net_output(C.byref(self.s), _ptr(x))

    @property
    def dim(self) -> int:
        return lib().orc_dim(C.byref(self.s))

    def loss_of(self, w, per_sample: bool = False):
        w = np.ascontiguousarray(w, dtype=np.float32)
        if per_sample:
            ps = np.zeros(self.s.n_samples, dtype=np.float64)
            v = lib().orc_loss(C.byref(self.s), _ptr(w), _ptr(ps))
            return v, ps
        return lib().orc_loss(C.byref(self.s), _ptr(w), None)

    def loss_rows(self, W):
        W = np.ascontiguousarray(W, dtype=np.float32)
        out = np.zeros(W.shape[0], dtype=np.float64)
        lib().orc_loss_rows(C.byref(self.s), _ptr(W), W.shape[0], W.shape[1], _ptr(out))
        return out

    def forward(self, w, sample: int):
        w = np.ascontiguousarray(w, dtype=np.float32)
        out = np.zeros(self.widths[-1], dtype=np.float64)
        lib().orc_forward(C.byref(self.s), _ptr(w), int(sample), _ptr(out))
        return out


def threads(n: int = 0) -> int:
    """Threads of the oracle's fitness loops: n > 0 sets them; returns the count in force."""
    return int(lib().orc_threads(int(n)))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def word(seed, tag, row, t, d):
    return int(lib().orc_word(int(seed), TAG[tag] if isinstance(tag, str) else int(tag),
                              int(row), int(t), int(d)))


def u01(r):
    return float(np.float32(lib().orc_u01(int(r))))


DEFAULTS = dict(B=1, N=4, lam=32, G=4, sigma=0.2, boost=1.0, amp_up=1.2, amp_down=0.9,
                amp_init=None, lb=-5.0, ub=5.0, T=100, seed=0, loser_out=1, use_target=0,
                target_loss=0.0, lag_guiding=0, map_range=0)


def make_config(**kw) -> _Config:
    d = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise TypeError(k)
        d[k] = v
    if d["amp_init"] is None:
        d["amp_init"] = float(np.float32(d["ub"]) - np.float32(d["lb"]))
    c = _Config()
    for k, v in d.items():
        setattr(c, k, v)
    return c


def init_row(cfg: _Config, dim, row, t, tag="init"):
    out = np.zeros(dim, dtype=np.float32)
    lib().orc_init_row(C.byref(cfg), int(dim), int(row), int(t), TAG[tag], _ptr(out))
    return out


def explosion_row(cfg: _Config, x, amp, row, t, lo=None, hi=None):
    """Explosion spark; lo/hi: the population range for range mapping (None: the box)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.zeros_like(x)
    lo = None if lo is None else np.ascontiguousarray(lo, dtype=np.float32)
    hi = None if hi is None else np.ascontiguousarray(hi, dtype=np.float32)
    lib().orc_explosion_row(C.byref(cfg), x.shape[0], _ptr(x), float(amp), int(row), int(t),
                            _ptr(lo), _ptr(hi), _ptr(out))
    return out


def population_range(F):
    """Per-dimension (min, max) over the rows of F, as the oracle computes them."""
    F = np.ascontiguousarray(F, dtype=np.float32)
    lo = np.zeros(F.shape[1], dtype=np.float32)
    hi = np.zeros(F.shape[1], dtype=np.float32)
    lib().orc_population_range(F.shape[0], F.shape[1], _ptr(F), _ptr(lo), _ptr(hi))
    return lo, hi


def guide_group(sparks, y, x, k, boost=1.0):
    """One guiding group: returns (top, bottom, tie, unmapped guiding spark)."""
    sparks = np.ascontiguousarray(sparks, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    m, dim = sparks.shape
    top = np.zeros(k, dtype=np.int32)
    bot = np.zeros(k, dtype=np.int32)
    tie = np.zeros(1, dtype=np.int32)
    gs = np.zeros(dim, dtype=np.float32)
    inv_k = float(np.float32(1.0 / k))
    lib().orc_guide_group(m, k, dim, _ptr(sparks), _ptr(y), _ptr(x), float(boost), inv_k,
                          _ptr(top), _ptr(bot), _ptr(tie), _ptr(gs))
    return top, bot, int(tie[0]), gs


class Oracle:
    """One MGFWA run on the CPU, steppable phase by phase."""

    def __init__(self, problem: Problem, **cfg):
        self.problem = problem
        self.cfg = make_config(**cfg)
        h = lib().orc_create(C.byref(self.cfg), C.byref(problem.s))
        if not h:
            raise ValueError(lib().orc_error().decode())
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def _call(self, name, *args):
        rc = getattr(lib(), name)(self.h, *args)
        if rc != 0:
            raise RuntimeError(lib().orc_error().decode())

    # phases
    def init_positions(self): self._call("orc_init_positions")
    def eval_init(self): self._call("orc_eval_init")
    def explode(self): self._call("orc_explode")
    def eval_explosion(self): self._call("orc_eval_explosion")
    def guide(self): self._call("orc_guide")
    def eval_guiding(self): self._call("orc_eval_guiding")
    def select(self): self._call("orc_select")

    def tell_init(self, y): self._tell("orc_tell_init", y)
    def tell_explosion(self, y): self._tell("orc_tell_explosion", y)
    def tell_guiding(self, y): self._tell("orc_tell_guiding", y)

    def _tell(self, name, y):
        y = np.ascontiguousarray(y, dtype=np.float32)
        self._call(name, _ptr(y))

    def init(self):
        self.init_positions()
        self.eval_init()

    def generation(self):
        if self.cfg.lag_guiding:   # Alg. 1 literally: guide from the previous sparks first
            self.guide()
            self.explode()
            self.eval_explosion()
            self.eval_guiding()
        else:
            self.explode()
            self.eval_explosion()
            self.guide()
            self.eval_guiding()
        self.select()

    def run(self, n):
        self._call("orc_run", int(n))

    # state
    def view(self):
        v = _View()
        lib().orc_get_view(self.h, C.byref(v))
        c = self.cfg
        BN, D, lam, G, k = c.B * c.N, v.D, c.lam, c.G, v.k
        Cn = lam + G

        def arr(p, shape, dt):
            n = int(np.prod(shape))
            if n == 0:
                return np.zeros(shape, dtype=dt)
            buf = (C.c_char * (n * np.dtype(dt).itemsize)).from_address(p)
            return np.frombuffer(buf, dtype=dt).reshape(shape).copy()

        return dict(
            D=v.D, m=v.m, k=v.k, t=v.t, done=v.done, inv_k=v.inv_k,
            F=arr(v.F, (BN, D), np.float32), A=arr(v.A, (BN,), np.float32),
            Y=arr(v.Y, (BN,), np.float32), Yprev=arr(v.Yprev, (BN,), np.float32),
            fresh=arr(v.fresh, (BN,), np.int32),
            SE=arr(v.SE, (BN * lam, D), np.float32), SG=arr(v.SG, (BN * G, D), np.float32),
            Yc=arr(v.Yc, (BN, Cn), np.float32), Yc64=arr(v.Yc64, (BN, Cn), np.float64),
            top=arr(v.top, (BN * G, k), np.int32), bottom=arr(v.bottom, (BN * G, k), np.int32),
            tie=arr(v.tie, (BN * G,), np.int32), cstar=arr(v.cstar, (BN,), np.int32),
            improved=arr(v.improved, (BN,), np.int32), reinit=arr(v.reinit, (BN,), np.int32),
            best_f=arr(v.best_f, (c.B,), np.int32), best_x=arr(v.best_x, (c.B, D), np.float32),
            best_y=arr(v.best_y, (c.B,), np.float32), best_gen=arr(v.best_gen, (c.B,), np.int32))
