"""Thin ctypes binding of libmgfwa.so (declared in include/mgfwa.h).

Argument marshalling only: every step of the generation loop runs in the HIP
library.  PyTorch supplies device memory (the workspace and problem buffers)
and the stream.  Importing this module fails loudly when the library has not
been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgfwa.so")

MAX_LAYERS = 12         # Linear layers of a problem's MLP
MAX_TRAIN_LAYERS = 4    # ... when the spark is the MLP's weights
MAX_WIDTH = 256
KIND = {"weights": 0, "input": 1}
N_PHASES = 5
PHASES = ("explosion", "fitness_explosion", "guiding", "fitness_guiding", "selection")

OK, EINVAL, ENOMEM, EHIP, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
ACT = {"identity": 0, "relu": 1, "tanh": 2, "gelu": 3}
LOSS = {"mse": 0, "ce": 1}
PRECISION = {"fp32": 0, "bf16": 1}


class mgfwa_problem(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("widths", C.c_int * (MAX_LAYERS + 1)),
                ("hidden_act", C.c_int * MAX_LAYERS), ("loss", C.c_int), ("n_samples", C.c_int),
                ("x_dev", C.c_void_p), ("y_dev", C.c_void_p), ("labels_dev", C.c_void_p),
                ("kind", C.c_int), ("net_dev", C.c_void_p)]


class mgfwa_config(C.Structure):
    _fields_ = [("n_populations", C.c_int), ("n_fireworks", C.c_int), ("n_sparks", C.c_int),
                ("n_guiding", C.c_int), ("sigma", C.c_float), ("boost", C.c_float),
                ("amp_up", C.c_float), ("amp_down", C.c_float), ("amp_init", C.c_float),
                ("lb", C.c_float), ("ub", C.c_float), ("max_generations", C.c_int),
                ("loser_out", C.c_int), ("precision", C.c_int), ("external_fitness", C.c_int),
                ("use_target", C.c_int), ("target_loss", C.c_float), ("seed", C.c_uint64),
                ("lag_guiding", C.c_int), ("map_range", C.c_int), ("fit_path", C.c_int), ("regen_sparks", C.c_int)]


_STATE_ARRAYS = ("F", "A", "Y", "Yprev", "fresh", "SE", "SG", "Yc", "top", "bottom", "tie",
                 "cstar", "improved", "reinit", "best_x", "best_y", "best_f", "best_gen", "gen",
                 "done")


class mgfwa_state_info(C.Structure):
    _fields_ = [("D", C.c_int), ("Dp", C.c_int), ("m", C.c_int), ("k", C.c_int),
                ("n_candidates", C.c_int), ("generation", C.c_int)] + [
        (n, C.c_size_t) for n in _STATE_ARRAYS] + [("se_written", C.c_int)]


class mgfwa_timing_info(C.Structure):
    _fields_ = [("ms", C.c_double * N_PHASES), ("gen_ms_p50", C.c_double),
                ("gen_ms_p99", C.c_double), ("gen_ms_mean", C.c_double),
                ("fit_kernel_ms", C.c_double), ("check_fit_ms", C.c_double),
                ("generations", C.c_int)]


class mgfwa_job_info(C.Structure):
    _fields_ = [("state", C.c_int), ("generations", C.c_int), ("best_fitness", C.c_float),
                ("workspace_bytes", C.c_size_t), ("submit_ms", C.c_double),
                ("admit_ms", C.c_double), ("finish_ms", C.c_double)]


class mgfwa_server_stats(C.Structure):
    _fields_ = [("queued", C.c_int), ("running", C.c_int), ("done", C.c_int), ("failed", C.c_int),
                ("generations", C.c_long), ("gen_ms_p50", C.c_double), ("gen_ms_p99", C.c_double),
                ("wall_ms", C.c_double), ("spark_evals_per_s", C.c_double),
                ("arena_bytes", C.c_size_t), ("arena_used", C.c_size_t),
                ("arena_peak", C.c_size_t)]


JOB_STATE = {0: "queued", 1: "running", 2: "done", 3: "failed"}


class mgfwa_plan_info(C.Structure):
    _fields_ = [("wide", C.c_int), ("rows", C.c_int), ("wavefronts", C.c_int), ("slabs", C.c_int),
                ("lds_weights", C.c_int), ("blocks_per_row", C.c_int),
                ("samples_per_block", C.c_int), ("lds_bytes", C.c_int),
                ("row_blocks", C.c_int * 4), ("net_kernel", C.c_int)]


class MgfwaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"mgfwa status {status}: {message}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2501_03944_amd.build` (needs hipcc)")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    L.mgfwa_workspace_bytes.argtypes = [P(mgfwa_config), P(mgfwa_problem)]
    L.mgfwa_workspace_bytes.restype = C.c_size_t
    L.mgfwa_init.argtypes = [P(C.c_void_p), P(mgfwa_config), P(mgfwa_problem), C.c_void_p,
                             C.c_size_t, C.c_void_p]
    L.mgfwa_step.argtypes = [C.c_void_p, C.c_int]
    L.mgfwa_best.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.mgfwa_best_all.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.mgfwa_ask.argtypes = [C.c_void_p, P(C.c_void_p), P(C.c_int), P(C.c_int)]
    L.mgfwa_tell.argtypes = [C.c_void_p, C.c_void_p]
    L.mgfwa_evaluate.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    L.mgfwa_evaluate_noalloc.argtypes = [P(mgfwa_problem), C.c_int, C.c_void_p, C.c_int, C.c_int,
                                         C.c_void_p, C.c_void_p]
    L.mgfwa_state.argtypes = [C.c_void_p, P(mgfwa_state_info)]
    L.mgfwa_set_timing.argtypes = [C.c_void_p, C.c_int]
    L.mgfwa_timing.argtypes = [C.c_void_p, P(mgfwa_timing_info)]
    L.mgfwa_destroy.argtypes = [C.c_void_p]
    L.mgfwa_destroy.restype = None
    L.mgfwa_last_error.restype = C.c_char_p
    L.mgfwa_version.restype = C.c_char_p
    L.mgfwa_autotune.argtypes = [C.c_void_p, C.c_int]
    L.mgfwa_fit_plan.argtypes = [C.c_void_p, C.c_int, P(mgfwa_plan_info)]
    L.mgfwa_fit_candidates.argtypes = [C.c_void_p, C.c_int, P(mgfwa_plan_info), C.c_int,
                                       P(C.c_int)]
    L.mgfwa_set_fit_plan.argtypes = [C.c_void_p, C.c_int, C.c_int]
    L.mgfwa_batch_create.argtypes = [P(C.c_void_p), P(C.c_void_p), C.c_int, C.c_void_p]
    L.mgfwa_batch_step.argtypes = [C.c_void_p, C.c_int]
    L.mgfwa_batch_destroy.argtypes = [C.c_void_p]
    L.mgfwa_batch_destroy.restype = None
    L.mgfwa_server_create.argtypes = [P(C.c_void_p), C.c_void_p, C.c_size_t, C.c_int]
    L.mgfwa_server_submit.argtypes = [C.c_void_p, P(mgfwa_config), P(mgfwa_problem),
                                      P(C.c_int64)]
    L.mgfwa_server_tick.argtypes = [C.c_void_p]
    L.mgfwa_server_drain.argtypes = [C.c_void_p]
    L.mgfwa_server_job.argtypes = [C.c_void_p, C.c_int64, P(mgfwa_job_info), C.c_void_p]
    L.mgfwa_server_stats_get.argtypes = [C.c_void_p, P(mgfwa_server_stats)]
    L.mgfwa_server_destroy.argtypes = [C.c_void_p]
    L.mgfwa_server_destroy.restype = None
    for name in ("mgfwa_init", "mgfwa_step", "mgfwa_best", "mgfwa_best_all", "mgfwa_ask",
                 "mgfwa_tell", "mgfwa_evaluate", "mgfwa_evaluate_noalloc", "mgfwa_state",
                 "mgfwa_set_timing",
                 "mgfwa_timing", "mgfwa_autotune", "mgfwa_fit_plan", "mgfwa_fit_candidates",
                 "mgfwa_set_fit_plan", "mgfwa_batch_create",
                 "mgfwa_batch_step", "mgfwa_server_create", "mgfwa_server_submit",
                 "mgfwa_server_tick", "mgfwa_server_drain", "mgfwa_server_job",
                 "mgfwa_server_stats_get"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status: int) -> None:
    if status != OK:
        raise MgfwaError(status, lib().mgfwa_last_error().decode())


def make_config(n_fireworks=4, n_sparks=32, n_guiding=4, n_populations=1, sigma=0.2, boost=1.0,
                amp_up=1.2, amp_down=0.9, amp_init=0.0, lb=-5.0, ub=5.0, max_generations=100,
                loser_out=True, precision="fp32", external_fitness=False, target_loss=None,
                seed=0, lag_guiding=False, map_range=False, fit_path=0,
                regen_sparks=False) -> mgfwa_config:
    c = mgfwa_config()
    c.n_populations, c.n_fireworks, c.n_sparks, c.n_guiding = (
        n_populations, n_fireworks, n_sparks, n_guiding)
    c.sigma, c.boost, c.amp_up, c.amp_down, c.amp_init = sigma, boost, amp_up, amp_down, amp_init
    c.lb, c.ub, c.max_generations = lb, ub, max_generations
    c.loser_out = int(bool(loser_out))
    c.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    c.external_fitness = int(bool(external_fitness))
    c.use_target = int(target_loss is not None)
    c.target_loss = 0.0 if target_loss is None else float(target_loss)
    c.seed = int(seed)
    c.lag_guiding = int(bool(lag_guiding))
    c.map_range = int(bool(map_range))
    c.fit_path = int(fit_path)
    c.regen_sparks = int(bool(regen_sparks))
    return c


def make_problem(widths, acts, loss, n_samples, x_ptr=0, y_ptr=0, labels_ptr=0,
                 net_ptr=None) -> mgfwa_problem:
    """A weights problem, or with net_ptr (0 for external fitness) an input
    problem: the spark is the input of the fixed network at net_ptr."""
    p = mgfwa_problem()
    p.n_layers = len(widths) - 1
    for i, w in enumerate(widths):
        p.widths[i] = int(w)
    for i, a in enumerate(acts):
        p.hidden_act[i] = ACT[a] if isinstance(a, str) else int(a)
    p.loss = LOSS[loss] if isinstance(loss, str) else int(loss or 0)
    p.n_samples = int(n_samples)
    p.x_dev, p.y_dev, p.labels_dev = x_ptr or None, y_ptr or None, labels_ptr or None
    p.kind = KIND["weights" if net_ptr is None else "input"]
    p.net_dev = net_ptr or None
    return p


# ---- C-ABI entry points under their own names (serving below) ---------------------------------------
def mgfwa_workspace_bytes(config: mgfwa_config, problem: mgfwa_problem) -> int:
    return int(lib().mgfwa_workspace_bytes(C.byref(config), C.byref(problem)))


def mgfwa_init(config, problem, workspace_ptr: int, workspace_bytes: int, stream: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().mgfwa_init(C.byref(h), C.byref(config), C.byref(problem), C.c_void_p(workspace_ptr),
                            workspace_bytes, C.c_void_p(stream or None)))
    return h


def mgfwa_step(ctx, n: int) -> None:
    _check(lib().mgfwa_step(ctx, int(n)))


def mgfwa_best(ctx, dim: int):
    x = np.zeros(dim, dtype=np.float32)
    f = C.c_float()
    g = C.c_int()
    _check(lib().mgfwa_best(ctx, x.ctypes.data_as(C.c_void_p), C.byref(f), C.byref(g)))
    return x, float(f.value), int(g.value)


def mgfwa_best_all(ctx, B: int, dim: int):
    x = np.zeros((B, dim), dtype=np.float32)
    f = np.zeros(B, dtype=np.float32)
    g = np.zeros(B, dtype=np.int32)
    _check(lib().mgfwa_best_all(ctx, x.ctypes.data_as(C.c_void_p), f.ctypes.data_as(C.c_void_p),
                                g.ctypes.data_as(C.c_void_p)))
    return x, f, g


def mgfwa_ask(ctx):
    p = C.c_void_p()
    rows = C.c_int()
    ld = C.c_int()
    _check(lib().mgfwa_ask(ctx, C.byref(p), C.byref(rows), C.byref(ld)))
    return int(p.value or 0), int(rows.value), int(ld.value)


def mgfwa_tell(ctx, fitness_ptr: int) -> None:
    _check(lib().mgfwa_tell(ctx, C.c_void_p(fitness_ptr)))


def mgfwa_evaluate(ctx, w_ptr: int, rows: int, ld: int, out_ptr: int) -> None:
    _check(lib().mgfwa_evaluate(ctx, C.c_void_p(w_ptr), int(rows), int(ld), C.c_void_p(out_ptr)))


def mgfwa_evaluate_noalloc(problem: mgfwa_problem, precision: int, w_ptr: int, rows: int,
                           ld: int, out_ptr: int, stream: int) -> None:
    _check(lib().mgfwa_evaluate_noalloc(C.byref(problem), int(precision), w_ptr, rows, ld,
                                        out_ptr, stream))


def mgfwa_state(ctx) -> mgfwa_state_info:
    info = mgfwa_state_info()
    _check(lib().mgfwa_state(ctx, C.byref(info)))
    return info


def mgfwa_set_timing(ctx, on: bool) -> None:
    _check(lib().mgfwa_set_timing(ctx, int(bool(on))))


def mgfwa_timing(ctx) -> dict:
    info = mgfwa_timing_info()
    _check(lib().mgfwa_timing(ctx, C.byref(info)))
    return {"phase_ms": dict(zip(PHASES, list(info.ms))), "gen_ms_p50": info.gen_ms_p50,
            "gen_ms_p99": info.gen_ms_p99, "gen_ms_mean": info.gen_ms_mean,
            "fit_kernel_ms": info.fit_kernel_ms, "check_fit_ms": info.check_fit_ms,
            "generations": info.generations}


def mgfwa_destroy(ctx) -> None:
    lib().mgfwa_destroy(ctx)


def mgfwa_last_error() -> str:
    return lib().mgfwa_last_error().decode()


def mgfwa_version() -> str:
    return lib().mgfwa_version().decode()


# ---- convenience wrapper holding the torch-owned device buffers -------------------------
def mgfwa_autotune(ctx, reps: int = 3) -> None:
    _check(lib().mgfwa_autotune(ctx, int(reps)))


def mgfwa_fit_plan(ctx, which: int) -> dict:
    info = mgfwa_plan_info()
    _check(lib().mgfwa_fit_plan(ctx, int(which), C.byref(info)))
    return _plan_dict(info)


def _plan_dict(info: mgfwa_plan_info) -> dict:
    d = {name: getattr(info, name) for name, _ in mgfwa_plan_info._fields_}
    d["row_blocks"] = list(info.row_blocks)
    return d


def mgfwa_fit_candidates(ctx, which: int) -> list:
    n = C.c_int()
    _check(lib().mgfwa_fit_candidates(ctx, int(which), None, 0, C.byref(n)))
    arr = (mgfwa_plan_info * max(1, n.value))()
    _check(lib().mgfwa_fit_candidates(ctx, int(which), arr, n.value, C.byref(n)))
    return [_plan_dict(arr[i]) for i in range(n.value)]


def mgfwa_set_fit_plan(ctx, which: int, index: int) -> None:
    _check(lib().mgfwa_set_fit_plan(ctx, int(which), int(index)))


def mgfwa_batch_create(ctxs, stream: int) -> C.c_void_p:
    arr = (C.c_void_p * len(ctxs))(*[c.value if isinstance(c, C.c_void_p) else c for c in ctxs])
    h = C.c_void_p()
    _check(lib().mgfwa_batch_create(C.byref(h), arr, len(ctxs), C.c_void_p(stream or None)))
    return h


def mgfwa_batch_step(batch, n: int) -> None:
    _check(lib().mgfwa_batch_step(batch, int(n)))


def mgfwa_batch_destroy(batch) -> None:
    lib().mgfwa_batch_destroy(batch)


def mgfwa_server_create(arena_ptr: int, arena_bytes: int, n_streams: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().mgfwa_server_create(C.byref(h), C.c_void_p(arena_ptr), arena_bytes, n_streams))
    return h


def mgfwa_server_submit(server, config: mgfwa_config, problem: mgfwa_problem) -> int:
    jid = C.c_int64()
    _check(lib().mgfwa_server_submit(server, C.byref(config), C.byref(problem), C.byref(jid)))
    return jid.value


def mgfwa_server_tick(server) -> None:
    _check(lib().mgfwa_server_tick(server))


def mgfwa_server_drain(server) -> None:
    _check(lib().mgfwa_server_drain(server))


def mgfwa_server_job(server, job_id: int, dim: int = 0):
    info = mgfwa_job_info()
    x = np.zeros(dim, dtype=np.float32) if dim else None
    _check(lib().mgfwa_server_job(server, job_id, C.byref(info),
                                  x.ctypes.data_as(C.c_void_p) if dim else None))
    d = {name: getattr(info, name) for name, _ in mgfwa_job_info._fields_}
    d["state"] = JOB_STATE[d["state"]]
    return d, x


def mgfwa_server_stats_get(server) -> dict:
    st = mgfwa_server_stats()
    _check(lib().mgfwa_server_stats_get(server, C.byref(st)))
    return {name: getattr(st, name) for name, _ in mgfwa_server_stats._fields_}


def mgfwa_server_destroy(server) -> None:
    lib().mgfwa_server_destroy(server)


class MGFWA:
    """One optimisation job: problem buffers and workspace as torch CUDA tensors.
    With net= (the fixed network's parameters) the spark is that network's input
    and the fitness its output (the paper's testbed); loss and samples are then
    unused."""

    def __init__(self, widths, acts, loss=None, x=None, y=None, labels=None, device="cuda",
                 stream=None, net=None, **config):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.widths = [int(w) for w in widths]
        self.acts = list(acts)
        self.loss = loss
        self._keep = []

        def dev(a, dtype):
            if a is None:
                return None
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            t = t.to(device=self.device, dtype=dtype).contiguous()
            self._keep.append(t)
            return t

        xt = dev(x, torch.float32)
        yt = dev(y, torch.float32) if loss == "mse" else None
        lt = dev(labels, torch.int32) if loss == "ce" else None
        n_samples = 0 if xt is None else xt.shape[0]
        # net=True: an input problem without parameters (external fitness)
        nt = dev(net, torch.float32) if net is not None and not isinstance(net, bool) else None
        self.problem = make_problem(self.widths, self.acts, loss, n_samples,
                                    0 if xt is None else xt.data_ptr(),
                                    0 if yt is None else yt.data_ptr(),
                                    0 if lt is None else lt.data_ptr(),
                                    None if net is None else
                                    (0 if isinstance(net, bool) else nt.data_ptr()))
        self.config = make_config(**config)
        self.nbytes = mgfwa_workspace_bytes(self.config, self.problem)
        if self.nbytes == 0:
            raise MgfwaError(EINVAL, mgfwa_last_error())
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        # the library runs on a stream of its own (never the null stream); the
        # uploads above, queued on torch's current stream, complete first
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self.ctx = mgfwa_init(self.config, self.problem, self.ws.data_ptr(), self.nbytes,
                              self.stream.cuda_stream)
        self.info = mgfwa_state(self.ctx)
        self.D = self.info.D
        self.Dp = self.info.Dp
        self.B = self.config.n_populations
        self.BN = self.B * self.config.n_fireworks
        # whether mgfwa_step writes the explosion sparks to SE
        self.sparks_materialised = bool(self.info.se_written)

    @classmethod
    def from_workload(cls, wl, **config):
        kw = dict(n_fireworks=wl.n_fireworks, n_sparks=wl.n_sparks, n_guiding=wl.n_guiding,
                  lb=wl.lb, ub=wl.ub, max_generations=wl.generations)
        kw.update(config)
        if getattr(wl, "net", None) is not None:
            if kw.get("external_fitness"):
                return cls(wl.widths, wl.acts, net=True, **kw)
            return cls(wl.widths, wl.acts, net=wl.net, **kw)
        return cls(wl.widths, wl.acts, wl.loss, wl.x, wl.y, wl.labels, **kw)

    def close(self):
        if getattr(self, "ctx", None):
            mgfwa_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the loop
    def step(self, n: int = 1):
        mgfwa_step(self.ctx, n)

    def best(self):
        return mgfwa_best(self.ctx, self.D)

    def best_all(self):
        return mgfwa_best_all(self.ctx, self.B, self.D)

    # torch's current stream and the library's stream are ordered explicitly
    # around every call that hands device data from one to the other
    def _lib_after_torch(self, *tensors):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        for t in tensors:
            t.record_stream(self.stream)

    def _torch_after_lib(self):
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def ask(self):
        """Device view [rows, Dp] of the sparks to evaluate (valid until the next tell)."""
        ptr, rows, ld = mgfwa_ask(self.ctx)
        self._torch_after_lib()
        off = ptr - self.ws.data_ptr()
        return self._view(off, (rows, ld), self.torch.float32)

    def tell(self, fitness):
        f = fitness.to(device=self.device, dtype=self.torch.float32).contiguous()
        self._lib_after_torch(f)
        mgfwa_tell(self.ctx, f.data_ptr())

    def evaluate(self, W):
        """Fitness of the rows of W (torch [rows, ld] float32 on the device)."""
        W = W.contiguous()
        out = self.torch.empty(W.shape[0], dtype=self.torch.float32, device=self.device)
        self._lib_after_torch(W, out)
        mgfwa_evaluate(self.ctx, W.data_ptr(), W.shape[0], W.shape[1], out.data_ptr())
        self._torch_after_lib()
        return out

    def autotune(self, reps: int = 3):
        mgfwa_autotune(self.ctx, reps)

    def fit_plan(self, which: int = 0) -> dict:
        return mgfwa_fit_plan(self.ctx, which)

    def fit_candidates(self, which: int = 0) -> list:
        return mgfwa_fit_candidates(self.ctx, which)

    def set_fit_plan(self, which: int, index: int):
        mgfwa_set_fit_plan(self.ctx, which, index)

    def set_timing(self, on: bool):
        mgfwa_set_timing(self.ctx, on)

    def timing(self):
        return mgfwa_timing(self.ctx)

    # -- state inspection (views into the workspace)
    def _view(self, off, shape, dtype):
        n = int(np.prod(shape)) * self.torch.tensor([], dtype=dtype).element_size()
        return self.ws[off:off + n].view(dtype).view(*shape)

    def state(self) -> dict:
        i = mgfwa_state(self.ctx)
        c = self.config
        BN, Dp, lam, G, k, Cn = self.BN, i.Dp, c.n_sparks, c.n_guiding, i.k, i.n_candidates
        f32, i32 = self.torch.float32, self.torch.int32
        shapes = dict(F=((BN, Dp), f32), A=((BN,), f32), Y=((BN,), f32), Yprev=((BN,), f32),
                      fresh=((BN,), i32), SE=((BN * lam, Dp), f32), SG=((BN * G, Dp), f32),
                      Yc=((BN, Cn), f32), top=((BN * G, k), i32), bottom=((BN * G, k), i32),
                      tie=((BN * G,), i32), cstar=((BN,), i32), improved=((BN,), i32),
                      reinit=((BN,), i32), best_x=((self.B, Dp), f32), best_y=((self.B,), f32),
                      best_f=((self.B,), i32), best_gen=((self.B,), i32), gen=((1,), i32),
                      done=((1,), i32))
        self._torch_after_lib()
        out = {name: self._view(getattr(i, name), shp, dt) for name, (shp, dt) in shapes.items()}
        out["D"], out["Dp"], out["m"], out["k"] = i.D, i.Dp, i.m, i.k
        return out

    def state_numpy(self) -> dict:
        """Host copies of the state (synchronises)."""
        self.stream.synchronize()
        return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in self.state().items()}


class Batch:
    """Jobs (MGFWA objects) advanced together: one HIP graph launch per generation."""

    def __init__(self, jobs, stream=None):
        import torch
        self.jobs = list(jobs)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.h = mgfwa_batch_create([j.ctx for j in self.jobs], self.stream.cuda_stream)

    def step(self, n: int = 1):
        mgfwa_batch_step(self.h, n)

    def close(self):
        if getattr(self, "h", None):
            mgfwa_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over one device arena (a torch uint8 tensor)."""

    def __init__(self, arena_bytes: int, n_streams: int = 4, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        self.h = mgfwa_server_create(self.arena.data_ptr(), int(arena_bytes), int(n_streams))
        self._keep = {}
        self._dims = {}

    def submit(self, widths, acts, loss=None, x=None, y=None, labels=None, sync=True, net=None,
               **config) -> int:
        """Queue one job; the problem's device copies live until the server is closed.
        net= makes it an input problem (the spark is the fixed network's input).
        sync=False skips the device synchronisation that makes freshly uploaded inputs
        visible to the job's stream (pass it for inputs already complete on the device)."""
        torch = self.torch

        def dev(a, dtype):
            if a is None:
                return None
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            return t.to(device=self.device, dtype=dtype).contiguous()

        xt = dev(x, torch.float32)
        yt = dev(y, torch.float32) if loss == "mse" else None
        lt = dev(labels, torch.int32) if loss == "ce" else None
        nt = dev(net, torch.float32)
        prob = make_problem(widths, acts, loss, 0 if xt is None else xt.shape[0],
                            0 if xt is None else xt.data_ptr(),
                            0 if yt is None else yt.data_ptr(),
                            0 if lt is None else lt.data_ptr(),
                            None if nt is None else nt.data_ptr())
        if sync:
            torch.cuda.synchronize(self.device)   # the copies above are complete before admission
        jid = mgfwa_server_submit(self.h, make_config(**config), prob)
        self._keep[jid] = (xt, yt, lt, nt)
        self._dims[jid] = (int(widths[0]) if nt is not None else
                           sum((widths[i] + 1) * widths[i + 1] for i in range(len(widths) - 1)))
        return jid

    def submit_workload(self, wl, sync=True, **config) -> int:
        kw = dict(n_fireworks=wl.n_fireworks, n_sparks=wl.n_sparks, n_guiding=wl.n_guiding,
                  lb=wl.lb, ub=wl.ub, max_generations=wl.generations)
        kw.update(config)
        if getattr(wl, "net", None) is not None:
            return self.submit(wl.widths, wl.acts, sync=sync, net=wl.net, **kw)
        return self.submit(wl.widths, wl.acts, wl.loss, wl.x, wl.y, wl.labels, sync=sync, **kw)

    def tick(self):
        mgfwa_server_tick(self.h)

    def drain(self):
        mgfwa_server_drain(self.h)

    def job(self, jid: int):
        return mgfwa_server_job(self.h, jid, self._dims[jid])

    def stats(self) -> dict:
        return mgfwa_server_stats_get(self.h)

    def close(self):
        if getattr(self, "h", None):
            mgfwa_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
