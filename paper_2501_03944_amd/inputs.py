"""Seeded synthetic workloads for MGFWA weight optimisation of small MLPs.

This module only synthesises inputs: sample matrices, class labels or regression
targets, and the seeded teacher network that produces the regression targets.
It evaluates no fitness and performs no MGFWA step, so the oracle-side tests and
the GPU path can both draw their inputs from it without sharing any of the
method's arithmetic.

The paper (Sec. 4.1, eq. (1); Table 2) optimises a fixed random MLP over its
input; the workloads here instead optimise an MLP's weights on a fixed synthetic
data set, where every spark is the full weight vector.  Three shapes are
provided, each at full size and at any smaller size a test wants:

* ``teacher_regression``  8-16-1 tanh MLP, MSE, x ~ N(0, I_8), targets from a
  seeded teacher of the same shape plus Gaussian noise of variance 0.01.
* ``gaussian_mixture``    64-128-128-10 ReLU MLP, cross-entropy, 10 classes with
  means ~ N(0, 4 I_64), unit covariance, balanced labels.
* ``sparse_prototypes``   784-256-10 ReLU MLP, cross-entropy, inputs in
  [0, 1]^784 built from 10 seeded class prototypes with 20 % support plus noise.
* ``mixed_jobs``          many Gaussian-mixture jobs of uneven depth, width, sample
  count and spark count, for batched generations and serving.
* ``testbed_net``         the paper's own testbed (Sec. 4.1, eq. (1), Table 2): a
  fixed MLP d -> h -> (k hidden h -> h layers) -> 1 whose parameters are drawn
  once, per layer from U(-1/sqrt(fan_in), +1/sqrt(fan_in)) (the paper says only
  that they are random and fixed); the spark is the network's input.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

ACTS = ("identity", "relu", "tanh", "gelu")
LOSSES = ("mse", "ce")


@dataclasses.dataclass
class Workload:
    """One optimisation problem plus the MGFWA shape it is run with."""

    name: str
    widths: tuple            # widths[0] = input dim ... widths[-1] = output dim
    acts: tuple              # activation of every hidden layer (output layer is identity)
    loss: str                # "mse" or "ce"
    x: np.ndarray            # float32 [S, widths[0]], C-contiguous
    y: Optional[np.ndarray]  # float32 [S, widths[-1]] for MSE, else None
    labels: Optional[np.ndarray]  # int32 [S] for CE, else None
    # MGFWA shape (fireworks, sparks per firework, generations, bounds)
    n_fireworks: int = 4
    n_sparks: int = 32
    n_guiding: int = 4
    generations: int = 100
    lb: float = -5.0
    ub: float = 5.0
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n_samples(self) -> int:
        return int(self.x.shape[0])

    @property
    def dim(self) -> int:
        """Number of weights + biases, D = sum_l (in_l * out_l + out_l)."""
        w = self.widths
        return int(sum(w[i] * w[i + 1] + w[i + 1] for i in range(len(w) - 1)))

    def flops_per_eval(self) -> int:
        """Algorithmic matmul work of one spark evaluation: 2 S sum_l in_l out_l."""
        w = self.widths
        return int(2 * self.n_samples * sum(w[i] * w[i + 1] for i in range(len(w) - 1)))


def _uniform_layer(rng: np.random.Generator, fan_in: int, fan_out: int):
    bound = 1.0 / np.sqrt(fan_in)
    W = rng.uniform(-bound, bound, size=(fan_out, fan_in))
    b = rng.uniform(-bound, bound, size=(fan_out,))
    return W, b


def teacher_weights(widths: Sequence[int], seed: int) -> np.ndarray:
    """Seeded teacher weight vector in the nn.Linear layout (W_l row-major, then b_l).

    Each layer is drawn from U(-1/sqrt(fan_in), +1/sqrt(fan_in)); returned as float32.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(widths) - 1):
        W, b = _uniform_layer(rng, widths[i], widths[i + 1])
        parts.append(W.reshape(-1))
        parts.append(b)
    return np.concatenate(parts).astype(np.float32)


def _teacher_outputs(widths, acts, wvec: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Targets of the synthetic regression set (float64 forward of the teacher)."""
    h = x.astype(np.float64)
    off = 0
    w = wvec.astype(np.float64)
    L = len(widths) - 1
    for i in range(L):
        fi, fo = widths[i], widths[i + 1]
        W = w[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = w[off:off + fo]
        off += fo
        h = h @ W.T + b
        if i < L - 1:
            a = acts[i]
            if a == "tanh":
                h = np.tanh(h)
            elif a == "relu":
                h = np.maximum(h, 0.0)
            elif a == "identity":
                pass
            else:
                raise ValueError(f"teacher activation {a!r} not supported")
    return h


def teacher_regression(n_samples: int = 256, widths=(8, 16, 1), act: str = "tanh",
                       noise_var: float = 0.01, seed: int = 1001, **shape) -> Workload:
    """x ~ N(0, I), y = teacher(x) + N(0, noise_var); MSE objective."""
    widths = tuple(int(v) for v in widths)
    acts = tuple([act] * (len(widths) - 2))
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n_samples, widths[0]))
    wt = teacher_weights(widths, seed + 7)
    clean = _teacher_outputs(widths, acts, wt, x.astype(np.float32))
    noise = rng.standard_normal(clean.shape) * np.sqrt(noise_var)
    y = (clean + noise).astype(np.float32)
    wl = Workload(name="teacher_regression", widths=widths, acts=acts, loss="mse",
                  x=np.ascontiguousarray(x.astype(np.float32)), y=np.ascontiguousarray(y),
                  labels=None, extra={"teacher": wt, "noise": noise.astype(np.float64),
                                      "clean": clean})
    _apply_shape(wl, shape, defaults=dict(n_fireworks=4, n_sparks=32, generations=100))
    return wl


def _balanced_labels(rng: np.random.Generator, n: int, classes: int) -> np.ndarray:
    lab = np.arange(n) % classes
    rng.shuffle(lab)
    return lab.astype(np.int32)


def gaussian_mixture(n_samples: int = 4096, widths=(64, 128, 128, 10), act: str = "relu",
                     mean_var: float = 4.0, seed: int = 1002, **shape) -> Workload:
    """Balanced 10-class mixture in R^dim: means ~ N(0, mean_var I), x = mu_c + N(0, I)."""
    widths = tuple(int(v) for v in widths)
    dim, classes = widths[0], widths[-1]
    rng = np.random.default_rng(seed)
    means = rng.standard_normal((classes, dim)) * np.sqrt(mean_var)
    labels = _balanced_labels(rng, n_samples, classes)
    x = means[labels] + rng.standard_normal((n_samples, dim))
    wl = Workload(name="gaussian_mixture", widths=widths, acts=tuple([act] * (len(widths) - 2)),
                  loss="ce", x=np.ascontiguousarray(x.astype(np.float32)), y=None,
                  labels=labels, extra={"means": means})
    _apply_shape(wl, shape, defaults=dict(n_fireworks=8, n_sparks=256, generations=500))
    return wl


def sparse_prototypes(n_samples: int = 8192, widths=(784, 256, 10), act: str = "relu",
                      density: float = 0.2, noise_std: float = 0.1, seed: int = 1003,
                      **shape) -> Workload:
    """Inputs in [0,1]^dim from 10 prototypes, each with a random support of
    round(density*dim) pixels valued U(0.5, 1); a sample is its class prototype plus
    N(0, noise_std^2) on the support, clipped to [0, 1], and zero off the support."""
    widths = tuple(int(v) for v in widths)
    dim, classes = widths[0], widths[-1]
    rng = np.random.default_rng(seed)
    nsup = int(round(density * dim))
    protos = np.zeros((classes, dim))
    masks = np.zeros((classes, dim), dtype=bool)
    for c in range(classes):
        sup = rng.choice(dim, size=nsup, replace=False)
        masks[c, sup] = True
        protos[c, sup] = rng.uniform(0.5, 1.0, size=nsup)
    labels = _balanced_labels(rng, n_samples, classes)
    x = protos[labels] + rng.standard_normal((n_samples, dim)) * noise_std
    x = np.clip(x, 0.0, 1.0) * masks[labels]
    wl = Workload(name="sparse_prototypes", widths=widths, acts=tuple([act] * (len(widths) - 2)),
                  loss="ce", x=np.ascontiguousarray(x.astype(np.float32)), y=None,
                  labels=labels, extra={"prototypes": protos})
    _apply_shape(wl, shape, defaults=dict(n_fireworks=16, n_sparks=256, generations=300))
    return wl


def random_mlp_problem(widths, acts, loss: str, n_samples: int, seed: int,
                       x_scale: float = 1.0) -> Workload:
    """Arbitrary-shape problem for tests: x ~ x_scale*N(0,1); MSE targets ~ N(0,1)
    or uniformly random labels for CE."""
    widths = tuple(int(v) for v in widths)
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((n_samples, widths[0])) * x_scale).astype(np.float32)
    y = labels = None
    if loss == "mse":
        y = rng.standard_normal((n_samples, widths[-1])).astype(np.float32)
    else:
        labels = rng.integers(0, widths[-1], size=n_samples).astype(np.int32)
    return Workload(name="random_mlp", widths=widths, acts=tuple(acts), loss=loss,
                    x=np.ascontiguousarray(x), y=y, labels=labels)


def random_weights(dim: int, rows: int, seed: int, lo: float = -5.0, hi: float = 5.0) -> np.ndarray:
    """Uniform random weight vectors (float32 [rows, dim]) for fitness-only tests."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(rows, dim)).astype(np.float32)


def mixed_jobs(n_jobs: int = 64, seed: int = 1004, d_range=(1000, 50000), width_range=(32, 256),
               sample_range=(1024, 4096), sparks=(16, 32, 64, 128), n_fireworks: int = 4,
               inputs=(16, 32, 64), classes: int = 10, generations: int = 300) -> list:
    """Independent jobs of uneven shape for batched generations: per job a target
    D log-uniform in d_range, 2 or 3 weight layers, input width from `inputs`, one
    hidden width (clamped to width_range) that brings D nearest the target, 10-class
    Gaussian-mixture data with a sample count uniform in sample_range, and
    n_fireworks x lambda sparks with lambda from `sparks` (4 guiding sparks)."""
    rng = np.random.default_rng(seed)
    jobs = []
    lo_w, hi_w = width_range
    for j in range(n_jobs):
        target = float(np.exp(rng.uniform(np.log(d_range[0]), np.log(d_range[1]))))
        layers = int(rng.integers(2, 4))
        fin = int(rng.choice(inputs))
        if layers == 2:    # D = fin*h + h + h*C + C
            h = (target - classes) / (fin + 1 + classes)
        else:              # D = fin*h + h + h*h + h + h*C + C
            b = fin + 2 + classes
            h = (-b + np.sqrt(b * b + 4.0 * (target - classes))) / 2.0
        h = int(min(max(round(h), lo_w), hi_w))
        widths = (fin,) + (h,) * (layers - 1) + (classes,)
        n_samples = int(rng.integers(sample_range[0], sample_range[1] + 1))
        lam = int(rng.choice(sparks))
        wl = gaussian_mixture(n_samples=n_samples, widths=widths, seed=10_000 + j,
                              n_fireworks=n_fireworks, n_sparks=lam, n_guiding=4,
                              generations=generations)
        wl.name = f"job{j}"
        wl.extra["target_dim"] = target
        jobs.append(wl)
    return jobs


def _apply_shape(wl: Workload, shape: dict, defaults: dict) -> None:
    for k, v in defaults.items():
        setattr(wl, k, v)
    for k, v in shape.items():
        if not hasattr(wl, k):
            raise TypeError(f"unknown workload field {k!r}")
        setattr(wl, k, v)


# The three full-size workloads, by name (data seed = 1000 + index).
def workload(name: str, **overrides) -> Workload:
    if name in ("mlp8-16-1", "teacher"):
        return teacher_regression(**overrides)
    if name in ("mlp64-128-128-10", "gmm"):
        return gaussian_mixture(**overrides)
    if name in ("mlp784-256-10", "prototypes"):
        return sparse_prototypes(**overrides)
    if name.startswith("net") and name[3:].isdigit() and int(name[3:]) in TESTBED_NETS:
        return testbed_net(int(name[3:]), **overrides)
    raise KeyError(name)


WORKLOAD_NAMES = ("mlp8-16-1", "mlp64-128-128-10", "mlp784-256-10")


# The paper's testbed networks (Table 2): id -> (scale, activation, input dim d,
# hidden width h, "Layer num" k).  The network is Linear(d, h), k hidden
# Linear(h, h) layers, and Linear(h, 1), with the activation after every layer
# but the last, so it has d*h + h + k*(h*h + h) + h + 1 parameters.
TESTBED_NETS = {
    1: ("small", "relu", 10, 16, 4),
    2: ("small", "gelu", 10, 32, 4),
    3: ("small", "relu", 20, 16, 4),
    4: ("small", "gelu", 20, 32, 4),
    5: ("medium", "relu", 100, 64, 7),
    6: ("medium", "gelu", 100, 128, 7),
    7: ("medium", "relu", 200, 64, 7),
    8: ("medium", "gelu", 200, 128, 7),
    9: ("large", "relu", 1000, 256, 10),
    10: ("large", "gelu", 1000, 512, 10),
    11: ("large", "relu", 2000, 256, 10),
    12: ("large", "gelu", 2000, 512, 10),
}


@dataclasses.dataclass
class NetInputWorkload:
    """Input optimisation of a fixed MLP (the spark is the input, the fitness
    the network's scalar output) plus the MGFWA shape it is run with."""

    name: str
    widths: tuple            # (d, h, ..., h, 1)
    acts: tuple              # activation after every layer but the last
    net: np.ndarray          # float32 parameters, nn.Linear layout (W_l row-major, then b_l)
    n_fireworks: int = 8
    n_sparks: int = 512
    n_guiding: int = 8
    generations: int = 100
    lb: float = -5.0
    ub: float = 5.0
    extra: dict = dataclasses.field(default_factory=dict)
    loss = None
    x = y = labels = None

    @property
    def dim(self) -> int:
        """Spark dimension: the input width d."""
        return int(self.widths[0])

    @property
    def n_params(self) -> int:
        w = self.widths
        return int(sum(w[i] * w[i + 1] + w[i + 1] for i in range(len(w) - 1)))

    def flops_per_eval(self) -> int:
        """Algorithmic matmul work of one spark evaluation: 2 sum_l in_l out_l."""
        w = self.widths
        return int(2 * sum(w[i] * w[i + 1] for i in range(len(w) - 1)))


def net_input_problem(widths, acts, seed: int, **shape) -> NetInputWorkload:
    """A fixed MLP of any shape (widths[-1] must be 1) with seeded parameters."""
    widths = tuple(int(v) for v in widths)
    if widths[-1] != 1:
        raise ValueError("the fixed network has one output")
    wl = NetInputWorkload(name="net_input", widths=widths, acts=tuple(acts),
                          net=teacher_weights(widths, seed))
    _apply_shape(wl, shape, {})
    return wl


def testbed_net(net_id: int, seed: Optional[int] = None, **shape) -> NetInputWorkload:
    """Table 2 network `net_id` with parameters drawn from seed (default
    3000 + net_id)."""
    scale, act, d, h, k = TESTBED_NETS[int(net_id)]
    widths = (d,) + (h,) * (k + 1) + (1,)
    wl = net_input_problem(widths, (act,) * (k + 1),
                           seed=3000 + int(net_id) if seed is None else seed, **shape)
    wl.name = f"net{int(net_id)}"
    wl.extra.update(scale=scale, layer_num=k)
    return wl
