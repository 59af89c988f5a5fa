"""Pins of the oracle's binary64 fitness (no GPU).

Fitness = loss of the MLP whose weights are the spark, over the shared samples
(the black-box objective of Alg. 1 with the weights as the decision variable).
Checked against closed forms and against torch's float64 CPU library routines
(F.linear, activations, F.mse_loss, F.cross_entropy) on random tiny networks.
"""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

from oracle.oracle import Problem
from paper_2501_03944_amd import inputs


def _torch_loss(wl, w):
    """Library reference: unpack w in nn.Linear order and run torch float64 ops."""
    h = torch.from_numpy(wl.x.astype(np.float64))
    wt = torch.from_numpy(w.astype(np.float64))
    off = 0
    L = len(wl.widths) - 1
    for i in range(L):
        fi, fo = wl.widths[i], wl.widths[i + 1]
        W = wt[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = wt[off:off + fo]
        off += fo
        h = Fn.linear(h, W, b)
        if i < L - 1:
            a = wl.acts[i]
            h = {"relu": torch.relu, "tanh": torch.tanh, "identity": lambda z: z,
                 "gelu": lambda z: Fn.gelu(z, approximate="none")}[a](h)
    if wl.loss == "mse":
        return float(Fn.mse_loss(h, torch.from_numpy(wl.y.astype(np.float64))))
    return float(Fn.cross_entropy(h, torch.from_numpy(wl.labels.astype(np.int64))))


@pytest.mark.parametrize("widths,acts,loss", [
    ((8, 16, 1), ("tanh",), "mse"),
    ((5, 7, 3), ("relu",), "mse"),
    ((6, 9, 4), ("relu",), "ce"),
    ((3, 4, 5, 2), ("gelu", "tanh"), "ce"),
    ((4, 3), (), "mse"),
    ((7, 6, 6, 6, 10), ("relu", "identity", "tanh"), "ce"),
])
def test_loss_matches_torch_float64(widths, acts, loss):
    wl = inputs.random_mlp_problem(widths, acts, loss, n_samples=37, seed=sum(widths))
    p = Problem.from_workload(wl)
    W = inputs.random_weights(wl.dim, 6, seed=3, lo=-2.0, hi=2.0)
    got = p.loss_rows(W)
    for r in range(W.shape[0]):
        ref = _torch_loss(wl, W[r])
        assert got[r] == pytest.approx(ref, rel=1e-12, abs=1e-300)


def test_zero_weights_closed_forms():
    wl = inputs.random_mlp_problem((5, 8, 3), ("relu",), "mse", n_samples=50, seed=1)
    p = Problem.from_workload(wl)
    zero = np.zeros(wl.dim, dtype=np.float32)
    y = wl.y.astype(np.float64)
    assert p.loss_of(zero) == pytest.approx(float(np.mean(y * y)), rel=1e-14)
    wl = inputs.random_mlp_problem((5, 8, 10), ("relu",), "ce", n_samples=50, seed=2)
    p = Problem.from_workload(wl)
    assert p.loss_of(np.zeros(wl.dim, dtype=np.float32)) == pytest.approx(math.log(10), rel=1e-14)


def test_output_bias_only_closed_form():
    wl = inputs.random_mlp_problem((4, 6, 2), ("tanh",), "mse", n_samples=64, seed=4)
    p = Problem.from_workload(wl)
    w = np.zeros(wl.dim, dtype=np.float32)
    b = np.array([0.75, -1.5], dtype=np.float32)
    w[-2:] = b
    y = wl.y.astype(np.float64)
    want = float(np.mean((y - b.astype(np.float64)) ** 2))
    assert p.loss_of(w) == pytest.approx(want, rel=1e-14)


def test_teacher_weights_give_noise_variance():
    wl = inputs.teacher_regression()
    p = Problem.from_workload(wl)
    want = float(np.mean(wl.extra["noise"] ** 2))
    # targets are stored in binary32, so agreement is to binary32 rounding of y
    assert p.loss_of(wl.extra["teacher"]) == pytest.approx(want, rel=1e-6)


def test_ce_shift_invariance_and_per_sample():
    wl = inputs.random_mlp_problem((3, 5, 4), ("relu",), "ce", n_samples=20, seed=9)
    p = Problem.from_workload(wl)
    w = inputs.random_weights(wl.dim, 1, seed=10, lo=-1, hi=1)[0]
    w[-4:] = np.round(w[-4:] * 1024.0) / 1024.0   # biases on a coarse grid so the
    w2 = w.copy()                                 # shift below is exact in binary32
    w2[-4:] += np.float32(4.0)    # same constant on every output bias
    v1, ps1 = p.loss_of(w, per_sample=True)
    v2, ps2 = p.loss_of(w2, per_sample=True)
    assert v1 == pytest.approx(v2, rel=1e-12)
    assert v1 == pytest.approx(float(ps1.mean()), rel=1e-14)
    assert np.all(ps1 >= 0.0)


def test_ce_large_logits_stable():
    # a single-layer net with huge weights: logits ~1e4, result must stay finite and >= 0
    wl = inputs.random_mlp_problem((4, 3), (), "ce", n_samples=16, seed=11, x_scale=100.0)
    p = Problem.from_workload(wl)
    w = inputs.random_weights(wl.dim, 1, seed=12, lo=-50, hi=50)[0]
    v = p.loss_of(w)
    assert math.isfinite(v) and v >= 0.0
    assert v == pytest.approx(_torch_loss(wl, w), rel=1e-12)


def test_forward_matches_library():
    wl = inputs.random_mlp_problem((6, 5, 4, 3), ("tanh", "relu"), "mse", n_samples=8, seed=21)
    p = Problem.from_workload(wl)
    w = inputs.random_weights(wl.dim, 1, seed=22, lo=-1, hi=1)[0]
    lin = []
    off = 0
    for i in range(3):
        fi, fo = wl.widths[i], wl.widths[i + 1]
        lin.append((torch.from_numpy(w[off:off + fi * fo].reshape(fo, fi).astype(np.float64)),
                    torch.from_numpy(w[off + fi * fo:off + fi * fo + fo].astype(np.float64))))
        off += fi * fo + fo
    for s in range(8):
        h = torch.from_numpy(wl.x[s].astype(np.float64))
        h = torch.tanh(Fn.linear(h, *lin[0]))
        h = torch.relu(Fn.linear(h, *lin[1]))
        h = Fn.linear(h, *lin[2])
        np.testing.assert_allclose(p.forward(w, s), h.numpy(), rtol=1e-13)
