"""Pins of the oracle's input-optimisation fitness, the paper's testbed
(Sec. 4.1, eq. (1), Table 2): the spark is the input x of a fixed MLP and the
fitness is the network's scalar output f(x).  No GPU.

* Table 2: the networks' shapes give the printed parameter counts (nets 2-9;
  the others are misprints, checked as such).
* Closed forms: hand-built ReLU and GELU networks whose output is written out
  (GELU(x) = x Phi(x), with Phi(+-1) from the normal table); an all-identity
  network equals one affine map, the product of its layers.
* Invariants: a ReLU network without biases is positively homogeneous.
* Brute force: a float64 matrix-product chain on a Table 2 network.
* A whole run on a testbed network keeps Alg. 1's invariants and lowers f.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2501_03944_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table2_nets.json")))


def _net(widths, acts, params):
    return O.Problem(widths, acts, net=np.asarray(params, dtype=np.float32))


def test_table2_parameter_counts():
    for row in GOLD["nets"]:
        wl = inputs.testbed_net(row["id"])
        scale, act, d, h, k = inputs.TESTBED_NETS[row["id"]]
        assert (scale, act, d, h, k) == (row["scale"], row["act"], row["d"], row["h"], row["k"])
        p = O.Problem.from_workload(wl)
        assert p.dim == row["d"]                    # the spark is the input
        assert p.n_params == wl.n_params == wl.net.size
        assert (p.n_params == row["params"]) == row["consistent"], row
    assert sum(r["consistent"] for r in GOLD["nets"]) == 8


def test_relu_closed_form():
    # f(x) = 2 relu(x0) - 3 relu(0.5 - x1) + 0.25
    W1 = [[1.0, 0.0, 0.0], [0.0, -1.0, 0.0]]
    b1 = [0.0, 0.5]
    W2 = [[2.0, -3.0]]
    b2 = [0.25]
    p = _net((3, 2, 1), ("relu",), np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2]))
    for x, want in (([1.0, 0.0, 9.0], 2.0 - 1.5 + 0.25), ([-1.0, 2.0, 0.0], 0.25),
                    ([0.5, -0.5, 1.0], 1.0 - 3.0 + 0.25), ([0.0, 0.5, 0.0], 0.25)):
        assert p.output(np.array(x, np.float32)) == want
    X = np.array([[1.0, 0.0, 9.0], [-1.0, 2.0, 0.0]], np.float32)
    np.testing.assert_array_equal(p.loss_rows(X), [0.75, 0.25])


def test_gelu_closed_form():
    # one GELU unit: f(x) = GELU(x0 - 1) + GELU(x1); GELU(1) = Phi(1), GELU(-1) = -Phi(-1)
    phi1, phim1 = 0.8413447460685429, 0.15865525393145707   # standard normal table
    p = _net((2, 2, 1), ("gelu",), [1.0, 0.0, 0.0, 1.0, -1.0, 0.0, 1.0, 1.0, 0.0])
    assert p.output(np.array([2.0, 0.0], np.float32)) == pytest.approx(phi1, abs=1e-15)
    assert p.output(np.array([0.0, -1.0], np.float32)) == pytest.approx(-2.0 * phim1, abs=1e-15)
    assert p.output(np.array([1.0, 1.0], np.float32)) == pytest.approx(phi1, abs=1e-15)


def test_identity_network_is_one_affine_map():
    rng = np.random.default_rng(3)
    widths = (7, 5, 6, 1)
    wl = inputs.net_input_problem(widths, ("identity", "identity"), seed=9)
    p = O.Problem.from_workload(wl)
    # collapse the layers into one affine map y = M x + c
    M, c, off = np.eye(7), np.zeros(7), 0
    for fi, fo in zip(widths[:-1], widths[1:]):
        W = wl.net[off:off + fi * fo].astype(np.float64).reshape(fo, fi)
        b = wl.net[off + fi * fo:off + fi * fo + fo].astype(np.float64)
        M, c = W @ M, W @ c + b
        off += fi * fo + fo
    X = rng.uniform(-5, 5, (40, 7)).astype(np.float32)
    np.testing.assert_allclose(p.loss_rows(X), (X.astype(np.float64) @ M.T + c)[:, 0],
                               rtol=1e-13, atol=1e-13)


def test_relu_without_bias_is_positively_homogeneous():
    wl = inputs.net_input_problem((12, 20, 20, 1), ("relu", "relu"), seed=4)
    net = wl.net.copy()
    off = 0
    for fi, fo in zip(wl.widths[:-1], wl.widths[1:]):
        net[off + fi * fo:off + fi * fo + fo] = 0.0
        off += fi * fo + fo
    p = _net(wl.widths, wl.acts, net)
    x = np.random.default_rng(1).uniform(-1, 1, 12).astype(np.float32)
    f = p.output(x)
    assert f != 0.0
    for a in (2.0, 4.0, 0.5, 0.25):             # powers of two: x*a is exact in binary32
        assert p.output(x * np.float32(a)) == pytest.approx(a * f, rel=1e-14)


@pytest.mark.parametrize("net_id", [3, 6, 9])
def test_matches_float64_matrix_chain(net_id):
    wl = inputs.testbed_net(net_id)
    p = O.Problem.from_workload(wl)
    X = np.random.default_rng(net_id).uniform(-5, 5, (16, wl.dim)).astype(np.float32)
    H, off = X.astype(np.float64), 0
    L = len(wl.widths) - 1
    for l, (fi, fo) in enumerate(zip(wl.widths[:-1], wl.widths[1:])):
        W = wl.net[off:off + fi * fo].astype(np.float64).reshape(fo, fi)
        b = wl.net[off + fi * fo:off + fi * fo + fo].astype(np.float64)
        Z = H @ W.T + b
        if l < L - 1:
            if wl.acts[l] == "relu":
                Z = np.maximum(Z, 0.0)
            else:
                from scipy.special import erf
                Z = 0.5 * Z * (1.0 + erf(Z / np.sqrt(2.0)))
        H = Z
        off += fi * fo + fo
    np.testing.assert_allclose(p.loss_rows(X), H[:, 0], rtol=1e-12, atol=1e-12)


def test_input_problem_rejects_bad_shapes():
    with pytest.raises(ValueError):
        inputs.net_input_problem((4, 3, 2), ("relu",), seed=1)
    with pytest.raises(ValueError):
        O.Problem((4, 3, 1), ("relu",), net=np.zeros(5, np.float32))


def test_testbed_run_keeps_invariants_and_descends():
    wl = inputs.testbed_net(4)
    p = O.Problem.from_workload(wl)
    o = O.Oracle(p, N=4, lam=32, G=4, T=40, seed=2)
    o.init()
    best = [float(o.view()["best_y"][0])]
    for _ in range(40):
        o.generation()
        v = o.view()
        assert v["SE"].min() >= -5.0 and v["SE"].max() <= 5.0
        assert v["best_y"][0] <= best[-1]
        best.append(float(v["best_y"][0]))
        assert float(v["best_y"][0]) == float(v["Y"].min())
        # the stored fitness is the network's output at the firework (a firework
        # that loser-out just re-initialised holds +inf until it is evaluated)
        kept = v["reinit"] == 0
        assert np.all(np.isinf(v["Y"][~kept]))
        np.testing.assert_array_equal(v["Y"][kept], p.loss_rows(v["F"][kept]).astype(np.float32))
    assert best[-1] < best[0]
