"""The paper's testbed on the HIP path (Sec. 4.1, eq. (1), Table 2; needs an
MI355X): the spark is the input of a fixed MLP and its fitness the network's
output, computed by the fused MFMA kernel that carries a tile of sparks through
every layer.

Fitness tolerance (FP32 products, FP32 accumulation, against the binary64
oracle), a first-order error bound.  A K-term FP32 dot product returns the exact
dot product of slightly perturbed operands, every weight off by a relative
gamma_K = K u at most (u = 2^-24), and an FP32 activation is off by a few units
in the last place of its value.  To first order the output then moves by at most
    B(x) = sum_l [ K_l u |g_l|^T (|W_l| |h_{l-1}| + |b_l|) + 4 u |d_l|^T |h_l| ]
where h_l are the exact activations, g_l = df/dz_l and d_l = df/dh_l (binary64
back-propagation).  The test allows 2 B(x) + 1e-6 |f(x)|.  State: bit-exact
with the oracle, as for weight problems, until a near-tie.
"""
import numpy as np
import pytest

from gpu_util import assert_bits, make_pair, near_tie_present, require_gpu
from oracle import oracle as O
from paper_2501_03944_amd import inputs
from test_gpu_parity import _lockstep

pytestmark = pytest.mark.gpu


def _layers(wl):
    off, out = 0, []
    for fi, fo in zip(wl.widths[:-1], wl.widths[1:]):
        W = wl.net[off:off + fi * fo].astype(np.float64).reshape(fo, fi)
        b = wl.net[off + fi * fo:off + fi * fo + fo].astype(np.float64)
        out.append((W, b))
        off += fi * fo + fo
    return out


def _error_bound(wl, X):
    """B(x) per row (module docstring): binary64 forward and backward passes."""
    from scipy.special import erf
    u = 2.0 ** -24
    layers = _layers(wl)
    L = len(layers)
    hs, zs = [X.astype(np.float64)], []
    for l, (W, b) in enumerate(layers):
        z = hs[-1] @ W.T + b
        zs.append(z)
        if l < L - 1:
            a = wl.acts[l]
            h = (np.maximum(z, 0.0) if a == "relu" else np.tanh(z) if a == "tanh" else
                 0.5 * z * (1.0 + erf(z / np.sqrt(2.0))) if a == "gelu" else z)
            hs.append(h)
    B = np.zeros(X.shape[0])
    g = np.ones((X.shape[0], 1))                     # df/dz of the output layer
    for l in range(L - 1, -1, -1):
        W, b = layers[l]
        K = (W.shape[1] + 15) // 16 * 16
        B += K * u * np.sum(np.abs(g) * (np.abs(hs[l]) @ np.abs(W).T + np.abs(b)), axis=1)
        if l == 0:
            break
        d = g @ W                                    # df/dh_{l-1}
        B += 4 * u * np.sum(np.abs(d) * np.abs(hs[l]), axis=1)
        z, a = zs[l - 1], wl.acts[l - 1]
        slope = ((z > 0).astype(np.float64) if a == "relu" else 1.0 - np.tanh(z) ** 2 if a == "tanh"
                 else 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi)
                 if a == "gelu" else np.ones_like(z))
        g = d * slope
    return B


def assert_net_close(wl, X, got, want, what):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    bound = 1e-6 * np.abs(want) + 2.0 * _error_bound(wl, X)
    err = np.abs(got - want)
    bad = ~(err <= bound)
    if np.any(bad):
        i = int(np.argwhere(bad)[0, 0])
        raise AssertionError(f"{what}: {int(bad.sum())}/{bad.size} outside the bound; first row {i}: "
                             f"{got[i]} vs {want[i]} (bound {bound[i]:.3e})")
    return float((err / np.maximum(bound, 1e-300)).max())


def _eval(torch, g, X, ld=None):
    rows, d = X.shape
    ld = ld or g.Dp
    Xd = torch.zeros((rows, ld), dtype=torch.float32, device="cuda")
    Xd[:, :d] = torch.from_numpy(X)
    return g.evaluate(Xd).cpu().numpy(), Xd


@pytest.mark.parametrize("net_id", list(range(1, 13)))
def test_fitness_matches_oracle_every_table2_net(net_id):
    torch, M = require_gpu()
    wl = inputs.testbed_net(net_id)
    g = M.MGFWA.from_workload(wl, n_fireworks=2, n_sparks=16, n_guiding=4)
    p = O.Problem.from_workload(wl)
    rng = np.random.default_rng(net_id)
    for rows, lo, hi in ((37, -5.0, 5.0), (100, -0.5, 0.5)):
        X = rng.uniform(lo, hi, (rows, wl.dim)).astype(np.float32)
        got, _ = _eval(torch, g, X)
        r = assert_net_close(wl, X, got, p.loss_rows(X), f"net {net_id} U({lo},{hi})")
        print(f"net {net_id} rows {rows}: worst error / bound = {r:.2e}")
    g.close()


def test_unpadded_rows_ignore_what_follows_the_input():
    """ld = d rounded up to 4 with NaN in the gap: the kernel reads exactly d
    inputs per row, also in the last partial chunk."""
    torch, M = require_gpu()
    for widths, acts in (((10, 32, 32, 1), ("gelu", "gelu")), ((100, 64, 1), ("relu",)),
                         ((3, 16, 1), ("tanh",))):
        wl = inputs.net_input_problem(widths, acts, seed=sum(widths))
        g = M.MGFWA.from_workload(wl, n_fireworks=2, n_sparks=16, n_guiding=4)
        p = O.Problem.from_workload(wl)
        d = widths[0]
        ld = (d + 3) // 4 * 4
        X = np.random.default_rng(d).uniform(-3, 3, (53, d)).astype(np.float32)
        Xd = torch.full((53, ld), float("nan"), dtype=torch.float32, device="cuda")
        Xd[:, :d] = torch.from_numpy(X)
        got = g.evaluate(Xd).cpu().numpy()
        assert np.all(np.isfinite(got))
        assert_net_close(wl, X, got, p.loss_rows(X), f"{widths} ld={ld}")
        g.close()


# (kernel path, rows): whole-network tiles of 16 and 32 rows; layer by layer
# with 64 x 128, 64 x 64, 32 x 32 and K-split 16 x 16 tiles (on 256 compute
# units); layer by layer with LDS-staged 64 x 128 (net 12) and 64 x 64 (net 6) tiles
PATHS = [(1, 37), (1, 9000), (2, 37), (2, 1000), (2, 2100), (2, 4101), (3, 37), (3, 4101)]


@pytest.mark.parametrize("net_id", [6, 12])
@pytest.mark.parametrize("path,rows", PATHS)
def test_every_kernel_path_sampled_against_oracle(net_id, path, rows):
    """Each tile shape of both kernels: sampled rows (the first and the ragged
    last tile included) against the oracle."""
    torch, M = require_gpu()
    wl = inputs.testbed_net(net_id)
    # 16 x 512 explosion sparks: evaluation runs in chunks of 8192 rows
    g = M.MGFWA.from_workload(wl, n_fireworks=16, n_sparks=512, n_guiding=8, fit_path=path)
    p = O.Problem.from_workload(wl)
    X = np.random.default_rng(rows).uniform(-5, 5, (rows, wl.dim)).astype(np.float32)
    got, _ = _eval(torch, g, X)
    idx = np.unique(np.concatenate([np.arange(min(rows, 40)), np.arange(max(0, rows - 45), rows),
                                    np.random.default_rng(6).integers(0, rows, 40)]))
    r = assert_net_close(wl, X[idx], got[idx], p.loss_rows(X[idx]),
                         f"net {net_id} path {path} rows {rows}")
    print(f"net {net_id} path {path} rows {rows}: worst error / bound = {r:.2e}")
    g.close()


def _free_run(wl, gens, **cfg):
    torch, M = require_gpu()
    o, g = make_pair(wl, **cfg)
    D = g.D
    o.init()
    gs, ov = g.state_numpy(), o.view()
    assert_bits(gs["F"][:, :D], ov["F"], "init F")
    lam, G = o.cfg.lam, o.cfg.G
    try:
        for gen in range(1, gens + 1):
            prev = o.view()
            o.generation()
            g.step(1)
            ov, gs = o.view(), g.state_numpy()
            fin = np.isfinite(ov["Yc64"])
            SEG = np.concatenate([ov["SE"], ov["SG"]])
            same = all(np.array_equal(gs[k][:, :D] if k == "F" else gs[k], ov[k])
                       for k in ("F", "A", "cstar", "reinit", "top", "bottom", "tie"))
            # candidate fitness: explosion rows then guiding rows of every firework
            BN = gs["Yc"].shape[0]
            Xc = np.concatenate([SEG[:BN * lam].reshape(BN, lam, D),
                                 SEG[BN * lam:].reshape(BN, G, D)], axis=1).reshape(-1, D)
            assert np.all(fin)
            if not same:
                # two decisions are equally valid when the values compared lie
                # within the fitness bound of each other
                tol = 4.0 * float(_error_bound(wl, Xc).max())
                assert near_tie_present(prev, ov, lam, G, ov["m"], ov["k"], rel=0.0, atol=tol), \
                    f"divergence at generation {gen} without a near-tie"
                return gen
            assert_bits(gs["SE"][:, :D], ov["SE"], f"gen {gen} SE")
            assert_bits(gs["SG"][:, :D], ov["SG"], f"gen {gen} SG")
            assert_net_close(wl, Xc, gs["Yc"].reshape(-1), ov["Yc64"].reshape(-1),
                             f"gen {gen} candidate fitness")
        return None
    finally:
        g.close()


@pytest.mark.parametrize("net_id,cfg", [
    (2, dict(n_fireworks=4, n_sparks=32, n_guiding=4, seed=1, T=40)),
    (5, dict(n_fireworks=3, n_sparks=24, n_guiding=3, seed=2, T=40, lag_guiding=True)),
    (9, dict(n_fireworks=2, n_sparks=16, n_guiding=2, seed=3, T=20, map_range=True)),
])
def test_free_running_testbed_matches_oracle(net_id, cfg):
    wl = inputs.testbed_net(net_id)
    at = _free_run(wl, 20, **cfg)
    print(f"net {net_id}: diverged_at={at}")


def test_lockstep_testbed_state_path():
    wl = inputs.testbed_net(3)
    _lockstep(wl, 10, check_fitness=False, n_fireworks=3, n_sparks=12, n_guiding=3, T=30, seed=4)


def test_full_size_generation_sampled():
    """One generation at the benchmark's size (net 12, 8 fireworks x 512
    sparks): sampled candidate fitness against the oracle."""
    torch, M = require_gpu()
    wl = inputs.testbed_net(12)
    g = M.MGFWA.from_workload(wl)
    p = O.Problem.from_workload(wl)
    g.step(1)
    s = g.state_numpy()
    D, lam = g.D, wl.n_sparks
    rng = np.random.default_rng(7)
    rows = rng.integers(0, s["SE"].shape[0], 24)
    X = s["SE"][rows, :D]
    got = s["Yc"][rows // lam, rows % lam]
    assert_net_close(wl, X, got, p.loss_rows(X), "full-size explosion fitness")
    Xg = s["SG"][:, :D]
    got = s["Yc"][:, lam:].reshape(-1)
    assert_net_close(wl, Xg, got, p.loss_rows(Xg), "full-size guiding fitness")
    g.close()


def test_autotuned_input_problem_matches_oracle():
    """The autotuner picks a tile shape per launch size; the tuned generation
    still agrees with the oracle."""
    torch, M = require_gpu()
    wl = inputs.testbed_net(10)
    g = M.MGFWA.from_workload(wl, n_fireworks=4, n_sparks=256, n_guiding=4, seed=3)
    assert g.fit_plan(0)["net_kernel"] == -1
    g.autotune(2)
    k0, k1 = g.fit_plan(0)["net_kernel"], g.fit_plan(1)["net_kernel"]
    assert 0 <= k0 <= 6 and 0 <= k1 <= 6
    print(f"tuned kernels: explosion {k0}, guiding {k1}")
    p = O.Problem.from_workload(wl)
    o = O.Oracle(p, N=4, lam=256, G=4, lb=wl.lb, ub=wl.ub, T=wl.generations, seed=3)
    o.init()
    o.generation()
    g.step(1)
    s, v = g.state_numpy(), o.view()
    D = g.D
    assert_bits(s["SE"][:, :D], v["SE"], "tuned generation SE")
    idx = np.random.default_rng(1).integers(0, 4 * 256, 40)
    assert_net_close(wl, v["SE"][idx], s["Yc"][idx // 256, idx % 256], v["Yc64"][idx // 256, idx % 256],
                     "tuned explosion fitness")
    assert_net_close(wl, v["SG"], s["Yc"][:, 256:].reshape(-1), v["Yc64"][:, 256:].reshape(-1),
                     "tuned guiding fitness")
    g.close()


@pytest.mark.parametrize("widths", [(7, 1), (300, 1), (5, 3, 1)])
def test_degenerate_networks(widths):
    """A single linear layer (no hidden activations at all) and a tiny hidden
    layer: fitness, and free-running generations with one firework per
    population."""
    torch, M = require_gpu()
    wl = inputs.net_input_problem(widths, ("relu",) * (len(widths) - 2), seed=len(widths) + widths[0])
    g = M.MGFWA.from_workload(wl, n_fireworks=2, n_sparks=16, n_guiding=4)
    p = O.Problem.from_workload(wl)
    X = np.random.default_rng(2).uniform(-5, 5, (45, wl.dim)).astype(np.float32)
    got, _ = _eval(torch, g, X)
    assert_net_close(wl, X, got, p.loss_rows(X), f"{widths}")
    g.close()
    at = _free_run(wl, 10, n_populations=2, n_fireworks=1, n_sparks=16, n_guiding=2, seed=9, T=20)
    print(f"{widths}: diverged_at={at}")


def test_input_problem_errors():
    torch, M = require_gpu()
    wl = inputs.testbed_net(2)
    with pytest.raises(M.MgfwaError) as e:
        M.MGFWA.from_workload(wl, precision="bf16")
    assert "FP32" in str(e.value)
    bad = inputs.testbed_net(2)
    bad.widths = (10, 600, 1)
    bad.net = np.zeros(10 * 600 + 600 + 600 + 1, np.float32)
    with pytest.raises(M.MgfwaError):
        M.MGFWA.from_workload(bad)
