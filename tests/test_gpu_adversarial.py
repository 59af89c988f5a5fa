"""The device state path fed adversarial fitness through ask/tell, against the
oracle fed the same values (needs an MI355X).

Both sides receive identical fitness, so every array must agree bit for bit:
initial positions, explosion sparks, the top/bottom member lists and all-tie
flags of every guiding group, guiding sparks, selection (c*, improvement),
amplitudes, loser-out restarts, fresh flags and the best-so-far record.  The
fitness pools are built to hit the corners of the rank key and the decisions
(Alg. 1, guiding, selection and loser-out steps; the tie, NaN and signed-zero
readings): many equal values, equal keys at the k-th place of a group, -0 next
to +0, NaN (stored as +inf), +inf, whole groups that tie, and the hand-worked
guiding groups and loser-out tables of tests/golden replayed on the device.
"""
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN
from gpu_util import assert_bits, compare_state, gpu_rows, make_pair, require_gpu
from paper_2501_03944_amd import inputs

pytestmark = pytest.mark.gpu

POOL = np.array([0.0, -0.0, 1.0, 1.0, 2.5, 0.5, -3.0, np.inf, np.nan, 7.0], dtype=np.float32)


def _tie_heavy(rng, rows, m):
    """Fitness for `rows` sparks in groups of m: values from a small pool with
    repeats, and per group one of: pool draws, an all-equal group, or a group
    whose k-th and (k+1)-th smallest values are equal (keys tie at the cut)."""
    y = POOL[rng.integers(0, POOL.size, rows)].copy()
    for g0 in range(0, rows - m + 1, m):
        kind = rng.integers(0, 5)
        if kind == 0:
            y[g0:g0 + m] = POOL[rng.integers(0, POOL.size)]           # the group ties
        elif kind == 1:
            y[g0:g0 + m] = rng.choice([0.0, -0.0], m).astype(np.float32)  # +0 / -0 only
        elif kind == 2:
            y[g0:g0 + m] = np.round(rng.normal(size=m), 1).astype(np.float32)  # near-continuous
    return y


class _Pair:
    """The oracle and a tell-mode library context driven with the same fitness."""

    def __init__(self, wl, **cfg):
        self.torch, self.M = require_gpu()
        self.o, self.g = make_pair(wl, external=True, **cfg)
        self.D = self.g.D
        self.c = self.o.cfg

    def tell(self, what, y):
        y = np.ascontiguousarray(y, dtype=np.float32)
        getattr(self.o, "tell_" + what)(y)
        self.g.tell(self.torch.from_numpy(y.copy()))

    def init(self, y):
        self.o.init_positions()
        assert_bits(gpu_rows(self.g.ask(), self.D), self.o.view()["F"], "init F")
        self.tell("init", y)
        compare_state(self.o.view(), self.g.state_numpy(), self.D, self.c.B, "init",
                      with_sparks=False)

    def generation(self, gen, y_expl, y_guide):
        D = self.D
        self.o.explode()
        assert_bits(gpu_rows(self.g.ask(), D), self.o.view()["SE"], f"gen {gen} SE")
        self.tell("explosion", y_expl)
        self.o.guide()
        sg = gpu_rows(self.g.ask(), D)
        ov, gs = self.o.view(), self.g.state_numpy()
        for k in ("top", "bottom", "tie"):
            assert_bits(gs[k], ov[k], f"gen {gen} {k}")
        assert_bits(sg, ov["SG"], f"gen {gen} SG")
        self.tell("guiding", y_guide)
        self.o.select()
        ov, gs = self.o.view(), self.g.state_numpy()
        compare_state(ov, gs, D, self.c.B, f"gen {gen}")
        for k in ("cstar", "improved", "reinit"):
            assert_bits(gs[k], ov[k], f"gen {gen} {k}")
        return ov, gs

    def close(self):
        self.g.close()


SHAPES = [
    dict(n_fireworks=3, n_sparks=16, n_guiding=2, T=12, seed=1),                    # k = 1
    dict(n_fireworks=2, n_sparks=128, n_guiding=2, T=12, seed=2),                   # m = 64: one wavefront
    dict(n_fireworks=2, n_sparks=256, n_guiding=2, sigma=0.3, T=12, seed=3),        # m = 128: k_rank
    dict(n_populations=2, n_fireworks=3, n_sparks=12, n_guiding=3, sigma=0.5, boost=1.75,
         T=12, seed=4),                                                             # m = 4, k = 2
    dict(n_fireworks=4, n_sparks=8, n_guiding=1, sigma=0.5, T=5, seed=5),           # short budget
]


@pytest.mark.parametrize("cfg", SHAPES)
def test_tie_heavy_fitness_bit_exact(cfg):
    wl = inputs.teacher_regression(n_samples=16, widths=(5, 7, 2), seed=77)
    p = _Pair(wl, **cfg)
    c = p.c
    BN, m = c.B * c.N, c.lam // c.G
    rng = np.random.default_rng(100 + cfg["seed"])
    p.init(POOL[rng.integers(0, POOL.size, BN)])
    seen_tie = seen_reinit = 0
    for gen in range(1, 13):
        ov, gs = p.generation(gen, _tie_heavy(rng, BN * c.lam, m),
                              _tie_heavy(rng, BN * c.G, c.G))
        seen_tie += int(gs["tie"].sum())
        seen_reinit += int(gs["reinit"].sum())
    print(f"{cfg}: tied groups {seen_tie}, restarts {seen_reinit}")
    assert seen_tie > 0
    p.close()


def test_tie_heavy_fitness_wide_spark_rows():
    """A long spark row (D = 26,122: many 4-coordinate chunks per row)."""
    wl = inputs.gaussian_mixture(n_samples=16)
    p = _Pair(wl, n_fireworks=2, n_sparks=16, n_guiding=4, T=8, seed=6)
    c = p.c
    rng = np.random.default_rng(6)
    p.init(POOL[rng.integers(0, POOL.size, c.N)])
    for gen in range(1, 6):
        p.generation(gen, _tie_heavy(rng, c.N * c.lam, c.lam // c.G), _tie_heavy(rng, c.N * c.G, 1))
    p.close()


def _f(v):
    return np.float32(float(v))


def test_golden_guiding_groups_on_device():
    """tests/golden/guiding_groups.json: the hand-worked groups' fitness told to
    one group of m sparks; the device's member lists and tie flag equal the
    hand-worked ones, and its guiding spark equals the oracle's (both built
    from the same generated sparks)."""
    cases = json.load(open(os.path.join(GOLDEN, "guiding_groups.json")))["cases"]
    wl = inputs.teacher_regression(n_samples=16, widths=(5, 7, 2), seed=77)
    for case in cases:
        m, k = case["m"], case["k"]
        p = _Pair(wl, n_fireworks=1, n_sparks=m, n_guiding=1, sigma=k / m, boost=case["boost"],
                  T=4, seed=31)
        assert p.o.view()["k"] == k
        p.init([5.0])
        y = np.array([_f(v) for v in case["fitness"]], dtype=np.float32)
        D = p.D
        p.o.explode()
        p.g.ask()
        p.tell("explosion", y)
        p.o.guide()
        sg = gpu_rows(p.g.ask(), D)
        gs, ov = p.g.state_numpy(), p.o.view()
        assert gs["top"][0].tolist() == case["top"], case["name"]
        assert gs["bottom"][0].tolist() == case["bottom"], case["name"]
        assert int(gs["tie"][0]) == case["tie"], case["name"]
        assert_bits(sg, ov["SG"], f"{case['name']} SG")
        if case["tie"]:
            assert_bits(sg, gs["F"][:, :D], f"{case['name']}: a tied group leaves the firework")
        p.close()


def test_golden_loser_out_tables_on_device():
    """tests/golden/loser_out_scenarios.json replayed through ask/tell: the
    device's decisions equal the hand-worked tables and the oracle's state."""
    scen = json.load(open(os.path.join(GOLDEN, "loser_out_scenarios.json")))["scenarios"]
    wl = inputs.teacher_regression(n_samples=16, widths=(5, 7, 2), seed=77)
    for sc in scen:
        p = _Pair(wl, n_fireworks=sc["N"], n_sparks=sc["lam"], n_guiding=sc["G"],
                  sigma=sc["sigma"], T=sc["T"], seed=41)
        a0 = np.float32(wl.ub) - np.float32(wl.lb)
        p.init([_f(v) for v in sc["init"]])
        for gen, step in enumerate(sc["generations"], start=1):
            ye = np.array([[_f(v) for v in row] for row in step["explosion"]]).reshape(-1)
            yg = np.array([[_f(v) for v in row] for row in step["guiding"]]).reshape(-1)
            ov, gs = p.generation(gen, ye, yg)
            what = f"{sc['name']} gen {gen}"
            assert gs["cstar"].tolist() == step["cstar"], what
            assert gs["improved"].tolist() == step["improved"], what
            assert gs["reinit"].tolist() == step["reinit"], what
            assert gs["fresh"].tolist() == step["fresh"], what
            assert_bits(gs["Y"], np.array([_f(v) for v in step["Y"]]), f"{what} Y")
            for f, reset in enumerate(step["A_reset"]):
                if reset:
                    assert gs["A"][f] == a0, what
            assert gs["best_y"][0] == _f(step["best_y"]), what
            assert int(gs["best_f"][0]) == step["best_f"], what
            assert int(gs["best_gen"][0]) == step["best_gen"], what
        p.close()


def test_signed_zero_and_nan_selection():
    """-0 never improves on +0 (strict <), NaN is +inf, equal candidates keep
    the lowest index, and an all-inf population keeps its fireworks."""
    wl = inputs.teacher_regression(n_samples=16, widths=(5, 7, 2), seed=77)
    p = _Pair(wl, n_fireworks=3, n_sparks=4, n_guiding=2, T=10, seed=51)
    p.init([0.0, np.nan, np.inf])
    ye = np.array([-0.0, 0.0, -0.0, 1.0,      # f0: nothing below +0
                   np.nan, 3.0, 3.0, np.nan,   # f1: 3 at c = 1 beats +inf
                   np.inf, np.inf, np.nan, np.inf], dtype=np.float32)
    yg = np.array([-0.0, 5.0, 3.0, 9.0, np.nan, np.inf], dtype=np.float32)
    ov, gs = p.generation(1, ye, yg)
    assert gs["improved"].tolist() == [0, 1, 0]
    assert gs["cstar"].tolist()[:2] == [0, 1]
    p.close()
