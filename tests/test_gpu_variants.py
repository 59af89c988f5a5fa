"""Alg. 1 variants on the HIP path against the oracle (needs an MI355X).

* Population-range random mapping (map_range): driven through ask/tell with the
  oracle's fitness, every array agrees bit for bit after every phase; driven by
  the library's own fitness, the states agree until a near-tie.
* One-generation-lag guiding order (lag_guiding): the guiding sparks of a
  generation come from the previous generation's sparks and fitness, and one
  fitness launch covers the explosion and the guiding sparks.  Free-running
  generations agree with the oracle's bit for bit (sparks, ranking sets,
  selection, amplitudes) until a decision compares two fitness values within
  the FP32 tolerance; every fitness value stays within that tolerance.
* Sparks regenerated instead of stored (regen_sparks): the fitness kernel draws
  each explosion spark from the counter-based generator while staging its
  weights; the state equals the stored-sparks run bit for bit and follows the
  oracle like every other run.
"""
import numpy as np
import pytest

from gpu_util import (assert_bits, assert_fitness_close, check_generation, make_pair,
                      require_gpu)
from oracle import oracle as O
from paper_2501_03944_amd import inputs
from test_gpu_parity import _lockstep

pytestmark = pytest.mark.gpu

def _free_run(wl, gens, **cfg):
    """Step the library and the oracle one generation at a time; returns the
    generation where they parted at a near-tie (None if they never did)."""
    torch, M = require_gpu()
    o, g = make_pair(wl, **cfg)
    D = g.D
    lag = bool(cfg.get("lag_guiding"))
    o.init()
    gs, ov = g.state_numpy(), o.view()
    assert_bits(gs["F"][:, :D], ov["F"], "init F")
    assert_fitness_close(gs["Y"], ov["Y"], "init Y")
    G = o.cfg.G
    try:
        for gen in range(1, gens + 1):
            prev = o.view()
            o.generation()
            g.step(1)
            ov, gs = o.view(), g.state_numpy()
            if gen == 1 and lag:
                assert np.all(gs["tie"] == 1), "first lagged guiding vectors must be zero"
                assert_bits(gs["SG"][:, :D], np.repeat(prev["F"], G, axis=0), "gen 1 SG")
            if not check_generation(o, prev, ov, gs, D, gen, lag=lag, sparks=g.sparks_materialised):
                return gen
        return None
    finally:
        g.close()


@pytest.mark.parametrize("cfg", [
    dict(map_range=True, n_fireworks=3, n_sparks=12, n_guiding=3, boost=1.75, seed=8, T=40),
    dict(map_range=True, n_populations=3, n_fireworks=2, n_sparks=8, n_guiding=2, T=6, seed=12),
])
def test_lockstep_range_mapping(cfg):
    wl = inputs.teacher_regression(n_samples=96, widths=(5, 7, 2), seed=77)
    _lockstep(wl, 15, **cfg)


@pytest.mark.parametrize("cfg", [
    dict(lag_guiding=True),
    dict(lag_guiding=True, map_range=True, n_populations=2, seed=3),
    dict(map_range=True, seed=5),
    dict(lag_guiding=True, n_fireworks=3, n_sparks=12, n_guiding=3, boost=1.75, sigma=0.5,
         seed=9, loser_out=False),
])
def test_free_running_variants_match_oracle(cfg):
    wl = inputs.teacher_regression()
    at = _free_run(wl, 60, **cfg)
    print(f"{cfg}: diverged_at={at}")


def test_lag_order_through_the_wide_kernel():
    """The combined explosion + guiding launch routed to the wide-first-layer
    kernel writes each row's fitness to its own candidate slot."""
    wl = inputs.random_mlp_problem((40, 64, 5), ("relu",), "ce", 300, seed=3)
    at = _free_run(wl, 8, lag_guiding=True, n_fireworks=3, n_sparks=16, n_guiding=2, seed=5,
                   T=30, fit_path=2)
    print(f"wide lag: diverged_at={at}")


def test_lag_plan_covers_both_spark_kinds():
    torch, M = require_gpu()
    wl = inputs.gaussian_mixture(n_samples=300)
    g = M.MGFWA.from_workload(wl, n_fireworks=2, n_sparks=16, n_guiding=4, lag_guiding=True)
    assert g.fit_plan(0)["rows"] == 2 * (16 + 4)
    g.autotune(1)
    assert g.fit_plan(0)["rows"] == 2 * (16 + 4)
    p = O.Problem.from_workload(wl)
    o = O.Oracle(p, N=2, lam=16, G=4, lb=wl.lb, ub=wl.ub, T=wl.generations, seed=0,
                 lag_guiding=1)
    o.init()
    for gen in range(1, 3):
        o.generation()
        g.step(1)
        assert_fitness_close(g.state_numpy()["Yc"], o.view()["Yc64"], f"gen {gen} tuned lag")
    g.close()


@pytest.mark.parametrize("cfg", [
    dict(regen_sparks=True),
    dict(regen_sparks=True, map_range=True, n_populations=2, seed=3),
])
def test_free_running_regenerated_sparks_match_oracle(cfg):
    torch, M = require_gpu()
    wl = inputs.teacher_regression()
    probe = M.MGFWA.from_workload(wl, regen_sparks=True)
    assert probe.fit_plan(0)["lds_weights"] == 1 and not probe.sparks_materialised
    probe.close()
    at = _free_run(wl, 60, **cfg)
    print(f"{cfg}: diverged_at={at}")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_regenerated_sparks_equal_stored_sparks(precision):
    """The same job with its explosion sparks stored and regenerated inside the
    fitness kernel: every array of the state is bit-identical each generation."""
    torch, M = require_gpu()
    wl = inputs.gaussian_mixture(n_samples=512)
    kw = dict(n_fireworks=3, n_sparks=32, n_guiding=4, seed=7, precision=precision,
              max_generations=40)
    a = M.MGFWA.from_workload(wl, **kw)
    b = M.MGFWA.from_workload(wl, regen_sparks=True, **kw)
    assert a.sparks_materialised and not b.sparks_materialised
    assert a.fit_plan(0) == b.fit_plan(0)
    for gen in range(1, 9):
        a.step(1)
        b.step(1)
        sa, sb = a.state_numpy(), b.state_numpy()
        for name in ("F", "A", "Y", "Yc", "SG", "top", "bottom", "best_x", "best_y", "reinit"):
            assert_bits(sb[name], sa[name], f"generation {gen} {name}")
    a.close()
    b.close()
