"""Parity of the HIP path with the oracle (needs an MI355X).

Bit-exact: initial positions, explosion sparks, ranking sets, guiding sparks,
selection, amplitudes, loser-out and best-so-far, given the same fitness.
Within 1e-5 relative (FP32): every fitness value.
"""
import numpy as np
import pytest

from gpu_util import (assert_bits, assert_fitness_close, check_generation, compare_state,
                      gpu_rows, make_pair, require_gpu)
from oracle import oracle as O
from paper_2501_03944_amd import inputs

pytestmark = pytest.mark.gpu


def _lockstep(wl, gens, check_fitness=True, **cfg):
    """Drive the GPU state path with the oracle's fitness through ask/tell and
    compare every array after every phase."""
    torch, M = require_gpu()
    o, g = make_pair(wl, external=True, **cfg)
    D = g.D
    c = o.cfg
    lam, G = c.lam, c.G
    o.init_positions()
    F = gpu_rows(g.ask(), D)
    assert_bits(F, o.view()["F"], "init F")
    o.eval_init()
    ov = o.view()
    if check_fitness:
        yg = g.evaluate(g.state()["F"]).cpu().numpy()
        assert_fitness_close(yg, o.problem.loss_rows(ov["F"]), "init fitness")
    g.tell(torch.from_numpy(ov["Y"].copy()))
    gs = g.state_numpy()
    compare_state(ov, gs, D, c.B, "init", with_sparks=False)
    for gen in range(1, gens + 1):
        o.explode()
        se_dev = g.ask()
        se = gpu_rows(se_dev, D)
        assert_bits(se, o.view()["SE"], f"gen {gen} SE")
        o.eval_explosion()
        ov = o.view()
        if check_fitness:
            yg = g.evaluate(se_dev).cpu().numpy()
            assert_fitness_close(yg, ov["Yc64"][:, :lam].reshape(-1), f"gen {gen} explosion fitness")
        g.tell(torch.from_numpy(ov["Yc"][:, :lam].reshape(-1).copy()))
        o.guide()
        sg_dev = g.ask()
        ov = o.view()
        gs = g.state_numpy()
        assert_bits(gs["top"], ov["top"], f"gen {gen} top")
        assert_bits(gs["bottom"], ov["bottom"], f"gen {gen} bottom")
        assert_bits(gs["tie"], ov["tie"], f"gen {gen} tie")
        assert_bits(gpu_rows(sg_dev, D), ov["SG"], f"gen {gen} SG")
        o.eval_guiding()
        ov = o.view()
        if check_fitness:
            yg = g.evaluate(sg_dev).cpu().numpy()
            assert_fitness_close(yg, ov["Yc64"][:, lam:].reshape(-1), f"gen {gen} guiding fitness")
        g.tell(torch.from_numpy(ov["Yc"][:, lam:].reshape(-1).copy()))
        o.select()
        ov = o.view()
        gs = g.state_numpy()
        compare_state(ov, gs, D, c.B, f"gen {gen}")
        for k in ("cstar", "improved", "reinit"):
            assert_bits(gs[k], ov[k], f"gen {gen} {k}")
        assert int(gs["gen"][0]) == gen
    g.close()


def test_lockstep_teacher_100_generations():
    wl = inputs.teacher_regression()
    _lockstep(wl, 100)


@pytest.mark.parametrize("cfg", [
    dict(n_populations=3, n_fireworks=2, n_sparks=8, n_guiding=2, T=6, seed=11),
    dict(n_fireworks=3, n_sparks=12, n_guiding=3, boost=1.75, sigma=0.5, seed=5, T=40),
    dict(n_fireworks=5, n_sparks=2, n_guiding=1, sigma=0.5, seed=9, loser_out=False),
    # one firework per population: it is always its population's best (no loser-out)
    dict(n_populations=2, n_fireworks=1, n_sparks=8, n_guiding=2, seed=15, T=20),
    # groups of 64 (one wavefront each) and of 128 members (the per-firework path)
    dict(n_fireworks=2, n_sparks=128, n_guiding=2, seed=13, T=30),
    dict(n_fireworks=2, n_sparks=256, n_guiding=2, sigma=0.3, seed=14, T=30),
])
def test_lockstep_variants(cfg):
    wl = inputs.teacher_regression(n_samples=96, widths=(5, 7, 2), seed=77)
    _lockstep(wl, 15, **cfg)


def test_lockstep_gaussian_mixture_shape():
    # the 64-128-128-10 network (D = 26,122) on a reduced population and sample set
    wl = inputs.gaussian_mixture(n_samples=300)
    _lockstep(wl, 3, n_fireworks=2, n_sparks=16, n_guiding=4, T=50, seed=3)


def test_free_running_teacher_matches_oracle():
    """mgfwa_step with the library's own FP32 fitness against the oracle: the
    states agree bit for bit until a decision compares two fitness values that
    lie within the fitness tolerance of each other."""
    torch, M = require_gpu()
    wl = inputs.teacher_regression()
    o, g = make_pair(wl)
    D = g.D
    o.init()
    gs = g.state_numpy()
    ov = o.view()
    assert_bits(gs["F"][:, :D], ov["F"], "init F")
    assert_fitness_close(gs["Y"], ov["Y"], "init Y")
    diverged_at = None
    for gen in range(1, 101):
        prev = o.view()
        o.generation()
        g.step(1)
        if not check_generation(o, prev, o.view(), g.state_numpy(), D, gen):
            diverged_at = gen
            break
    print(f"free-running: diverged_at={diverged_at}")
    g.close()


def test_graph_replay_equals_direct_launches():
    torch, M = require_gpu()
    wl = inputs.teacher_regression()
    _, g1 = make_pair(wl, with_oracle=False, seed=4)
    _, g2 = make_pair(wl, with_oracle=False, seed=4)
    g2.set_timing(True)          # timing mode launches kernel by kernel
    for _ in range(3):
        g1.step(10)
        g2.step(10)
        torch.cuda.synchronize()
        s1, s2 = g1.state_numpy(), g2.state_numpy()
        for k in ("F", "A", "Y", "SE", "SG", "Yc", "best_x", "best_y", "gen"):
            assert_bits(s1[k], s2[k], f"graph vs direct {k}")
    t = g2.timing()
    assert t["generations"] == 30 and all(v > 0 for v in t["phase_ms"].values())
    x, f, gen = g1.best()
    assert gen == 30 and np.isfinite(f)
    assert_bits(x, s1["best_x"][0, :g1.D], "best x")
    g1.close()
    g2.close()


def test_same_seed_same_state_different_seed_differs():
    torch, M = require_gpu()
    wl = inputs.teacher_regression(n_samples=64)
    runs = []
    for seed in (21, 21, 22):
        _, g = make_pair(wl, with_oracle=False, seed=seed, n_fireworks=3, n_sparks=16, n_guiding=2)
        g.step(25)
        runs.append(g.state_numpy())
        g.close()
    assert_bits(runs[0]["F"], runs[1]["F"], "same seed")
    assert not np.array_equal(runs[0]["F"], runs[2]["F"])


def test_target_loss_stops_generations():
    """The stop test runs on the device: both sides stop at the same generation
    unless a decision on the way (or the stop test itself) compared values
    within the fitness tolerance."""
    torch, M = require_gpu()
    wl = inputs.teacher_regression()
    o, g = make_pair(wl, target=40.0, T=200)
    D = g.D
    o.init()
    assert_fitness_close(g.state_numpy()["Y"], o.view()["Y"], "init Y")
    parted = None
    for gen in range(1, 201):
        prev = o.view()
        o.generation()
        g.step(1)
        ov, gs = o.view(), g.state_numpy()
        if not check_generation(o, prev, ov, gs, D, gen):
            parted = gen
            break
        if int(gs["done"][0]) != ov["done"]:
            # only a best fitness within the tolerance of the target may stop one side only
            assert abs(float(ov["best_y"].min()) - 40.0) <= 2e-5 * 40.0, f"stop flag at {gen}"
            parted = gen
            break
        if ov["done"]:
            break
    x, f, gen = g.best()
    if parted is None:
        assert ov["done"] == 1 and gen == ov["t"] < 200
        assert f <= 40.0
    print(f"target stop: oracle t={ov['t']}, library generation {gen}, parted at {parted}")
    g.close()


def test_ask_tell_protocol_errors():
    torch, M = require_gpu()
    wl = inputs.teacher_regression(n_samples=32)
    _, g = make_pair(wl, with_oracle=False, external=True)
    with pytest.raises(M.MgfwaError) as e:
        g.step(1)
    assert e.value.status == M.ESTATE
    with pytest.raises(M.MgfwaError) as e:
        g.tell(torch.zeros(4, device="cuda"))
    assert e.value.status == M.ESTATE
    g.ask()
    with pytest.raises(M.MgfwaError):
        g.ask()
    g.tell(torch.full((4,), float("nan"), device="cuda"))   # NaN fitness is +inf
    st = g.state_numpy()
    assert np.all(np.isinf(st["Y"]))
    g.close()
