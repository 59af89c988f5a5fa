"""FP32 re-check of BF16 selections against the oracle (needs an MI355X).

With BF16 fitness the library ranks the candidates on their BF16 values but
re-evaluates each firework's best candidate in FP32 before the selection of
Alg. 1 compares it with the firework, so firework, initial and best-so-far
fitness are FP32 values.  Every generation is checked against the oracle:
c* is the argmin of the device's BF16 candidate fitness (lower index on ties,
exact), the oracle's binary64 loss of that candidate decides the move (unless
it is a near-tie), the moved row is the candidate bit for bit, the firework
fitness and best_y are within the FP32 tolerance of the oracle's loss of their
rows, and the amplitude follows the decision.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2501_03944_amd import inputs
from tests.gpu_util import assert_bits, assert_fitness_close, require_gpu

pytestmark = pytest.mark.gpu

REGISTER, WIDE = 1, 2   # fit_path: register-chain kernels, K-streamed wide-first-layer kernel

CASES = [
    # (problem, fit_path, fireworks, sparks, guiding, autotuned)
    ("teacher", REGISTER, 4, 16, 2, False),
    ("mlp-ce", REGISTER, 3, 16, 2, False),
    ("mlp-ce", REGISTER, 3, 16, 2, True),
    # FP32 hidden layers too wide for the LDS: the re-check reads the weights
    # from global memory (the tuner picks among those kernels)
    ("deep-ce", REGISTER, 3, 16, 2, False),
    ("deep-ce", REGISTER, 3, 16, 2, True),
    ("wide-ce", WIDE, 3, 16, 2, False),
    ("wide-mse", WIDE, 2, 24, 3, False),
]


def _problem(name):
    if name == "teacher":
        return inputs.teacher_regression(n_samples=192)
    if name == "mlp-ce":
        return inputs.random_mlp_problem((24, 48, 10), ("relu",), "ce", 400, seed=21)
    if name == "deep-ce":
        return inputs.random_mlp_problem((16, 176, 176, 10), ("relu", "relu"), "ce", 300, seed=17,
                                         x_scale=0.5)
    if name == "wide-ce":
        return inputs.random_mlp_problem((40, 64, 5), ("relu",), "ce", 300, seed=11)
    return inputs.random_mlp_problem((33, 48, 3), ("tanh",), "mse", 260, seed=13)


def _near(a, b, rel=2e-5):
    a, b = float(a), float(b)
    if not (np.isfinite(a) and np.isfinite(b)):
        return a == b
    return abs(a - b) <= rel * max(abs(a), abs(b))


@pytest.mark.parametrize("name,path,N,lam,G,tune", CASES)
def test_bf16_selection_rechecked_in_fp32(name, path, N, lam, G, tune):
    torch, M = require_gpu()
    wl = _problem(name)
    p = O.Problem.from_workload(wl)
    T = 40
    g = M.MGFWA(wl.widths, wl.acts, wl.loss, wl.x, wl.y, wl.labels, n_fireworks=N,
                n_sparks=lam, n_guiding=G, seed=3, precision="bf16", max_generations=T,
                fit_path=path)
    if tune:
        g.autotune(2)
    cfg = O.make_config(N=N, lam=lam, G=G, seed=3, T=T)
    D = g.D
    st = g.state_numpy()
    # the initial firework fitness is FP32
    assert_fitness_close(st["Y"], p.loss_rows(st["F"][:, :D].astype(np.float64)), "initial Y")
    moves = 0
    for gen in range(1, 9):
        before = st
        g.step(1)
        st = g.state_numpy()
        Yc = st["Yc"]
        for f in range(N):
            # c*: lowest BF16 candidate fitness, lower index on ties
            row = Yc[f]
            cs = int(np.flatnonzero(row == row.min())[0])
            assert int(st["cstar"][f]) == cs, (gen, f)
            if cs < lam:
                cand = O.explosion_row(cfg, before["F"][f, :D], before["A"][f], f * lam + cs, gen)
            else:
                cand = st["SG"][f * G + cs - lam, :D]
            y32 = float(p.loss_rows(cand[None, :].astype(np.float64))[0])
            yold = float(before["Y"][f])
            assert st["Yprev"][f] == np.float32(yold)
            if st["reinit"][f]:
                assert st["Y"][f] == np.inf and st["A"][f] == np.float32(cfg.ub - cfg.lb)
                continue
            if _near(y32, yold):
                continue
            want_move = np.float32(y32) < np.float32(yold)
            assert bool(st["improved"][f]) == want_move, (gen, f, y32, yold)
            if want_move:
                moves += 1
                assert_bits(st["F"][f, :D], cand, f"generation {gen} firework {f} row")
                assert_fitness_close([st["Y"][f]], [y32], f"generation {gen} firework {f} Y")
                assert st["A"][f] == np.float32(before["A"][f] * np.float32(1.2))
            else:
                assert st["Y"][f] == np.float32(yold)
                assert_bits(st["F"][f, :D], before["F"][f, :D], f"generation {gen} firework {f}")
                assert st["A"][f] == np.float32(before["A"][f] * np.float32(0.9))
        # best-so-far: FP32 fitness of the stored row
        assert_fitness_close(st["best_y"], p.loss_rows(st["best_x"][:, :D].astype(np.float64)),
                             f"generation {gen} best_y")
        assert st["best_y"][0] <= before["best_y"][0]
    assert moves > 0
    g.close()


def test_recheck_time_reported_for_bf16_only():
    torch, M = require_gpu()
    wl = inputs.random_mlp_problem((40, 64, 5), ("relu",), "ce", 300, seed=11)
    for prec in ("bf16", "fp32"):
        g = M.MGFWA(wl.widths, wl.acts, wl.loss, wl.x, wl.y, wl.labels, n_fireworks=3,
                    n_sparks=16, n_guiding=2, seed=5, precision=prec)
        g.set_timing(True)
        g.step(3)
        t = g.timing()
        g.close()
        assert t["generations"] == 3
        if prec == "bf16":
            assert 0.0 < t["check_fit_ms"] <= t["phase_ms"]["selection"]
        else:
            assert t["check_fit_ms"] == 0.0


def test_every_recheck_plan_matches_oracle():
    """Each candidate plan of the FP32 re-check launch (plan index 2), forced
    through mgfwa_set_fit_plan on a net whose re-check reads its weights from
    global memory: over a few generations every firework fitness and best_y is
    within the FP32 tolerance of the oracle's loss of its row, and some firework
    moved (so re-checked values were used)."""
    torch, M = require_gpu()
    wl = _problem("deep-ce")
    p = O.Problem.from_workload(wl)

    def ctx(precision="bf16"):
        return M.MGFWA(wl.widths, wl.acts, wl.loss, wl.x, wl.y, wl.labels, n_fireworks=3,
                       n_sparks=16, n_guiding=2, seed=4, precision=precision, max_generations=20,
                       fit_path=REGISTER)

    g0 = ctx()
    # before tuning, a launch of 3 rows (far too few to fill the chip) takes one
    # slab group per wavefront: as many blocks per row as the samples allow
    info = g0.fit_plan(2)
    assert info["samples_per_block"] == info["wavefronts"] * 16 * info["slabs"], info
    cands = g0.fit_candidates(2)
    assert len(cands) >= 2 and all(c["rows"] == 3 for c in cands)
    with pytest.raises(M.MgfwaError) as e:
        g0.set_fit_plan(2, len(cands))
    assert e.value.status == M.EINVAL
    with pytest.raises(M.MgfwaError) as e:
        g0.fit_plan(3)
    assert e.value.status == M.EINVAL
    g0.close()
    g32 = ctx("fp32")
    with pytest.raises(M.MgfwaError) as e:   # FP32 runs have no re-check launch
        g32.fit_plan(2)
    assert e.value.status == M.ESTATE
    g32.close()
    for i, plan in enumerate(cands):
        g = ctx()
        g.set_fit_plan(2, i)
        assert g.fit_plan(2) == plan
        moved = 0
        for gen in range(6):
            g.step(1)
            st = g.state_numpy()
            D = g.D
            moved += int(st["improved"].sum())
            keep = np.flatnonzero(st["reinit"] == 0)   # loser-out rows wait for their fitness
            assert_fitness_close(st["Y"][keep],
                                 p.loss_rows(st["F"][keep, :D].astype(np.float64)),
                                 f"plan {i} generation {gen + 1} Y")
            assert_fitness_close(st["best_y"],
                                 p.loss_rows(st["best_x"][:, :D].astype(np.float64)),
                                 f"plan {i} generation {gen + 1} best_y")
        assert moved > 0, f"plan {i}: no firework moved"
        g.close()
    print(f"{len(cands)} re-check plans checked")
