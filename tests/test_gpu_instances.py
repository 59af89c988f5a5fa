"""Every compiled fitness kernel instance at the full width of its row blocks
(needs an MI355X).

For networks whose hidden widths fill whole 16-row blocks, one generation is
run under every candidate plan of the explosion-fitness launch (every compiled
instance that covers the shape, with its sample splits).  FP32 plans must match
the oracle's binary64 loss within 1e-5; BF16 plans (same operand rounding, FP32
accumulation in a different order) must agree with each other within 1e-4
relative, and the first of them with the oracle within the BF16 bound.  A plan
that reads a stale register, a wrong LDS row or a padding column shows here.
"""
import numpy as np
import pytest

from gpu_util import assert_fitness_close, require_gpu
from oracle import oracle as O
from paper_2501_03944_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = ([(64, 16 * r, 10) for r in (2, 4, 6, 8, 10, 12, 14, 16)] +
          [(32, 16 * r, 16 * r, 10) for r in (2, 4, 6, 8, 10, 12, 14)] +
          [(16, 64, 64, 64, 10)])


def _explosion_fitness(M, wl, precision, plan, N, lam):
    g = M.MGFWA.from_workload(wl, precision=precision, seed=9, n_fireworks=N, n_sparks=lam,
                              n_guiding=2, max_generations=10)
    if plan is not None:
        g.set_fit_plan(0, plan)
    before = g.state_numpy()
    info = g.fit_plan(0)
    g.step(1)
    y = g.state_numpy()["Yc"][:, :lam].ravel().astype(np.float64)
    g.close()
    return y, before, info


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("widths", SHAPES, ids=lambda w: "-".join(map(str, w)))
def test_every_plan_at_full_width(widths, precision):
    torch, M = require_gpu()
    wl = inputs.random_mlp_problem(widths, ("relu",) * (len(widths) - 2), "ce", 300, seed=5,
                                   x_scale=0.5)
    N, lam = 2, 8
    probe = M.MGFWA.from_workload(wl, precision=precision, n_fireworks=N, n_sparks=lam, n_guiding=2)
    if probe.fit_plan(0)["wide"]:
        probe.close()
        pytest.skip("the wide kernel covers this shape (fixed tiles)")
    cands = probe.fit_candidates(0)
    probe.close()
    cfg = O.make_config(N=N, lam=lam, G=2, seed=9, T=10)
    p = O.Problem.from_workload(wl)
    ref = first = None
    for i, c in enumerate(cands):
        y, before, info = _explosion_fitness(M, wl, precision, i, N, lam)
        what = (f"{widths} {precision} plan {i}: lds={info['lds_weights']} "
                f"R={info['row_blocks']} P={info['slabs']} bpr={info['blocks_per_row']}")
        if ref is None:
            D = wl.dim
            se = np.stack([O.explosion_row(cfg, before["F"][r // lam, :D], before["A"][r // lam],
                                           r, 1) for r in range(N * lam)])
            ref = p.loss_rows(se)
        if precision == "fp32":
            assert_fitness_close(y, ref, what)
            continue
        rel = np.abs(y - ref) / np.abs(ref)
        if first is None:
            first = y
            assert rel.max() < 2e-2, f"{what}: max rel error {rel.max():.3e} against the oracle"
        else:
            d = np.abs(y - first) / np.abs(first)
            assert d.max() < 1e-4, f"{what}: differs from plan 0 by {d.max():.3e} (oracle {rel.max():.3e})"
