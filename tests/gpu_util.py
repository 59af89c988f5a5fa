"""Helpers for the GPU parity tests: oracle and HIP contexts with one configuration.

The oracle never receives a value produced by the HIP path; the HIP path may be
fed the oracle's fitness through the library's tell entry point.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

FIT_RTOL = 1e-5       # FP32 fitness tolerance (relative)
FIT_ATOL = 1e-7       # absolute floor for losses near zero


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm device")
    from paper_2501_03944_amd import mgfwa as M
    M.lib()            # raises if the library is missing: no fallback
    return torch, M


def make_pair(wl, n_populations=1, n_fireworks=None, n_sparks=None, n_guiding=None, sigma=0.2,
              boost=1.0, amp_up=1.2, amp_down=0.9, T=None, seed=0, loser_out=True, target=None,
              external=False, precision="fp32", with_oracle=True, lag_guiding=False,
              map_range=False, fit_path=0, regen_sparks=False):
    torch, M = require_gpu()
    N = n_fireworks or wl.n_fireworks
    lam = n_sparks or wl.n_sparks
    G = n_guiding or wl.n_guiding
    T = T or wl.generations
    o = None
    if with_oracle:
        p = O.Problem.from_workload(wl)
        o = O.Oracle(p, B=n_populations, N=N, lam=lam, G=G, sigma=sigma, boost=boost,
                     amp_up=amp_up, amp_down=amp_down, lb=wl.lb, ub=wl.ub, T=T, seed=seed,
                     loser_out=int(loser_out), use_target=int(target is not None),
                     target_loss=0.0 if target is None else target,
                     lag_guiding=int(lag_guiding), map_range=int(map_range))
    prob = (dict(net=wl.net) if getattr(wl, "net", None) is not None else
            dict(loss=wl.loss, x=wl.x, y=wl.y, labels=wl.labels))
    g = M.MGFWA(wl.widths, wl.acts, **prob, n_populations=n_populations,
                n_fireworks=N, n_sparks=lam, n_guiding=G, sigma=sigma, boost=boost,
                amp_up=amp_up, amp_down=amp_down, lb=wl.lb, ub=wl.ub, max_generations=T,
                loser_out=loser_out, precision=precision, external_fitness=external,
                target_loss=target, seed=seed, lag_guiding=lag_guiding, map_range=map_range,
                fit_path=fit_path, regen_sparks=regen_sparks)
    return o, g


def gpu_rows(t, D):
    """Host copy of a [rows, Dp] device view; checks that the padding is zero."""
    a = t.cpu().numpy()
    assert np.all(a[:, D:] == 0.0), "row padding must stay zero"
    return a[:, :D]


def assert_bits(a, b, what):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if a.dtype.kind == "f":
        same = (a.view(np.uint32 if a.dtype == np.float32 else np.uint64) ==
                b.astype(a.dtype).view(np.uint32 if a.dtype == np.float32 else np.uint64))
    else:
        same = a == b
    if not np.all(same):
        idx = np.argwhere(~same)[:5]
        raise AssertionError(f"{what}: {int((~same).sum())} mismatches, first at {idx.tolist()}: "
                             f"{[a[tuple(i)] for i in idx]} vs {[b[tuple(i)] for i in idx]}")


def assert_fitness_close(got, want64, what, rtol=FIT_RTOL, atol=FIT_ATOL):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want64, dtype=np.float64)
    with np.errstate(invalid="ignore"):         # inf - inf where both are infinite
        err = np.abs(got - want)
    bound = rtol * np.abs(want) + atol
    bad = ~(err <= bound) & ~(got == want)      # equal infinities (reinitialised) agree
    if np.any(bad):
        i = np.argwhere(bad)[:5]
        raise AssertionError(f"{what}: {int(bad.sum())}/{bad.size} outside tolerance; "
                             f"max rel err {float((err / np.maximum(np.abs(want), 1e-30)).max()):.3e}; "
                             f"first {i.tolist()}: {got[tuple(i[0])]} vs {want[tuple(i[0])]}")


def compare_state(ov, gs, D, B, what, with_sparks=True):
    """Bit-exact comparison of the oracle view and the GPU state (host copies)."""
    F = gs["F"][:, :D]
    assert np.all(gs["F"][:, D:] == 0)
    assert_bits(F, ov["F"], f"{what} F")
    for k in ("A", "Y", "Yprev"):
        assert_bits(gs[k], ov[k], f"{what} {k}")
    for k in ("fresh",):
        assert_bits(gs[k], ov[k], f"{what} {k}")
    assert_bits(gs["best_y"], ov["best_y"], f"{what} best_y")
    assert_bits(gs["best_f"], ov["best_f"], f"{what} best_f")
    assert_bits(gs["best_gen"], ov["best_gen"], f"{what} best_gen")
    assert_bits(gs["best_x"][:, :D], ov["best_x"], f"{what} best_x")
    if with_sparks:
        assert_bits(gs["SE"][:, :D], ov["SE"], f"{what} SE")
        assert_bits(gs["SG"][:, :D], ov["SG"], f"{what} SG")


def near_tie_present(prev, cur, lam, G, m, k, rel=2 * FIT_RTOL, guide_yc=None, check_guide=True,
                     atol=1e-30, T=None, N=None, loser_out=True, target=None):
    """True when some decision of the oracle's last generation compared two
    fitness values within `rel` of each other (either branch is then valid).
    guide_yc: the candidate fitness the guiding cut ranked (the previous
    generation's in the lag order; the current one by default); check_guide
    False when no guiding cut was made (the lag order's first generation);
    atol: an absolute closeness floor (fitness bounds that are not relative).
    With T (generation budget) and N (fireworks per population) the loser-out
    comparison fma(-(Yprev - Y), max(T - t, 0), Y) > Y_b is checked too, with
    the margin an error of `rel` in Y and Yprev propagates to both sides; with
    target, the stop test best_y <= target."""
    def close(a, b):
        a, b = float(a), float(b)
        if not (np.isfinite(a) and np.isfinite(b)):
            return False
        return abs(a - b) <= rel * max(abs(a), abs(b)) + atol

    if target is not None and close(np.min(cur["best_y"]), target):
        return True
    if T is not None and N is not None and loser_out and loser_out_near_tie(prev, cur, T, N, rel,
                                                                             atol):
        return True

    Yc = cur["Yc"]
    Yg = Yc if guide_yc is None else guide_yc
    BN = Yc.shape[0]
    for gf in range(BN):
        row = Yc[gf]
        # guiding cut: ranks k-1 / k and m-k-1 / m-k inside each group
        for g in range(G if check_guide else 0):
            grp = np.sort(Yg[gf, g * m:(g + 1) * m].astype(np.float64))
            if close(grp[k - 1], grp[k]) or close(grp[m - k - 1], grp[m - k]):
                return True
        srt = np.sort(row.astype(np.float64))
        if close(srt[0], srt[1]):
            return True                       # argmin over candidates
        if close(srt[0], prev["Y"][gf]):
            return True                       # improvement test
    Y = cur["Y"]
    fin = np.sort(Y[np.isfinite(Y)].astype(np.float64))
    if fin.size > 1 and close(fin[0], fin[1]):
        return True                           # population best
    return False


def loser_out_near_tie(prev, cur, T, N, rel=2 * FIT_RTOL, atol=1e-30):
    """True when a loser-out comparison of the oracle's last generation lies
    within the margin an FP32 fitness error of `rel` could move it across.
    The fitness after selection is rebuilt from the decisions (a restarted
    firework's stored fitness is +inf)."""
    Yc = cur["Yc"].astype(np.float64)
    BN = Yc.shape[0]
    ysel = np.where(cur["improved"] == 1, Yc[np.arange(BN), cur["cstar"]],
                    prev["Y"].astype(np.float64))
    yprev = prev["Y"].astype(np.float64)
    rem = float(max(T - int(cur["t"]), 0))
    for b0 in range(0, BN, N):
        ys = ysel[b0:b0 + N]
        fb = int(np.argmin(ys))
        yb = ys[fb]
        if not np.isfinite(yb):
            continue
        for f in range(N):
            gf = b0 + f
            if f == fb or prev["fresh"][gf]:
                continue
            y, yp = ysel[gf], yprev[gf]
            if not (np.isfinite(y) and np.isfinite(yp)):
                continue
            pred = y - (yp - y) * rem
            margin = rel * (abs(y) + rem * (abs(yp) + abs(y)) + abs(yb)) + atol
            if abs(pred - yb) <= margin:
                return True
    return False


EXACT_KEYS = ("F", "A", "cstar", "reinit", "top", "bottom", "tie")


def check_generation(o, prev, ov, gs, D, gen, lag=False, sparks=True, atol=1e-30, what=""):
    """One free-running generation of the library (host state gs) against the
    oracle's (view ov; prev = its view before the generation).  Every fitness
    must lie within the FP32 tolerance.  Positions, amplitudes and decisions must
    agree bit for bit, unless a decision of the generation compared two values
    within that tolerance (either branch is then correct).  Returns True while
    the two agree and False at the generation where they part at a near-tie."""
    c = o.cfg
    assert_fitness_close(gs["Yc"], ov["Yc64"], f"{what} gen {gen} candidate fitness")
    assert_fitness_close(gs["Y"], ov["Y"], f"{what} gen {gen} firework fitness")
    same = all(np.array_equal(gs[k][:, :D] if k == "F" else gs[k], ov[k]) for k in EXACT_KEYS)
    if not same:
        diff = [k for k in EXACT_KEYS
                if not np.array_equal(gs[k][:, :D] if k == "F" else gs[k], ov[k])]
        print(f"{what} gen {gen}: {diff} differ")
        assert near_tie_present(prev, ov, c.lam, c.G, ov["m"], ov["k"],
                                guide_yc=prev["Yc"] if lag else None,
                                check_guide=not (lag and gen == 1), atol=atol, T=c.T, N=c.N,
                                loser_out=bool(c.loser_out),
                                target=c.target_loss if c.use_target else None), \
            f"{what}: divergence at generation {gen} without a near-tie"
        return False
    assert_bits(gs["best_x"][:, :D], ov["best_x"], f"{what} gen {gen} best_x")
    assert_bits(gs["best_f"], ov["best_f"], f"{what} gen {gen} best_f")
    assert_bits(gs["best_gen"], ov["best_gen"], f"{what} gen {gen} best_gen")
    assert_fitness_close(gs["best_y"], ov["best_y"], f"{what} gen {gen} best_y")
    if sparks:
        assert_bits(gs["SE"][:, :D], ov["SE"], f"{what} gen {gen} SE")
    assert_bits(gs["SG"][:, :D], ov["SG"], f"{what} gen {gen} SG")
    assert int(gs["gen"][0]) == int(ov["t"]), f"{what} gen counter"
    return True


def oracle_near_tie_generation(o, gens):
    """Run the oracle from initialisation for up to `gens` generations (or to its
    stop flag); the first generation whose decisions compared two values within
    the FP32 fitness tolerance, or None.  Up to that generation a library run of
    the same job must agree with the oracle bit for bit."""
    c = o.cfg
    o.init()
    v = o.view()
    B, N = c.B, c.N
    y = v["Y"].astype(np.float64).reshape(B, N)
    for b in range(B):                        # the initial population best
        srt = np.sort(y[b][np.isfinite(y[b])])
        if srt.size > 1 and abs(srt[0] - srt[1]) <= 2 * FIT_RTOL * max(abs(srt[0]), abs(srt[1])):
            return 0
    for gen in range(1, gens + 1):
        prev = o.view()
        o.generation()
        cur = o.view()
        if near_tie_present(prev, cur, c.lam, c.G, cur["m"], cur["k"], T=c.T, N=N,
                            loser_out=bool(c.loser_out),
                            target=c.target_loss if c.use_target else None,
                            guide_yc=prev["Yc"] if c.lag_guiding else None,
                            check_guide=not (c.lag_guiding and gen == 1)):
            return gen
        if B > 1:                             # the answer picks the best population
            by = np.sort(cur["best_y"].astype(np.float64))
            if abs(by[0] - by[1]) <= 2 * FIT_RTOL * max(abs(by[0]), abs(by[1])):
                return gen
        if cur["done"]:
            break
    return None
