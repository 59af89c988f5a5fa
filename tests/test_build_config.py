"""Build configuration of the fitness kernel instances (no GPU, no compiler).

The instance files whose kernels all read the spark weights from global memory
are compiled with a raised full-unroll limit (their fully unrolled layer loops
exceed the default one, and a partly rolled loop indexes the activation tiles at
run time, which puts them in scratch memory).  The LDS-staged and mixed files
keep the default.  This checks that the build's list of such files matches the
instance tables, so a new or edited table cannot silently fall on the wrong side.
"""
import os
import re

from paper_2501_03944_amd import build

CSRC = os.path.join(os.path.dirname(build.__file__), "csrc")

# (macro, index of the weight-source argument among the macro's arguments); the
# two-precision macros fix it
WL_ARG = {"FIT_ENTRY": 1, "FIT_ENTRY_ACT": 1, "FIT_ENTRY_SCHED": 1}
FIXED = {"FIT_BOTH": "false", "FIT_BOTH_LDS": "true"}


def _weight_sources(path):
    text = open(path).read()
    body = text[text.index("kEntries[] = {"):]
    body = body[:body.index("};")]
    body = re.sub(r"//[^\n]*", "", body)
    found = []
    for m in re.finditer(r"\b(FIT_ENTRY_SCHED|FIT_ENTRY_ACT|FIT_ENTRY|FIT_BOTH_LDS|FIT_BOTH)\s*\(([^)]*)\)", body):
        name, args = m.group(1), [a.strip() for a in m.group(2).split(",")]
        found.append(FIXED[name] if name in FIXED else args[WL_ARG[name]])
    return found


def test_unroll_limit_goes_to_the_global_weight_files():
    tables = sorted(f for f in os.listdir(CSRC)
                    if f.startswith("fit_") and f.endswith(".hip") and f != "fit_wide.hip")
    assert tables, "no instance tables found"
    global_only = set()
    for f in tables:
        wl = _weight_sources(os.path.join(CSRC, f))
        assert wl and set(wl) <= {"true", "false"}, (f, wl)
        if set(wl) == {"false"}:
            global_only.add(f)
    assert global_only == set(build.GLOBAL_WEIGHT_SOURCES)
    assert set(build.GLOBAL_WEIGHT_SOURCES) <= set(build.SOURCES)


def test_unroll_flags_reach_only_those_files(monkeypatch):
    seen = {}

    class Done(Exception):
        pass

    def fake_run(cmd, **kw):
        src = os.path.basename(cmd[cmd.index("-c") + 1])
        seen[src] = " ".join(cmd)
        raise Done

    monkeypatch.setattr(build.subprocess, "run", fake_run)
    for src in ("fit_l3_wide_f32.hip", "fit_lds_bf16.hip", "fit_wide.hip", "fit_std.hip"):
        try:
            build._compile(src, verbose=False)
        except Done:
            pass
    flag = " ".join(build.UNROLL_FLAGS)
    assert flag in seen["fit_l3_wide_f32.hip"]
    for src in ("fit_lds_bf16.hip", "fit_wide.hip", "fit_std.hip"):
        assert flag not in seen[src], src
