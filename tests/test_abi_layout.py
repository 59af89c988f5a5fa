"""The ctypes mirrors of the C-ABI structs match include/mgfwa.h, and the
oracle's match oracle/mgfwa_oracle.h (no GPU).

A small C program, compiled with the host compiler against the header, prints
sizeof and offsetof of every field; the binding's ctypes structures must agree,
so a field added on one side only fails here instead of corrupting arguments.
"""
import ctypes as C
import os
import subprocess

import pytest

from oracle import oracle as O
from paper_2501_03944_amd import mgfwa as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["mgfwa_problem", "mgfwa_config", "mgfwa_state_info", "mgfwa_timing_info",
           "mgfwa_plan_info", "mgfwa_job_info", "mgfwa_server_stats"]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mgfwa.h"', "int main(void) {"]
    for name in STRUCTS:
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in getattr(M, name)._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines))
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    layout = {}
    for line in out.splitlines():
        parts = line.split()
        layout[tuple(parts[:-1])] = int(parts[-1])
    return layout


@pytest.mark.parametrize("name", STRUCTS)
def test_ctypes_struct_matches_header(c_layout, name):
    cls = getattr(M, name)
    assert C.sizeof(cls) == c_layout[(name, "size")], name
    for field, _ in cls._fields_:
        assert getattr(cls, field).offset == c_layout[(name, field)], (name, field)


ORACLE = {"orc_problem": O._Problem, "orc_config": O._Config, "orc_view": O._View}


def test_oracle_ctypes_structs_match_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mgfwa_oracle.h"', "int main(void) {"]
    for name, cls in ORACLE.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            cfield = {"lam": "lambda"}.get(field, field)
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {cfield}));')
    lines += ["return 0;", "}"]
    src, exe = tmp_path / "olayout.c", tmp_path / "olayout"
    src.write_text("\n".join(lines))
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "oracle"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    layout = {tuple(l.split()[:-1]): int(l.split()[-1]) for l in out.splitlines()}
    for name, cls in ORACLE.items():
        assert C.sizeof(cls) == layout[(name, "size")], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == layout[(name, field)], (name, field)
