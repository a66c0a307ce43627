"""The ctypes mirrors of the C ABI structs match the header's layout.

A small probe is compiled with the host C compiler against include/hfcr.h and
prints sizeof/offsetof of every struct field; the Python structs must agree.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_1409_2081_amd as hf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "hfcr_mesh": hf.Mesh,
    "hfcr_opts": hf.Opts,
    "hfcr_stats": hf.Stats,
    "hfcr_result": hf.Result,
    "hfcr_tuning": hf.Tuning,
    "hfcr_pair": hf.PairDesc,
    "hfcr_server_cfg": hf.ServerCfg,
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_struct_layouts_match_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hfcr.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            cname, field, val = line.split()
            got[(cname, field)] = int(val)
    for cname, py in STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
