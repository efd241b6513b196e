"""The ctypes structures of the binding have the layout of the C header's structures: each
size and each field offset, as a C compiler lays out include/rpf.h.  CPU only (gcc)."""

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1812_11689_amd import rpf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# binding structure -> C typedef
PAIRS = [(rpf.Params, "rpf_params"), (rpf.Info, "rpf_info"), (rpf.BatchEntry, "rpf_batch_entry"),
         (rpf.KnnStats, "rpf_knn_stats"), (rpf.ProfileRecord, "rpf_profile_record"),
         (rpf.ServerConfig, "rpf_server_config"), (rpf.ServerStats, "rpf_server_report"),
         (rpf.PlanEntry, "rpf_plan_entry"), (rpf.PlanPartInfo, "rpf_plan_part_info"),
         (rpf.ServerBatch, "rpf_server_batch"), (rpf.Node, "rpf_node")]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_binding_structures_match_the_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rpf.h"', "int main(void) {"]
    expect = []
    for py, c in PAIRS:
        lines.append(f'    printf("%zu\\n", sizeof({c}));')
        expect.append(ctypes.sizeof(py))
        for name, _ in py._fields_:
            lines.append(f'    printf("%zu\\n", offsetof({c}, {name}));')
            expect.append(getattr(py, name).offset)
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True, capture_output=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect
