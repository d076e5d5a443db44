"""The binding's ctypes structures have the header's layout (not gpu): a C program built
against include/vms.h prints sizeof and offsetof of every field the binding declares, and
both must agree field by field."""
import ctypes
import json
import os
import shutil
import subprocess

import pytest

from paper_0809_4802_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [(B.MeshDesc, "vms_mesh_desc"), (B.CreateOpts, "vms_create_opts"), (B.SolveOpts, "vms_solve_opts"),
         (B.SolveInfo, "vms_solve_info"), (B.NewtonOpts, "vms_newton_opts"), (B.NewtonInfo, "vms_newton_info")]


def test_structures_match_the_header(tmp_path):
    cc = shutil.which("gcc")
    if cc is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("gcc or the ROCm headers are not installed")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "vms.h"', "int main(void) {", 'printf("{");']
    for k, (py, c) in enumerate(PAIRS):
        sep = "," if k else ""
        lines.append(f'printf("{sep}\\"{c}\\": [%zu", sizeof({c}));')
        for name, _ in py._fields_:
            lines.append(f'printf(", %zu", offsetof({c}, {name}));')
        lines.append('printf("]");')
    lines += ['printf("}\\n");', "return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(src), "-o", str(exe)])
    got = json.loads(subprocess.check_output([str(exe)], text=True))
    for py, c in PAIRS:
        want = [ctypes.sizeof(py)] + [getattr(py, name).offset for name, _ in py._fields_]
        assert got[c] == want, (c, got[c], want)
