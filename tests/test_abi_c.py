"""The C header as a C compiler sees it (no GPU): every function the binding exports is
declared with a valid C prototype, and the layouts of the structs passed by pointer
(ltl_rule_t, ltl_tuning_t) match the ctypes structures of the binding field by field."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2406_17284_amd import ltl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM_INCLUDE = "/opt/rocm/include"

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or not os.path.isdir(ROCM_INCLUDE),
                                reason="needs gcc and the ROCm headers")


def compile_and_run(tmp_path, source):
    src = tmp_path / "probe.c"
    exe = tmp_path / "probe"
    src.write_text(source)
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror=implicit-function-declaration", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROOT, "include"), "-I", ROCM_INCLUDE, str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    return subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()


def test_struct_layouts_match_the_binding(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ltl.h"', "int main(void) {"]
    for cname, pystruct in (("ltl_rule_t", ltl.ltl_rule_t), ("ltl_tuning_t", ltl.ltl_tuning_t)):
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for field, _ in pystruct._fields_:
            lines.append(f'printf("{cname}.{field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["return 0; }"]
    out = compile_and_run(tmp_path, "\n".join(lines))
    got = dict(zip(out[0::2], (int(x) for x in out[1::2])))
    for cname, pystruct in (("ltl_rule_t", ltl.ltl_rule_t), ("ltl_tuning_t", ltl.ltl_tuning_t)):
        assert got[cname] == ctypes.sizeof(pystruct), cname
        for field, _ in pystruct._fields_:
            assert got[f"{cname}.{field}"] == getattr(pystruct, field).offset, f"{cname}.{field}"


def test_every_exported_function_has_a_c_prototype(tmp_path):
    """Taking each exported function's address compiles (as C, warnings as errors) only if
    the header declares it."""
    body = "\n".join(f"    p = (const void *)&{name}; (void)p;" for name in ltl.EXPORTS)
    src = tmp_path / "decl.c"
    src.write_text(f'#include "ltl.h"\nvoid probe(void);\nvoid probe(void) {{\n    const void *p;\n{body}\n}}\n')
    r = subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-fsyntax-only", "-D__HIP_PLATFORM_AMD__",
                        "-I", os.path.join(ROOT, "include"), "-I", ROCM_INCLUDE, str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
