"""The C-ABI library loads and exports every function include/cpf.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cpf.h")
LIB = os.path.join(ROOT, "paper_2309_09102_amd", "libcpf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cpf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("cpf_plan_init", "cpf_fk_batch", "cpf_dp_search", "cpf_lm_refine",
                     "cpf_submit", "cpf_poll", "cpf_ctx_create", "cpf_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcpf.so not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (same HIP runtime as the binding uses)
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcpf.so not built")
def test_binding_covers_every_export():
    from paper_2309_09102_amd import cpf
    assert set(cpf.EXPORTS) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcpf.so not built")
def test_opts_default_values():
    from paper_2309_09102_amd import cpf
    o = cpf.opts_default()
    assert (o.w_pose, o.w_smooth, o.lambda0, o.limit_penalty, o.refine_steps) == (1.0, 0.1, 1e-3, 10.0, 1)
    assert abs(o.limit_margin - 0.026179938779914945) < 1e-15


STRUCTS = ("cpf_robot", "cpf_problem", "cpf_opts", "cpf_lm_report", "cpf_result")
C_NAME = {"lambda_": "lambda"}   # Python keywords renamed in the binding


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcpf.so not built")
def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes mirror has the size and field offsets the C compiler gives
    the header's struct (a small C program compiled here prints them)."""
    import subprocess
    from paper_2309_09102_amd import cpf
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "cpf.h"', "int main(void) {"]
    for st in STRUCTS:
        lines.append(f'  printf("{st} size %zu\\n", sizeof({st}));')
        for name, _ in getattr(cpf, st)._fields_:
            lines.append(f'  printf("{st} {name} %zu\\n", offsetof({st}, {C_NAME.get(name, name)}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        st, key, val = line.split()
        got[(st, key)] = int(val)
    for st in STRUCTS:
        cls = getattr(cpf, st)
        assert got[(st, "size")] == ctypes.sizeof(cls), st
        for name, _ in cls._fields_:
            assert got[(st, name)] == getattr(cls, name).offset, (st, name)


def test_oracle_and_product_share_no_code():
    """The oracle neither includes nor imports the HIP path, and vice versa."""
    csrc = os.path.join(ROOT, "paper_2309_09102_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "oracle" not in text.lower(), f
    for f in ("cpf.py", "build.py", "synth.py", "__init__.py"):
        text = open(os.path.join(ROOT, "paper_2309_09102_amd", f)).read()
        assert "import oracle" not in text and "from oracle" not in text, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".py")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2309_09102_amd" not in text and "csrc" not in text, f


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: with --gpus 2 it exits with a message before
    touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
