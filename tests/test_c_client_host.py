"""The C ABI as C (no GPU): the public headers compile as strict C99 on their
own, and a C client that drives the library through them alone builds and
links against the in-tree library (tests/test_gpu_c_client.py runs it)."""
import os
import subprocess

from c_abi_client import ROOT, build_client


def test_headers_are_strict_c99(tmp_path):
    src = tmp_path / "h.c"
    src.write_text('#include "lb.h"\n#include "mlp.h"\nint main(void) { return (int)LB_OK; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I", os.path.join(ROOT, "include"), "-c", str(src), "-o", str(tmp_path / "h.o")],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr


def test_c_client_builds_and_links(tmp_path):
    exe = build_client(tmp_path)
    assert os.path.exists(exe)
