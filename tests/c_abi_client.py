"""Builds tests/c_client/lb_client.c (a plain C client of the library) with
gcc: C11, -pedantic -Werror on the library's headers (HIP's own headers are
included as system headers), linked against the in-tree liblbmi.so."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SRC = os.path.join(ROOT, "tests", "c_client", "lb_client.c")
LIBDIR = os.path.join(ROOT, "paper_1004_5058_amd", "_lib")


def build_client(out_dir):
    exe = os.path.join(str(out_dir), "lb_client")
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-pedantic", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-isystem", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"), SRC,
           "-L", LIBDIR, "-llbmi", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + LIBDIR, "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        raise RuntimeError("building the C client failed:\n" + r.stderr)
    return exe
