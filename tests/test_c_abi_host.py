"""The C ABI from a C program (no GPU): tests/c_abi_host.c includes the
header as C11 with warnings as errors, links against the built library and
checks a rewritten chain against its closed form."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sp():
    import paper_2103_11445_amd as m
    m.load()
    return m


def test_c_program_against_the_library(tmp_path, sp):
    lib_dir = os.path.dirname(sp.library_path())
    exe = str(tmp_path / "c_abi_host")
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c_abi_host.c"),
                    "-L" + lib_dir, "-lsptrsv", "-Wl,-rpath," + lib_dir, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
