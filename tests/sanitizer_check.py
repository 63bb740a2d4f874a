"""AddressSanitizer + UBSan check of the host code (CPU only; not collected
by pytest).

Builds, in a temporary directory, the library's host passes (analyse,
rewrite, pack, C ABI) and the oracle with -fsanitize=address,undefined
(g++ / gcc; the kernels are compiled as usual, since device code cannot be
sanitized here), links them with g++, and runs the CPU test suite
(-m "not gpu") against that build through SPTRSV_LIB and ORACLE_LIB with the
sanitizer runtimes preloaded into Python.  Any out-of-bounds access, use
after free, signed overflow, misaligned or out-of-range shift in the host
index arithmetic aborts the run.

    python tests/sanitizer_check.py [extra pytest args]
"""
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2103_11445_amd.build import CSRC, HIP_FLAGS, HIP_SOURCES, HOST_FLAGS, HOST_SOURCES, ROCM  # noqa: E402

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:
        sys.stderr.write(r.stdout[-4000:] + r.stderr[-4000:])
        raise SystemExit(f"failed: {' '.join(cmd[:3])} ...")
    return r


def main() -> int:
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        for src in HOST_SOURCES:
            o = os.path.join(tmp, src + ".o")
            run(["g++", *HOST_FLAGS, *SAN, "-c", os.path.join(CSRC, src), "-o", o])
            objs.append(o)
        for src in HIP_SOURCES:
            o = os.path.join(tmp, src + ".o")
            run([os.path.join(ROCM, "bin", "hipcc"), *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
            objs.append(o)
        lib = os.path.join(tmp, "libsptrsv.so")  # the C program test links -lsptrsv from its folder
        run(["g++", "-shared", "-fPIC", *SAN, "-o", lib, *objs, f"-L{ROCM}/lib", "-lamdhip64", "-lpthread",
             f"-Wl,-rpath,{ROCM}/lib"])
        olib = os.path.join(tmp, "liboracle_san.so")
        run(["gcc", "-O1", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", *SAN,
             os.path.join(ROOT, "oracle", "oracle.c"), "-o", olib, "-lm"])
        pre = [run(["gcc", f"-print-file-name={n}"]).stdout.strip() for n in ("libasan.so", "libubsan.so")]
        env = {**os.environ, "SPTRSV_LIB": lib, "ORACLE_LIB": olib, "LD_PRELOAD": ":".join(pre),
               "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:detect_odr_violation=0",
               "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}
        r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-x", "-q", "-m", "not gpu",
                            "-p", "no:cacheprovider", *sys.argv[1:]], env=env, cwd=ROOT)
        return r.returncode


if __name__ == "__main__":
    sys.exit(main())
