"""Mutation check of the library's host passes against the host tests (CPU
only; not collected by pytest).

Plants one plausible mistake at a time in a copy of a host source of the
library (levels, validation, the stage rule and its budgets, the elimination
that rewrites rows, the packer's choices, the byte counts), builds that
variant of ``libsptrsv.so`` in a temporary directory (the kernels are
compiled once and reused), and runs ``tests/test_capi_host.py`` against a
copy of the package that loads it.  Every mutant must make a host test fail
(they compare plans with the oracle bit for bit).  Mistakes that only change
the device image are caught by the GPU parity tests instead and are not
planted here.  The repository's own library is never touched.

    python tests/library_mutations.py
"""
import os
import re
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2103_11445_amd")
sys.path.insert(0, ROOT)
from paper_2103_11445_amd import build as B  # noqa: E402  (flags and source lists)

# (file, what the mistake is, pattern, replacement)
MUTANTS = [
    ("analyse.cpp", "level off by one", r"lv = std::max\(lv, p\.level\[\(size_t\)ci\[q\]\] \+ 1\);",
     "lv = std::max(lv, p.level[(size_t)ci[q]]);"),
    ("analyse.cpp", "zero diagonal accepted", r"if \(val\[e - 1\] == 0\.0\)", "if (val[e - 1] != val[e - 1])"),
    ("analyse.cpp", "level-set counts shifted", r"\+\+ptr\[\(size_t\)level\[i\] \+ 1\];", "++ptr[(size_t)level[i]];"),
    ("rewrite.cpp", "sign of an M entry", r"p\.m_val\[\(size_t\)\(mo \+ t\)\] = -c;", "p.m_val[(size_t)(mo + t)] = c;"),
    ("rewrite.cpp", "sign of an eliminated product", r"acc\[\(size_t\)k\] = acc\[\(size_t\)k\] - prod;",
     "acc[(size_t)k] = acc[(size_t)k] + prod;"),
    ("rewrite.cpp", "width rule < for <=", r"candidate = width <= pol\.max_width", "candidate = width < pol.max_width"),
    ("rewrite.cpp", "depth rule <= for <", r"width <= pol\.max_width && depth < pol\.max_depth;",
     "width <= pol.max_width && depth <= pol.max_depth;"),
    ("rewrite.cpp", "fill budget < for <=", r"take = added \+ delta <= budget", "take = added + delta < budget"),
    ("rewrite.cpp", "bit-set union drops a word of a dependency's set",
     r"for \(int32_t t = 0; t < sp\.uwords\[\(size_t\)u\]; \+\+t\) B\[t\] \|= S\[t\];",
     "for (int32_t t = 1; t < sp.uwords[(size_t)u]; ++t) B[t] |= S[t];"),
    ("rewrite.cpp", "closed stage not renumbered by row id",
     r"const int32_t r = rank\[\(size_t\)\(w \* 64 \+ __builtin_ctzll\(m\)\)\];",
     "const int32_t r = w * 64 + __builtin_ctzll(m);"),
    ("rewrite.cpp", "M's entries kept for the stage solve", r"const bool keep_m = p\.is_sub \|\| nm == 0 \|\| ",
     "const bool keep_m = true || "),
    ("pack.cpp", "8-chunk instance threshold", r"longer \+= T\.nch > 4 \? 1 : -1;", "longer += T.nch > 8 ? 1 : -1;"),
    ("pack.cpp", "one-level stages as segments", r"ok && depth >= 2 &&", "ok && depth >= 1 &&"),
    ("capi.cpp", "bytes of the M pass", r"o->bytes_rw \+= 2 \* vb \* \(int64_t\)p\.n;", "o->bytes_rw += vb * (int64_t)p.n;"),
]


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{r.stdout}{r.stderr}")
    return r


def main() -> int:
    hipcc = os.path.join(B.ROCM, "bin", "hipcc")
    survived = 0
    with tempfile.TemporaryDirectory() as tmp:
        csrc = os.path.join(tmp, "csrc")
        shutil.copytree(B.CSRC, csrc)
        objs = {}
        for src in B.HIP_SOURCES:
            objs[src] = os.path.join(tmp, src + ".o")
            run([hipcc, *B.HIP_FLAGS, "-c", os.path.join(csrc, src), "-o", objs[src]])
        for src in B.HOST_SOURCES:
            objs[src] = os.path.join(tmp, src + ".o")
            run(["g++", *B.HOST_FLAGS, "-c", os.path.join(csrc, src), "-o", objs[src]])
        # a copy of the package (Python files, trained model) that loads the variant
        pkg_root = os.path.join(tmp, "pkg")
        pkg = os.path.join(pkg_root, "paper_2103_11445_amd")
        os.makedirs(pkg)
        for f in os.listdir(PKG):
            if f.endswith(".py") or f.endswith(".npz"):
                shutil.copy(os.path.join(PKG, f), pkg)
        for fname, what, pat, rep in MUTANTS:
            orig = open(os.path.join(B.CSRC, fname)).read()
            mutated, count = re.subn(pat, rep, orig, count=1)
            if count != 1:
                print(f"NOT APPLIED ({fname}: {what})")
                survived += 1
                continue
            with open(os.path.join(csrc, fname), "w") as f:
                f.write(mutated)
            mobj = os.path.join(tmp, "mutant.o")
            run(["g++", *B.HOST_FLAGS, "-c", os.path.join(csrc, fname), "-o", mobj])
            link = [mobj if k == fname else objs[k] for k in B.HOST_SOURCES + B.HIP_SOURCES]
            run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", os.path.join(pkg, "libsptrsv.so"),
                 *link, "-lpthread"])
            with open(os.path.join(csrc, fname), "w") as f:
                f.write(orig)
            # (python -m puts the working directory first on the path)
            r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_capi_host.py"),
                                "-x", "-q", "-p", "no:cacheprovider"], cwd=pkg_root, capture_output=True, text=True,
                               env={**os.environ, "PYTHONPATH": pkg_root + os.pathsep + ROOT})
            failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
            if r.returncode == 0:
                print(f"SURVIVED ({fname}: {what})")
                survived += 1
            else:
                print(f"killed ({fname}: {what}): {failed[0] if failed else r.stdout.strip().splitlines()[-1]}")
    return 1 if survived else 0


if __name__ == "__main__":
    sys.exit(main())
