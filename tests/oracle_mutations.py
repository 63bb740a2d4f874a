"""Mutation check of the oracle's pins (CPU only; not collected by pytest).

Plants one plausible mistake at a time in a copy of ``oracle/oracle.c`` (a
dropped or flipped sign, a wrong index, an off-by-one test), builds the copy
in a temporary directory and runs ``tests/test_oracle_pins.py`` against it
through ``ORACLE_LIB``.  Every mutant must make at least one pin fail; the
repository's own oracle is never touched.

    python tests/oracle_mutations.py
"""
import os
import re
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (what the mistake is, pattern, replacement)
MUTANTS = [
    ("sign of an M entry", r"mv\[mlen\] = -c;", "mv[mlen] = c;"),
    ("sign of a new entry", r"aval\[lo\] = 0\.0 - t;", "aval[lo] = t;"),
    ("sign of a product in the solve", r"s = s \+ val\[p\] \* x\[j\];", "s = s - val[p] * x[j];"),
    ("in-stage test > for >=", r"if \(level\[k\] >= a\) \{", "if (level[k] > a) {"),
    ("diagonal of the wrong row", r"double c = aval\[p\] / diag\[j\];", "double c = aval[p] / diag[i];"),
    ("level off by one", r"if \(j < i && level\[j\] \+ 1 > lv\)", "if (j < i && level[j] > lv)"),
    ("stage depth test", r"candidate = width <= max_width && depth < max_depth;",
     "candidate = width <= max_width && depth <= max_depth;"),
    ("b index of a b-term", r"bi = bi \+ m_val\[p\] \* b\[m_col\[p\]\];", "bi = bi + m_val[p] * b[i];"),
    ("sign in the long-double solve", r"s = s \+ \(long double\)val\[p\] \* xl\[j\];",
     "s = s - (long double)val[p] * xl[j];"),
    ("diagonal test of the backward solve", r"if \(j > i\)\n", "if (j >= i)\n"),
    ("level-set counts shifted", r"level_ptr\[level\[i\] \+ 1\] \+= 1;", "level_ptr[level[i]] += 1;"),
    ("width rule < for <=", r"candidate = width <= max_width", "candidate = width < max_width"),
    ("fill budget < for <=", r"take = added \+ delta <= budget", "take = added + delta < budget"),
    ("b-terms left out of a level's entries", r"delta \+= nx \+ nb - ", "delta += nx - "),
    ("sign in the rewritten solve", r"s = s \+ lp_val\[p\] \* x\[k\];", "s = s - lp_val[p] * x[k];"),
]


def main() -> int:
    src = open(SRC).read()
    survived = 0
    with tempfile.TemporaryDirectory() as tmp:
        for what, pat, rep in MUTANTS:
            mutated, count = re.subn(pat, rep, src, count=1)
            if count != 1:
                print(f"NOT APPLIED ({what}): pattern not found")
                survived += 1
                continue
            c = os.path.join(tmp, "oracle.c")
            lib = os.path.join(tmp, "liboracle.so")
            with open(c, "w") as f:
                f.write(mutated)
            subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", c, "-o", lib,
                            "-lm"], check=True)
            r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                                "-x", "-q", "-p", "no:cacheprovider"],
                               env={**os.environ, "ORACLE_LIB": lib}, cwd=ROOT, capture_output=True, text=True)
            failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
            if r.returncode == 0:
                print(f"SURVIVED ({what})")
                survived += 1
            else:
                print(f"killed ({what}): {failed[0] if failed else r.stdout.strip().splitlines()[-1]}")
    return 1 if survived else 0


if __name__ == "__main__":
    sys.exit(main())
