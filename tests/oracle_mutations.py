"""Mutation check of the oracle's pins (CPU only; not collected by pytest).

Plants one plausible mistake at a time in a copy of ``oracle/oracle.c`` (a
dropped or flipped sign, a wrong index, an off-by-one test), builds the copy
in a temporary directory and runs ``tests/test_oracle_pins.py`` against it
through ``ORACLE_LIB``; likewise for the cost model's ``oracle/mlp.py`` (a
copy of the package first on the path) against ``tests/test_oracle_mlp.py``,
and for the package's own Python (the FLOP count) against the pins.
Every mutant must make at least one pin fail; the repository's own oracle is
never touched.

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
    ("sign in the long-double solve", r"s = s \+ \(ext_t\)val\[p\] \* xl\[j\];",
     "s = s - (ext_t)val[p] * xl[j];"),
    ("extended solve carried in double", r"typedef long double ext_t;", "typedef double ext_t;"),
    ("diagonal test of the backward solve", r"if \(j > i\)\n", "if (j >= i)\n"),
    ("level-set counts shifted", r"level_ptr\[level\[i\] \+ 1\] \+= 1;", "level_ptr[level[i]] += 1;"),
    ("width rule < for <=", r"candidate = width <= max_width", "candidate = width < max_width"),
    ("fill budget < for <=", r"take = added \+ delta <= budget", "take = added + delta < budget"),
    ("b-terms left out of a level's entries", r"delta \+= nx \+ nb - ", "delta += nx - "),
    ("sign in the rewritten solve", r"s = s \+ lp_val\[p\] \* x\[k\];", "s = s - lp_val[p] * x[k];"),
    ("level-set solve skips the last level",
     r"for \(int l = 0; l < nlev; \+\+l\) \{\n(\s*)/\* the implicit barrier",
     "for (int l = 0; l + 1 < nlev; ++l) {\n\\1/* the implicit barrier"),
    ("b-terms dropped in the level-set solve", r"(double bi = b\[i\];\n(\s*)for \(int64_t p = m_ptr\[i\]; p < m_ptr\[i \+ 1\]; \+\+p\)\n\s*bi = bi \+ m_val\[p\] \* b\[m_col\[p\]\];)(?![\s\S]*oracle_solve_rewritten)",
     "double bi = b[i];"),
]


# mistakes in the cost model's oracle (oracle/mlp.py), checked by
# tests/test_oracle_mlp.py against a copy of the package placed first on the path
MLP_MUTANTS = [
    ("tanh derivative sign", r"\(1\.0 - h2 \*\* 2\)", "(1.0 + h2 ** 2)"),
    ("factor 2 of the squared error", r"g = 2\.0 \* \(y - t\) / m", "g = (y - t) / m"),
    ("bias gradient averaged", r'"b1": d1\.sum\(axis=0\)', '"b1": d1.mean(axis=0)'),
    ("first-layer gradient transposed", r'"W1": d1\.T @ X', '"W1": (X.T @ d1).T.reshape(X.shape[1], -1).T'),
    ("Adam without bias correction", r"mh = m1 / \(1\.0 - beta1 \*\* step\)", "mh = m1"),
    ("output bias dropped", r"return h2 @ q\[\"w3\"\] \+ q\[\"b3\"\]\[0\]", "return h2 @ q[\"w3\"]"),
]


# mistakes in the oracle's Python side (oracle/__init__.py), checked by
# tests/test_oracle_pins.py against a copy of the package placed first on the path
INIT_MUTANTS = [
    ("b-terms counted once in the FLOPs", r"return 2 \* \(off \+ nm\) \+ n", "return 2 * off + nm + n"),
    ("divisions left out of the FLOPs", r"return 2 \* \(off \+ nm\) \+ n", "return 2 * (off + nm)"),
]


def run_pins(test_file, env, cwd=ROOT):
    # (python -m puts the working directory first on the path: a mutated
    # package copy is found first only when the run starts in its directory)
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", test_file), "-x", "-q",
                        "-p", "no:cacheprovider"], env={**os.environ, **env}, cwd=cwd, capture_output=True, text=True)
    failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return r.returncode, (failed[0] if failed else (r.stdout.strip().splitlines() or [""])[-1])


def main() -> int:
    src = open(SRC).read()
    survived = 0
    with tempfile.TemporaryDirectory() as tmp:
        mlp_src = open(os.path.join(ROOT, "oracle", "mlp.py")).read()
        pkg = os.path.join(tmp, "oracle")
        os.makedirs(pkg)
        with open(os.path.join(pkg, "__init__.py"), "w") as f:
            f.write(open(os.path.join(ROOT, "oracle", "__init__.py")).read())
        lib_real = os.path.join(ROOT, "oracle", "liboracle.so")
        for what, pat, rep in MLP_MUTANTS:
            mutated, count = re.subn(pat, rep, mlp_src, count=1)
            if count != 1:
                print(f"NOT APPLIED ({what}): pattern not found")
                survived += 1
                continue
            with open(os.path.join(pkg, "mlp.py"), "w") as f:
                f.write(mutated)
            rc, msg = run_pins("test_oracle_mlp.py", {"PYTHONPATH": tmp + os.pathsep + ROOT, "ORACLE_LIB": lib_real},
                               cwd=tmp)
            if rc == 0:
                print(f"SURVIVED ({what})")
                survived += 1
            else:
                print(f"killed ({what}): {msg}")
        with open(os.path.join(pkg, "mlp.py"), "w") as f:
            f.write(mlp_src)
        init_src = open(os.path.join(ROOT, "oracle", "__init__.py")).read()
        for what, pat, rep in INIT_MUTANTS:
            mutated, count = re.subn(pat, rep, init_src, count=1)
            if count != 1:
                print(f"NOT APPLIED ({what}): pattern not found")
                survived += 1
                continue
            with open(os.path.join(pkg, "__init__.py"), "w") as f:
                f.write(mutated)
            rc, msg = run_pins("test_oracle_pins.py", {"PYTHONPATH": tmp + os.pathsep + ROOT,
                                                       "ORACLE_LIB": lib_real}, cwd=tmp)
            if rc == 0:
                print(f"SURVIVED ({what})")
                survived += 1
            else:
                print(f"killed ({what}): {msg}")
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
            subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", c,
                            "-o", lib, "-lm"], check=True)
            rc, msg = run_pins("test_oracle_pins.py", {"ORACLE_LIB": lib})
            if rc == 0:
                print(f"SURVIVED ({what})")
                survived += 1
            else:
                print(f"killed ({what}): {msg}")
    return 1 if survived else 0


if __name__ == "__main__":
    sys.exit(main())
