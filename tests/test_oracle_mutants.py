"""Strength of the oracle's pins: copies of the oracle's C source with one
planted mistake each (the kind a transcription of the method could make) are
compiled on the CPU, and the pin named beside each mistake must fail on that
copy.  The same pins pass on the real oracle in the rest of the suite."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "smc_oracle.c")

# (mistake, original text, planted text, pin that must catch it)
MUTANTS = [
    ("homodimer count without the -1 (Sec. 2.2)",
     "double pairs = (xa * (double)(x[ra] - 1)) * 0.5;",
     "double pairs = (xa * (double)(x[ra])) * 0.5;",
     "tests/test_oracle_ssa.py::test_bimolecular_against_master_equation[homodimer]"),
    ("holding time at twice the rate (eq. 2a)",
     "double tau = (-oracle_log(u1)) / a0;",
     "double tau = (-oracle_log(u1)) / (2.0 * a0);",
     "tests/test_oracle_ssa.py::test_immigration_death_poisson[5.0]"),
    ("channel chosen with the holding-time uniform (eq. 2b)",
     "double target = u2 * a0;",
     "double target = u1 * a0;",
     "tests/test_oracle_ssa.py::test_immigration_death_poisson[5.0]"),
    ("state change applied with the wrong sign",
     "if (s >= 0) x[s] += n->chg_val[4 * jsel + q];",
     "if (s >= 0) x[s] -= n->chg_val[4 * jsel + q];",
     "tests/test_oracle_ssa.py::test_immigration_death_poisson[5.0]"),
    ("Philox key schedule constant",
     "k0 += 0x9E3779B9u;",
     "k0 += 0x9E3779B8u;",
     "tests/test_oracle_primitives.py::test_philox_matches_rocrand"),
    ("u1 drawn from [0, 1) instead of (0, 1]",
     "return (double)(v + 1u) * 0x1p-53;",
     "return (double)v * 0x1p-53;",
     "tests/test_oracle_primitives.py::test_uniform_conversions_exact"),
    ("ln: exponent not raised when the mantissa is halved",
     "if (m > sqrt2) { m = m * 0.5; e = e + 1; }",
     "if (m > sqrt2) { m = m * 0.5; }",
     "tests/test_oracle_primitives.py::test_log_within_one_ulp"),
    ("until measured in absolute instead of relative time (Sec. 3.1)",
     "double d = P->t[j] - P->t[i];",
     "double d = P->t[j];",
     "tests/test_oracle_semantics.py::test_golden_trace[A:F[0,10](G[0,1.6](X>=1))]"),
    ("negation dropped (G as not F not, Sec. 3.1)",
     "static int not3(int v) { return v == V_U ? V_U : (v == V_T ? V_F : V_T); }",
     "static int not3(int v) { return v; }",
     "tests/test_oracle_semantics.py::test_golden_trace[A:G[0,3](X<=2)]"),
    ("until's right operand accepted without the left one holding before it",
     "if (d >= lo) res = or3(res, and3(all1, eval3(f, f->b[node], j, P)));",
     "if (d >= lo) res = or3(res, eval3(f, f->b[node], j, P));",
     "tests/test_oracle_semantics.py::test_golden_trace[A:(F[0,10](X>=3)) U[0,10] (X>=1)]"),
]


@pytest.mark.parametrize("mistake,orig,planted,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(tmp_path, mistake, orig, planted, pin):
    text = open(SRC).read()
    assert text.count(orig) == 1, "the oracle source no longer has this text"
    src = tmp_path / "mutant.c"
    lib = tmp_path / "mutant.so"
    src.write_text(text.replace(orig, planted))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-pthread", str(src), "-o", str(lib), "-lm"])
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", pin], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    # exit code 1: the pin ran and failed (2 and above: it did not run)
    assert r.returncode == 1, (mistake, r.returncode, r.stdout[-2000:])
