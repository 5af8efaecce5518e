"""Strength of the oracle's pins: copies of the oracle with one planted
mistake each (the kind a transcription of the method could make), and the pin
named beside each mistake must fail on that copy.  C mistakes are compiled
into a separate library on the CPU; Wilson-rule mistakes are loaded as a
separate module.  The same pins pass on the real oracle."""
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
    ("model id in counter word 3 instead of 2",
     "uint32_t ctr[4] = {k, (uint32_t)idx, model_id, 0u};",
     "uint32_t ctr[4] = {k, (uint32_t)idx, 0u, model_id};",
     "tests/test_oracle_primitives.py::test_first_event_follows_the_stream_contract"),
    ("seed halves swapped in the key",
     "uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};",
     "uint32_t key[2] = {(uint32_t)(seed >> 32), (uint32_t)seed};",
     "tests/test_oracle_primitives.py::test_first_event_follows_the_stream_contract"),
    ("state sampled at 2T instead of T",
     "if (tn > T) break;", "if (tn > 2.0 * T) break;",
     "tests/test_oracle_ssa.py::test_isomerization_binomial[0.3]"),
    ("arithmetic predicate: subtraction operands swapped",
     "case E_SUB: sp--; st[sp - 1] = st[sp - 1] - st[sp]; break;",
     "case E_SUB: sp--; st[sp - 1] = st[sp] - st[sp - 1]; break;",
     "tests/test_oracle_semantics.py::test_golden_trace[B:(A > B) U[0,5] (B - A >= 1)]"),
    ("<= evaluated as <",
     "case OP_LE: return l <= r;", "case OP_LE: return l < r;",
     "tests/test_oracle_semantics.py::test_golden_trace[A:G[0,3](X<=2)]"),
    ("next operator measured in absolute time",
     "        double d = P->t[i + 1] - P->t[i];\n        if (!(d >= lo && d <= hi)) return V_F;\n        return eval3",
     "        double d = P->t[i + 1];\n        if (!(d >= lo && d <= hi)) return V_F;\n        return eval3",
     "tests/test_oracle_semantics.py::test_golden_trace[A:F[0,10](X[0,2](X>=3))]"),
    ("absorption reported as a time decision",
     "        else if (isinf(w->t[m + 1])) *reason = R_ABSORB;\n", "",
     "tests/test_oracle_semantics.py::test_driver_matches_brute_force[death_only-F[0,100](X>=40)-0]"),
    ("event cap one event early",
     "(uint64_t)m == (uint64_t)pr->max_events", "(uint64_t)m + 1 == (uint64_t)pr->max_events",
     "tests/test_oracle_semantics.py::test_tmax_pessimistic_rule_and_cap"),
    ("until skip: the window is not checked over the skipped positions",
     "        if (nj > j + 1 && P->t[nj - 1] - P->t[i] > hi) break;\n", "",
     "tests/test_oracle_semantics.py::test_skip_scan_equals_plain_scan"),
    ("until skip: a position where the right operand holds counted as neutral",
     "int neutral = eval3(f, f->a[node], k, P) == V_T && eval3(f, f->b[node], k, P) == V_F;",
     "int neutral = eval3(f, f->a[node], k, P) == V_T && eval3(f, f->b[node], k, P) != V_U;",
     "tests/test_oracle_semantics.py::test_skip_scan_equals_plain_scan"),
    ("until's right operand accepted without the left one holding before it",
     "if (d >= lo) res = or3(res, and3(all1, eval3(f, f->b[node], j, P)));",
     "if (d >= lo) res = or3(res, eval3(f, f->b[node], j, P));",
     "tests/test_oracle_semantics.py::test_golden_trace[A:(F[0,10](X>=3)) U[0,10] (X>=1)]"),
    ("pow: exponent bits taken least significant first",
     "if ((k >> b) & 1) r = r * x;",
     "if ((k >> (6 - b)) & 1) r = r * x;",
     "tests/test_oracle_pow.py::test_integer_powers_are_exact[2]"),
    ("pow: a plain left-to-right product instead of binary powering",
     "        double r = 1.0;\n        for (int b = 6; b >= 0; --b) {",
     "        double r = 1.0;\n        for (int i = 0; i < k; ++i) r = r * x;\n        return r;\n        for (int b = 6; b >= 0; --b) {",
     "tests/test_oracle_pow.py::test_multiplication_order_is_binary_powering[4]"),
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


# The Wilson rule (Sec. 3.3, eqs. 3-4, Fig. 2) lives in oracle/wilson.py: its
# mutants are loaded as modules and the pins are called with them in place.
WILSON_MUTANTS = [
    ("eq. 3 centre without z^2/2n",
     "center = p + z2 / (2.0 * nd)", "center = p",
     "test_table3_intervals"),
    ("eq. 3 half-width with z^2/4n instead of z^2/4n^2",
     "z2 / ((4.0 * nd) * nd)", "z2 / (4.0 * nd)",
     "test_table3_intervals"),
    ("eq. 4 with the sign of 2 eps^2 flipped",
     "num = (pq - 2.0 * e2) + math.sqrt(rad)", "num = (pq + 2.0 * e2) + math.sqrt(rad)",
     "test_conservative_sample_size"),
    ("sample size rounded to nearest instead of up",
     "return int(math.ceil(wilson_sample_value(p, eps, z)))", "return int(round(wilson_sample_value(p, eps, z)))",
     "test_first_batch_closed_form"),
    ("Fig. 2 moves the estimate away from 0.5",
     "        q = p + eps\n", "        q = p - eps\n",
     "test_rounding_towards_half"),
    ("z as sqrt(2) erfinv((1 + confidence) / 2), mixing two quantile forms",
     "mpmath.erfinv(mpmath.mpf(confidence))", "mpmath.erfinv(mpmath.mpf((1 + confidence) / 2))",
     "test_z_values"),
    ("Fig. 2 runs N' more trajectories instead of N' - N_tot",
     "n_new = n_prime - n_tot", "n_new = n_prime",
     "test_all_false_stream_95"),
    ("p-hat from the last batch only, not all batches so far",
     "yes += count_yes(n_tot, n_tot + n_run)", "yes = count_yes(n_tot, n_tot + n_run)",
     "test_iterative_reduction_claim"),
    ("first batch sized for p = 0.5 unless asked, and vice versa",
     "n_run = wilson_sample(0.5 if conservative else 1.0, eps, z)",
     "n_run = wilson_sample(1.0 if conservative else 0.5, eps, z)",
     "test_iterative_reduction_claim"),
]


@pytest.mark.parametrize("mistake,orig,planted,pin", WILSON_MUTANTS, ids=[m[0] for m in WILSON_MUTANTS])
def test_wilson_pin_catches_planted_mistake(monkeypatch, golden_dir, mistake, orig, planted, pin):
    import inspect
    import types

    import test_oracle_wilson as pins
    from oracle import wilson

    text = open(wilson.__file__).read()
    assert text.count(orig) == 1, "the Wilson oracle no longer has this text"
    mutant = types.ModuleType("wilson_mutant")
    exec(compile(text.replace(orig, planted), "wilson_mutant.py", "exec"), mutant.__dict__)
    monkeypatch.setattr(pins, "wilson", mutant)
    fn = getattr(pins, pin)
    args = [golden_dir] if "golden_dir" in inspect.signature(fn).parameters else []
    with pytest.raises(Exception):
        fn(*args)
    monkeypatch.undo()
    fn(*args)      # the same pin passes with the real oracle


# The MLP oracle (oracle/mlp.py), the BLTLc parser (oracle/bltlc.py) and the
# exact transient probabilities (oracle/uniformization.py), the same way.  A
# pin given as "module:function[:argument]" is called once; as
# "module:golden" it runs every hand-derived golden trace case.
PY_MUTANTS = [
    ("mlp", "layer-2 ReLU derivative dropped",
     '* (f["pre2"] > 0.0)', "",
     "test_oracle_mlp:test_exact_gradients_against_finite_differences"),
    ("mlp", "dW2 transposed",
     'dW2 = d2b.T @ f["h1"]', 'dW2 = f["h1"].T @ d2b',
     "test_oracle_mlp:test_exact_gradients_against_finite_differences"),
    ("mlp", "cross-entropy gradient with the wrong sign",
     "dz = w * (p - y) / wsum", "dz = w * (y - p) / wsum",
     "test_oracle_mlp:test_exact_gradients_against_finite_differences"),
    ("mlp", "bfloat16 by truncation instead of ties-to-even",
     "np.rint(np.ldexp(m, 8))", "np.trunc(np.ldexp(m, 8))",
     "test_oracle_mlp:test_bf16_rounding"),
    ("mlp", "Adam without the bias corrections",
     "m_hat = m / (1.0 - beta1 ** t)", "m_hat = m",
     "test_oracle_mlp:test_adam_first_step_and_constant_gradient"),
    ("mlp", "Adam second moment from g instead of g^2",
     "(1.0 - beta2) * (g * g)", "(1.0 - beta2) * np.abs(g)",
     "test_oracle_mlp:test_adam_two_steps_by_hand"),
    ("bltlc", "G rewritten without the inner negation (G p as not F p)",
     "neg = self.f.node(N_NOT, arg)", "neg = arg",
     "test_oracle_semantics:golden"),
    ("bltlc", "| parsed as &",
     "left = self.f.node(N_OR, left, right)", "left = self.f.node(N_AND, left, right)",
     "test_oracle_semantics:golden"),
    ("uniformization", "Poisson weights with (k-1)! instead of k!",
     "- lam - gammaln(k + 1))", "- lam - gammaln(k))",
     "test_oracle_probability:test_c1_against_uniformization"),
    ("uniformization", "master-equation homodimer rate without the -1",
     "return c * x[ra] * (x[ra] - 1) / 2.0", "return c * x[ra] * x[ra] / 2.0",
     "test_oracle_ssa:test_bimolecular_against_master_equation:homodimer"),
    ("uniformization", "until: paths where the left operand fails not stopped",
     "absorbing = lambda x: p2(x) or not p1(x)", "absorbing = lambda x: p2(x)",
     "test_oracle_probability:test_until_two_independent_species"),
]


@pytest.mark.parametrize("module,mistake,orig,planted,pin", PY_MUTANTS, ids=[m[1] for m in PY_MUTANTS])
def test_python_oracle_pin_catches_planted_mistake(monkeypatch, module, mistake, orig, planted, pin):
    import importlib
    import types

    real = importlib.import_module("oracle." + module)
    pins_name, fn_name, *args = pin.split(":")
    pins = importlib.import_module(pins_name)
    attr = next(k for k, v in vars(pins).items() if v is real)      # the name the pins use
    text = open(real.__file__).read()
    assert text.count(orig) == 1, "the oracle module no longer has this text"
    mutant = types.ModuleType(module + "_mutant")
    monkeypatch.setitem(sys.modules, mutant.__name__, mutant)     # dataclasses look their module up
    exec(compile(text.replace(orig, planted), module + "_mutant.py", "exec"), mutant.__dict__)

    def run():
        if fn_name == "golden":
            failed = 0
            for case in pins._golden():
                try:
                    pins.test_golden_trace(*case.values)
                except AssertionError:
                    failed += 1
            assert failed == 0, f"{failed} golden cases fail"
        else:
            getattr(pins, fn_name)(*args)

    monkeypatch.setattr(pins, attr, mutant)
    with pytest.raises(AssertionError):
        run()
    monkeypatch.undo()
    run()          # the same pins pass with the real oracle
