"""The library's formula compiler on the host (no GPU): which BLTLc forms the
GPU monitor runs, which it refuses, and the time horizon it derives, checked
against the oracle's parser and horizon."""
import math

import pytest

import oracle
from oracle import bltlc
from paper_0912_2551_amd import binding as B

NAMES = ["X", "Y", "Z"]

ACCEPTED = [
    "X >= 3",                                           # a predicate on the initial state
    "F[0,10](X>=3) & G[2,8](Y<=4) | !(Z=1)",            # bounded F, G with lower bounds, boolean combination
    "(X<=2) U[1,5] (Y>=3)",                             # until with a lower bound
    "X[0,0.5](X + 2*Y >= Z - 1)",                       # next, integer linear predicate
    "F[0,2](X*X <= sqrt(Y*400) + 3)",                   # arithmetic predicate
    "F(X>=100)",                                        # unbounded (needs t_max or a cap at run time)
    "(X<=6) U[0,4] ((Y>=2) U[0,1.5] (Z>=5))",           # nested until
    "(X<=6) U[2,4] F[0,1](Z>=5)",                       # nested until with F inside, outer lower bound
    "F[1,3]((Y>=2) U[0,1] (Z>=5))",                     # nested until as F I (q U r)
    "G[0,20](X<=5 | F[0,2](Y>=1))",                     # response
    "G[1,20]((F[0,2](Y>=1)) | X<=5)",                   # response, operands swapped
    "G[0,20](F[0,2](Y>=1))",                            # response without p
    "F[0,30]((X>=5) & G[0,2](Y<=1))",                   # persistence (the response's dual)
    "F[0,30](G[0,3](X>=5))",                            # persistence without p
    "X[0,1]((X>=1) U[0,2] (Y>=2))",                     # X over an until
    "X[0,1](F[1,2](Y>=2)) | X[0,0.5](G[0,1](Z<=3))",    # X over F and G
    "(X<=9) U[0,5] G[0,2](Y>=1)",                       # until over G
    "(X<=9) U[0,5] ((Z>=1) & G[0,2](Y>=1))",            # until over a conjunction with G
    "(X<=9) U[0,5] (G[0,2](Y>=1) & Z>=1)",
    "F[0,1](pow(X,2) + pow(Y/3,13) >= pow(Z,0) + pow(X,64))",   # pow with constant integral exponents
]

# outside the compact monitors: trace programs (accepted)
TRACE = [
    "F[0,10](G[1,2](X>1))",                  # inner window not starting at 0
    "G[0,10](X<=5 | F[1,2](Y>=1))",
    "X[0,1](X[0,1](X>1))",                   # X over X
    "(F[0,1](X>1)) U[0,5] (Y>1)",            # temporal left operand of U
    "F[0,1](F[0,1](F[0,1](X>1)))",           # nesting three levels deep
    "G[0,1](F[0,1](X>1)) & G[0,1](F[0,1](Y>1)) & G[0,1](F[0,1](Z>1))",   # three time registers
    "F(G[0,2](X>=3))",                       # unbounded outer window (needs t_max or a cap at run time)
    "(X>=1 & Y>=1 & Z>=1 & X+Y>=2 & Y+Z>=2 & X+Z>=4) U[0,3] (Y<=0)",   # six predicates in one state formula
]

UNSUPPORTED = [
    "F[0,1](pow(X,0.5)>1)",                  # pow: only constant integral exponents 0..64
    "F[0,1](pow(X,Y)>1)",
    "F[0,1](pow(X,-2)>1)",
    "F[0,1](pow(X,65)>1)",
    " | ".join(f"F[0,1](X>={i})" for i in range(17)),             # more than 16 predicates
    "F[0,1](" + " & ".join(f"G[0,{i + 1}](X>=1)" for i in range(7)) + ")",   # trace program over 32 nodes
]

PARSE_ERRORS = [
    "F[0,1](W>1)",          # unknown species
    "F[2,1](X>1)",          # empty interval
    "F[0,1](X>1",           # unbalanced parenthesis
    "X >> 1",
]


@pytest.mark.parametrize("text", ACCEPTED)
def test_accepted_with_the_oracles_horizon(text):
    rc, msg, hz = B.formula_check(text, NAMES)
    assert rc == B.SMC_OK, msg
    exp = oracle.horizon(bltlc.parse(text, NAMES))
    assert hz == exp or (math.isinf(hz) and math.isinf(exp))


@pytest.mark.parametrize("text", TRACE)
def test_trace_programs_with_the_oracles_horizon(text):
    rc, msg, hz = B.formula_check(text, NAMES)
    assert rc == B.SMC_OK, msg
    exp = oracle.horizon(bltlc.parse(text, NAMES))
    assert hz == exp or (math.isinf(hz) and math.isinf(exp))


@pytest.mark.parametrize("text", UNSUPPORTED)
def test_outside_the_gpu_classes(text):
    rc, msg, hz = B.formula_check(text, NAMES)
    assert rc == B.SMC_E_UNSUPPORTED, (rc, msg)
    assert msg and hz is None
    bltlc.parse(text, NAMES)     # the oracle evaluates every form


@pytest.mark.parametrize("text", PARSE_ERRORS)
def test_parse_errors_agree_with_the_oracle(text):
    rc, msg, _ = B.formula_check(text, NAMES)
    assert rc == B.SMC_E_PARSE, (rc, msg)
    with pytest.raises(bltlc.ParseError):
        bltlc.parse(text, NAMES)


def test_bad_arguments_and_message_truncation():
    L = B.lib()
    assert L.smc_formula_check(None, None, 0, None, None, 0) == B.SMC_E_INVALID
    import ctypes
    arr = (ctypes.c_char_p * 1)(b"X")
    buf = ctypes.create_string_buffer(8)
    rc = L.smc_formula_check(b"F[0,1](Q>1)", arr, 1, None, buf, 8)
    assert rc == B.SMC_E_PARSE and len(buf.value) == 7


def _random_formula(r, depth=0):
    """Random BLTLc text over X, Y and a species named F (Sec. 3.1 grammar)."""
    def interval():
        k = r.random()
        if k < 0.4:
            a = round(r.uniform(0, 3), 2)
            return f"[{a},{round(a + r.uniform(0, 4), 2)}]"
        if k < 0.7:
            return f"<={round(r.uniform(0, 5), 2)}"
        return "" if k < 0.8 else "[0,inf]"

    def val(d):
        k = r.random()
        if d > 1 or k < 0.4:
            return r.choice(["X", "Y", "F", "2", "3.5", "0"])
        if k < 0.6:
            return f"{val(d + 1)} {r.choice('+-*/')} {val(d + 1)}"
        if k < 0.7:
            return f"sqrt({val(d + 1)})"
        return f"-{val(d + 1)}" if k < 0.8 else f"({val(d + 1)})"

    k = r.random()
    if depth > 3 or k < 0.3:
        if r.random() < 0.9:
            return f"{val(0)} {r.choice(['<', '<=', '>=', '>', '=', '!=', '=='])} {val(0)}"
        return r.choice(["true", "false"])
    sub = lambda: _random_formula(r, depth + 1)   # noqa: E731
    if k < 0.4:
        return f"!{sub()}"
    if k < 0.5:
        return f"{sub()} & {sub()}"
    if k < 0.6:
        return f"{sub()} | {sub()}"
    if k < 0.75:
        return f"{r.choice('FGX')}{interval()} {sub()}"
    if k < 0.85:
        return f"{sub()} U{interval()} {sub()}"
    return f"({sub()})"


def test_random_formulas_read_alike():
    """The library's parser and the oracle's parser are separate code: on
    random text they must reject the same formulas, and on every formula the
    library accepts they must derive the same horizon (which depends on how
    the operators nest)."""
    import random
    r = random.Random(7)
    names = ["X", "Y", "F"]
    codes = {}
    for _ in range(2000):
        text = _random_formula(r)
        rc, msg, hz = B.formula_check(text, names)
        codes[rc] = codes.get(rc, 0) + 1
        try:
            f = bltlc.parse(text, names)
        except bltlc.ParseError:
            assert rc == B.SMC_E_PARSE, (text, rc, msg)
            continue
        assert rc != B.SMC_E_PARSE, (text, msg)
        if rc == B.SMC_OK:
            h = oracle.horizon(f)
            assert h == hz or (math.isinf(h) and math.isinf(hz)), (text, hz, h)
    assert min(codes.get(c, 0) for c in (B.SMC_OK, B.SMC_E_PARSE)) > 100, codes
