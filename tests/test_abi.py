"""The C ABI library loads and exports every entry point include/smc.h
declares; its host-side Wilson functions agree with the oracle's (no GPU)."""
import math
import os
import re

import pytest

from oracle import wilson
from paper_0912_2551_amd import binding as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "smc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smc_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = B.lib()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(B.EXPORTS) == names


def test_host_z_matches_oracle():
    for c in (0.8, 0.9, 0.95, 0.99, 0.999, 0.9999, 0.5):
        assert B.z_value(c) == wilson.z_value(c)
    assert math.isnan(B.z_value(1.0))


@pytest.mark.parametrize("eps,conf", [(0.01, 0.95), (0.025, 0.99), (0.005, 0.9999)])
def test_host_wilson_matches_oracle(eps, conf):
    z = wilson.z_value(conf)
    for k in range(0, 1001):
        p = k / 1000.0
        assert B.wilson_sample_value(p, eps, z) == wilson.wilson_sample_value(p, eps, z)
        assert B.wilson_sample(p, eps, z) == wilson.wilson_sample(p, eps, z)
    for n in (1, 7, 189, 454, 2648, 9600, 10**6):
        for k in sorted({0, 1, n // 3, n // 2, n - 1, n}):
            assert B.wilson_interval(k, n, z) == wilson.wilson_interval(k, n, z)


def test_context_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(B.SmcError):
        B.Context(0)
