"""The C-ABI library: loads, exports every declared entry point, host-side
helpers are exact; no device work (runs without a GPU)."""
import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest

from tests import bruteforce as bf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "upr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(upr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2308_15494_amd import upr
    return upr.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), f"{name} declared in upr.h but not exported"


def test_binding_covers_header():
    from paper_2308_15494_amd import upr
    bound = {s[0] for s in upr._SIGS}
    assert bound == set(declared_functions())


def test_lmax_host(lib):
    from paper_2308_15494_amd import upr
    rng = np.random.default_rng(3)
    for _ in range(2000):
        total = int(rng.integers(0, 1 << 40))
        k = int(rng.integers(2, 70000))
        eps = (int(rng.integers(1, 1000)), int(rng.integers(1, 1000)))
        assert upr.lmax(total, k, eps) == bf.lmax_exact(total, k, eps)
    assert upr.lmax(1_048_576, 64) == 16875


@pytest.mark.parametrize("tau", [(0, 1), (1, 2), (1, 1), (21, 38), (2**31 - 2, 2**31 - 1)])
def test_penalty_table_host(lib, tau):
    from paper_2308_15494_amd import upr
    q = upr.penalty_table(tau)
    for l in range(54):
        assert q[l] == math.floor(Fraction(*tau) * Fraction(3, 2) ** l * 65536)


def test_penalty_table_rejects(lib):
    from paper_2308_15494_amd import upr
    with pytest.raises(upr.UprError):
        upr.penalty_table((3, 2))


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2308_15494_amd import upr
    monkeypatch.setattr(upr, "_lib", None)
    monkeypatch.setattr(upr, "LIB_PATH", os.path.join(ROOT, "does_not_exist.so"))
    with pytest.raises(RuntimeError, match="not built"):
        upr.lib()


def test_create_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2308_15494_amd import upr
    with pytest.raises(upr.UprError):
        upr.Context(0)
