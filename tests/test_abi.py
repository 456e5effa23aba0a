"""The C-ABI library loads on the CPU host and exports every entry point its header
declares; its host-side IMM arithmetic matches the oracle bit for bit."""
import os
import re

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "imm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(imm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2009_07325_amd as imm
    L = imm.lib()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(imm.EXPORTS)


def test_binding_has_same_names():
    import paper_2009_07325_amd as imm
    for n in declared_functions():
        assert callable(getattr(imm, n)), n


@pytest.mark.parametrize("n,k,eps,ell", [
    (1000, 10, 0.5, 1.0), (1 << 20, 50, 0.1, 1.0), (1 << 22, 100, 0.1, 1.0),
    (1 << 24, 200, 0.05, 1.0), (2, 1, 0.3, 1.0), (3, 2, 0.9, 2.5), (10_000, 100, 0.2, 1.0),
    (123_457, 77, 0.37, 0.5)])
def test_sample_size_math_matches_oracle_bitwise(oracle_lib, n, k, eps, ell):
    import paper_2009_07325_amd as imm
    assert imm.imm_log_binom(n, k) == oracle_lib.log_binom(n, k)
    assert imm.imm_lambda_prime(n, k, eps, ell) == oracle_lib.lambda_prime(n, k, eps, ell)
    assert imm.imm_lambda_star(n, k, eps, ell) == oracle_lib.lambda_star(n, k, eps, ell)


def test_no_cpu_fallback_in_binding():
    """The binding never imports the oracle; a missing library raises."""
    src = open(os.path.join(ROOT, "paper_2009_07325_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("oracle and", "")
    import paper_2009_07325_amd as imm
    saved = imm.LIB_PATH, imm._lib
    try:
        imm.LIB_PATH, imm._lib = "/nonexistent/libimm.so", None
        with pytest.raises(RuntimeError):
            imm.lib()
    finally:
        imm.LIB_PATH, imm._lib = saved


@pytest.mark.parametrize("n,k,rounds,eps,ell", [
    (1000, 10, 5, 0.1, 1.0), (1 << 20, 50, 3, 0.2, 1.0), (4096, 1, 2, 0.5, 1.0),
    (77_777, 33, 32, 0.07, 2.0), (1000, 10, 1, 0.1, 1.0)])
def test_multi_round_sample_sizes_match_oracle_bitwise(oracle_lib, n, k, rounds, eps, ell):
    """The CR-NAIMM sample sizes (gIM Sec. IV-H) of the library's host code and the
    oracle's agree bit for bit; with one round they are IMM's."""
    import paper_2009_07325_amd as imm
    assert imm.imm_mr_lambda_prime(n, k, rounds, eps, ell) == oracle_lib.mr_lambda_prime(n, k, rounds, eps, ell)
    assert imm.imm_mr_lambda_star(n, k, rounds, eps, ell) == oracle_lib.mr_lambda_star(n, k, rounds, eps, ell)
    if rounds == 1:
        assert imm.imm_mr_lambda_star(n, k, 1, eps, ell) == imm.imm_lambda_star(n, k, eps, ell)
        assert imm.imm_mr_lambda_prime(n, k, 1, eps, ell) == imm.imm_lambda_prime(n, k, eps, ell)
