"""Autotuner of the leaf size, the core-SVD dispatch and the matrix-core tile
shape of narrow products, through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1701_00182_amd as acr  # noqa: E402
from oracle.assemble import operator_from_coef, relres  # noqa: E402
from workloads import problem, rhs_normal  # noqa: E402

DEV = torch.device("cuda:0")


def test_autotune_choice_is_a_candidate_cached_and_usable(tmp_path):
    n = 16
    coef = problem("convdiff", n)
    c = torch.from_numpy(coef).to(DEV)
    cache = str(tmp_path / "tune.txt")
    r1 = acr.autotune(c, eps=1e-2, precision="fp32", sample_planes=8, cache=cache)
    assert r1["leaf"] in (32, 64, 128) and not r1["from_cache"] and r1["tried"] >= 6
    assert r1["svd_fused_lds"] in (-1, 64 * 1024, 156 * 1024) and r1["seconds"] > 0
    assert r1["gemm_tiles"] in (0, 1) and r1["tried"] >= 7
    r2 = acr.autotune(c, eps=1e-2, precision="fp32", sample_planes=8, cache=cache)
    assert r2["from_cache"] and (r2["leaf"], r2["svd_fused_lds"], r2["gemm_tiles"]) == \
        (r1["leaf"], r1["svd_fused_lds"], r1["gemm_tiles"])
    # a different key measures again
    r3 = acr.autotune(c, eps=1e-3, precision="fp32", sample_planes=8, cache=cache)
    assert not r3["from_cache"]
    f = rhs_normal(n ** 3)
    fac = acr.Factor(c, eps=1e-2, leaf=r1["leaf"], precision="fp32", svd_fused_lds=r1["svd_fused_lds"],
                     gemm_tiles=r1["gemm_tiles"])
    x, info = fac.solve_refined(torch.from_numpy(f).to(DEV), tol=1e-10, method="gmres")
    assert info["converged"] and float(relres(operator_from_coef(coef), x.cpu().numpy(), f)) <= 1e-10
    fac.free()
