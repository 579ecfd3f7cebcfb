"""Stage-variant autotuner: it times every variant that applies to the
problem's (q, precision) on the problem's own launch shape and keeps the
fastest; an autotuned solve equals a solve run with that variant chosen by
hand, and batched solves stay equal to single solves under the tuned choice."""
import numpy as np
import pytest

from oracle import cmcg as ocmcg
from tests._pairs import pair, rel_norm_c

pytestmark = pytest.mark.gpu


@pytest.fixture
def keep_variants(lib):
    saved = {(q, p): lib.cmcg_tune_get_stage(q, p) for q in (1, 2, 3) for p in (0, 1)}
    yield
    for (q, p), v in saved.items():
        lib.cmcg_tune_stage(q, p, v)


def filtered(lib, r, K, Np):
    import torch
    fr = torch.zeros((K, 6, Np), dtype=torch.float64, device="cuda")
    fi = torch.zeros_like(fr)
    lib.cmcg_result_filtered_device(r, fr, fi)
    return fr.cpu().numpy() + 1j * fi.cpu().numpy()


@pytest.mark.parametrize("q,precision", [(1, 0), (2, 1), (3, 1)])
def test_autotune_keeps_fastest_applicable_variant(lib, keep_variants, q, precision):
    print(f"autotune q={q} prec={precision}", flush=True)
    op, s, lp = pair(lib, n=3 if q < 3 else 2, q=q, precision=precision, seed=30 + q)
    v, us = lib.cmcg_autotune_stage(lp)
    print(f"  chosen {v}, us per launch {us}")
    applies = [True, True] + [precision == 1 and q >= 2] * 3
    assert all((u > 0) == a for u, a in zip(us, applies))
    assert us[v] == min(u for u in us if u > 0)
    assert lib.cmcg_tune_get_stage(q, precision) == v


@pytest.mark.parametrize("q", [2, 3])
def test_autotuned_solve_equals_chosen_variant(lib, keep_variants, q):
    op, s, lp = pair(lib, n=2 if q < 3 else 1, q=q, precision=1, seed=40 + q, sigma=False)
    r_auto = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=3, autotune=1))
    v = lib.cmcg_tune_get_stage(q, 1)
    lib.cmcg_tune_stage(q, 1, v)
    r_hand = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=3))
    a, b = filtered(lib, r_auto, op.K, op.Np), filtered(lib, r_hand, op.K, op.Np)
    assert np.array_equal(a, b)
    ref = ocmcg.solve(op, fixed_iters=3)
    assert rel_norm_c(op, a, ref.F) < 1e-5


def test_batch_autotune_members_equal_single_solves(lib, keep_variants):
    from tests.test_gpu_batch import members
    s, probs, _, _ = members(lib, 2, 2, 1, 3, seed=91)
    info = lib.cmcg_space_info(s)
    K, Np = info["K"], info["Np"]
    res = lib.cmcg_solve_batch(probs, lib.cmcg_options_default(fixed_iters=3, autotune=1))
    v = lib.cmcg_tune_get_stage(2, 1)
    assert v in range(lib.CMCG_STAGE_VARIANTS)
    for p, r in zip(probs, res):
        single = lib.cmcg_solve(p, lib.cmcg_options_default(fixed_iters=3))
        assert np.array_equal(filtered(lib, r, K, Np), filtered(lib, single, K, Np))
