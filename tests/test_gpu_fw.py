"""Limiting-amplitude (FW) iteration on the GPU against the FP64 oracle:
filtered field and per-period relative state changes after a fixed number
of periods (RK2 + trapezoid for P1, RK4 + Hermite for P2), and the
tolerance stop."""
import numpy as np
import pytest

from oracle import fw
from tests._pairs import pair, rel_norm_c

pytestmark = pytest.mark.gpu


def filtered(lib, r, K, Np):
    import torch
    fr = torch.zeros((K, 6, Np), dtype=torch.float64, device="cuda")
    fi = torch.zeros_like(fr)
    lib.cmcg_result_filtered_device(r, fr, fi)
    return fr.cpu().numpy() + 1j * fi.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 2])
def test_fw_fixed_periods_against_oracle(lib, q, precision):
    op, s, lp = pair(lib, n=2, q=q, precision=precision, seed=4 + q, sigma=False)
    periods = 6
    ref = fw.solve(op, periods)
    r = lib.cmcg_fw_solve(lp, lib.cmcg_options_default(fixed_iters=periods))
    st = lib.cmcg_result_stats(r)
    assert st["periods"] == periods and st["status"] == lib.CMCG_OK
    err = rel_norm_c(op, filtered(lib, r, op.K, op.Np), ref.F)
    hist = lib.cmcg_result_history(r)
    print(f"fw q={q} prec={precision}: filtered rel err {err:.2e}, changes {hist[0]:.3e} .. {hist[-1]:.3e}")
    assert err < (1e-11 if precision == 0 else 1e-5)
    assert np.allclose(hist, ref.history, rtol=1e-8 if precision == 0 else 1e-3)


def test_fw_tolerance_stop(lib):
    op, s, lp = pair(lib, n=2, q=1, precision=0, seed=9, sigma=False, tags=2)
    r = lib.cmcg_fw_solve(lp, lib.cmcg_options_default(tol=1e-6, max_iter=500))
    st = lib.cmcg_result_stats(r)
    hist = lib.cmcg_result_history(r)
    assert st["status"] == lib.CMCG_OK and st["periods"] < 500
    assert hist[-1] <= 1e-6 < hist[-2] and st["periods"] == len(hist) + 1
    ref = fw.solve(op, st["periods"])
    assert rel_norm_c(op, filtered(lib, r, op.K, op.Np), ref.F) < 1e-11


# ---- run-up: limiting-amplitude periods before CMCG (cmcg_options.runup)

@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 2])
def test_cmcg_after_runup_against_oracle(lib, q, precision):
    from oracle import cmcg as ocmcg
    print(f"runup q={q} prec={precision}", flush=True)
    op, s, lp = pair(lib, n=2, q=q, precision=precision, seed=20 + q, sigma=False, tags=2)
    runup, iters = 3, 4
    ref = ocmcg.solve(op, fixed_iters=iters, runup=runup)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=iters, runup=runup))
    st = lib.cmcg_result_stats(r)
    # run-up, Algorithm 1, the first gradient, two per CG iteration, the filter
    assert st["periods"] == runup + 2 + 2 + 2 * iters + 1 and st["iters"] == iters
    err = rel_norm_c(op, filtered(lib, r, op.K, op.Np), ref.F)
    print(f"  filtered rel err {err:.2e}")
    assert err < (1e-11 if precision == 0 else 1e-5)
    # the reported first residual is the gradient's norm at the run-up state
    ops = ocmcg.Operators(op)
    _, Gs = ocmcg.initialise(ops)
    U = np.zeros((op.K, 6, op.Np))
    for _ in range(runup):
        U = ops.P_psi(U)
    R0 = ocmcg.gradient(ops, U, Gs)
    res0 = np.sqrt(ops.ip(R0, R0))
    assert abs(st["res0"] - res0) <= (1e-11 if precision == 0 else 1e-5) * res0


def test_runup_batch_members_equal_single_solves(lib):
    from tests.test_gpu_batch import initial, members
    s, probs, _, _ = members(lib, 2, 2, 1, 3, seed=77)
    info = lib.cmcg_space_info(s)
    K, Np = info["K"], info["Np"]
    o = lib.cmcg_options_default(tol=1e-7, max_iter=200, runup=4)
    res = lib.cmcg_solve_batch(probs, o)
    for p, r in zip(probs, res):
        single = lib.cmcg_solve(p, o)
        a, b = lib.cmcg_result_stats(r), lib.cmcg_result_stats(single)
        assert a["iters"] == b["iters"] and a["periods"] == b["periods"]
        assert np.array_equal(lib.cmcg_result_history(r), lib.cmcg_result_history(single))
        assert np.array_equal(filtered(lib, r, K, Np), filtered(lib, single, K, Np))
        assert np.array_equal(initial(lib, r, K, Np), initial(lib, single, K, Np))


def test_negative_runup_rejected(lib):
    op, s, lp = pair(lib, n=1, q=1, precision=0, seed=1, sigma=False)
    with pytest.raises(lib.CmcgError) as e:
        lib.cmcg_solve(lp, lib.cmcg_options_default(runup=-1))
    assert e.value.code == lib.CMCG_ERR_ARG
