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
