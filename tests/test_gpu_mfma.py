"""The matrix-core operand and accumulator lane layout the stage kernels
assume, checked on one 16x16x4 product against numpy: FP64
(v_mfma_f64_16x16x4f64, whose accumulator rows are interleaved differently
from FP32's) and FP32 (v_mfma_f32_16x16x4f32, inputs rounded to FP32)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_mfma_layout_against_numpy(lib, precision):
    import torch
    rng = np.random.default_rng(7 + precision)
    A, B = rng.standard_normal((16, 4)), rng.standard_normal((4, 16))
    if precision == 1:  # the product of the FP32-rounded inputs
        A, B = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    dA = torch.tensor(A, device="cuda")
    dB = torch.tensor(B, device="cuda")
    dD = torch.full((16, 16), float("nan"), dtype=torch.float64, device="cuda")
    lib.cmcg_debug_mfma(precision, dA, dB, dD)
    D = dD.cpu().numpy()
    ref = A @ B
    tol = 1e-14 if precision == 0 else 1e-6
    assert np.max(np.abs(D - ref)) <= tol * np.max(np.abs(ref)), np.abs(D - ref).max()
    # each output row sits where the layout puts it: a permuted layout fails here
    for i in range(16):
        assert np.argmax(np.abs(D[i] - ref[i])) >= 0 and np.allclose(D[i], ref[i], rtol=tol, atol=tol)
