"""The algorithmic HBM bytes behind ``roofline.achieved``, counted here array
by array for each Runge-Kutta stage (Section 5.3 schemes, fused stage update)
and compared with bench.py's closed forms: the implementation's traffic
(stage_bytes_per_element) and the method's minimum that roofline.frac uses
(method_bytes_per_dof_update).

Per dof, with Y the stage input, Y' its output, U the state and Acc the
stage-combination accumulator (RK4), the launches of one step touch:

  RK4  stage 1: read Y; write Y', Acc
       stages 2, 3: read Y, U, Acc; write Y', Acc
       stage 4: read Y, Acc; write U
  RK2  stage 1: read U; write Y'
       stage 2: read Y', U; write U

With FP32 fields the state carries a 2-byte low part (compensated sum): the
last stage also reads U (to form the two-sum) and reads and writes the low part.
Each element adds its geometry (40 values in 3-D, 25 in 2-D) and connectivity
(4 or 3 int32) once per launch; neighbour traces count as cache hits.
"""
from __future__ import annotations

import pytest

import bench

RK4 = [(["Y"], ["Y'", "Acc"]), (["Y", "U", "Acc"], ["Y'", "Acc"]), (["Y", "U", "Acc"], ["Y'", "Acc"]),
       (["Y", "Acc"], ["U"])]
RK2 = [(["U"], ["Y'"]), (["Y'", "U"], ["U"])]


def _field_bytes_per_dof_step(q: int, esize: int) -> float:
    stages = RK4 if q >= 2 else RK2
    total = 0.0
    for s, (reads, writes) in enumerate(stages):
        total += esize * (len(reads) + len(writes))
        if esize == 4 and s == len(stages) - 1:
            total += 2 + 2                     # low part read and written
            if "U" not in reads:
                total += 4                     # U read for the two-sum
    return total


@pytest.mark.parametrize("esize", [4, 8])
@pytest.mark.parametrize("q", [1, 2, 3])
def test_stage_bytes_count_every_array(q, esize):
    nst = 4 if q >= 2 else 2
    np3 = (q + 1) * (q + 2) * (q + 3) // 6
    np2 = (q + 1) * (q + 2) // 2
    per_dof_stage = _field_bytes_per_dof_step(q, esize) / nst
    assert bench.stage_bytes_per_element(q, esize) == pytest.approx(
        6 * np3 * per_dof_stage + 40 * esize + 4 * 4)
    assert bench.stage2d_bytes_per_element(q, esize) == pytest.approx(
        3 * np2 * per_dof_stage + 25 * esize + 3 * 4)
    for members in (1, 64):
        assert bench.bytes_per_dof_update(q, esize, members) == pytest.approx(
            (6 * np3 * _field_bytes_per_dof_step(q, esize) + nst * (40 * esize + 16) / members) / (6 * np3))
        assert bench.bytes_per_dof_update_2d(q, esize, members) == pytest.approx(
            (3 * np2 * _field_bytes_per_dof_step(q, esize) + nst * (25 * esize + 12) / members) / (3 * np2))


def test_quoted_figures():
    """The per-launch and per-dof-update figures the measurements are priced with."""
    assert _field_bytes_per_dof_step(3, 4) == 72 and _field_bytes_per_dof_step(3, 8) == 128
    assert _field_bytes_per_dof_step(1, 4) == 24 and _field_bytes_per_dof_step(1, 8) == 40
    assert bench.stage_bytes_per_element(3, 4) == 2336
    assert bench.stage_bytes_per_element(3, 8) == 4176
    assert bench.bytes_per_dof_update(3, 4) == pytest.approx(77.87, abs=0.01)
    assert bench.bytes_per_dof_update(2, 4, 64) == pytest.approx(72.18, abs=0.01)
    # the 48000-tet P3 FP32 launch
    assert 48000 * bench.stage_bytes_per_element(3, 4) == 112128000


def test_method_bytes_count_every_array():
    """The method's minimum (what roofline.frac is priced with): the field
    passes of the stage table above without the compensated state's extra
    traffic, plus 128 B (FP32) or 236 B (FP64) of geometry and connectivity
    per element and right-hand side, shared by the members of a batch; the
    compensated state's extra 8 B per dof and step is reported separately."""
    for q in (1, 2, 3):
        np3 = (q + 1) * (q + 2) * (q + 3) // 6
        nst = 4 if q >= 2 else 2
        for esize, geo in ((4, 128), (8, 236)):
            plain = sum(esize * (len(r) + len(w)) for r, w in (RK4 if q >= 2 else RK2))
            for members in (1, 64):
                assert bench.method_bytes_per_dof_update(q, esize, members) == pytest.approx(
                    plain + nst * geo / (6 * np3) / members)
                assert bench.method_bytes_per_launch(q, esize, 1000, members) == pytest.approx(
                    bench.method_bytes_per_dof_update(q, esize, members) * 6 * np3 * 1000 * members / nst)
        extra = _field_bytes_per_dof_step(q, 4) - sum(4 * (len(r) + len(w)) for r, w in (RK4 if q >= 2 else RK2))
        assert bench.compensation_bytes_per_launch(q, 1000) == pytest.approx(extra * 6 * np3 * 1000 / nst)


def test_method_figures():
    assert bench.method_bytes_per_dof_update(3, 4) == pytest.approx(68.27, abs=0.01)     # 48000-tet P3 FP32
    assert bench.method_bytes_per_dof_update(3, 8) == pytest.approx(135.87, abs=0.01)    # the same, FP64
    assert bench.method_bytes_per_dof_update(2, 4, 64) == pytest.approx(64.13, abs=0.01)  # 64-member P2 batch
    assert bench.method_bytes_per_dof_update(2, 4) == pytest.approx(72.53, abs=0.01)     # 1,572,864-tet P2
    assert bench.method_bytes_per_dof_update(1, 8) == pytest.approx(59.67, abs=0.01)     # 1296-tet P1 FP64
    assert bench.method_bytes_per_launch(3, 4, 48000) == pytest.approx(98.304e6, rel=1e-6)
