"""Counter workload for HBM-traffic measurement of the stage kernel.

    python -m paper_2106_02858_amd.counters [--n 20 --q 3 --periods 2]
    python -m paper_2106_02858_amd.counters --trap2d      # the 2-D disk trap instead
    python -m paper_2106_02858_amd.counters --fp64        # FP64 fields (either problem)
    python -m paper_2106_02858_amd.counters --scatterer   # the 1,572,864-tet P2 scatterer, one period
    python -m paper_2106_02858_amd.counters --batched     # 64 members on the 10368-tet P2 mesh

Runs whole homogeneous periods (4 M stage launches each) of the large
single-solve problem (48000 tets, P3, FP32 fields) -- or, with --trap2d, of
the 2-D dipole-in-trap problem (22500 triangles, P3, FP32), with --scatterer
one period of the 1,572,864-tet P2 scatterer, with --batched the batched
autotuner's timing launches of the 64-member P2 batch (every member active);
--fp64 takes FP64 fields instead -- then a plain elementwise
copy of known size (read 4 B, write 4 B per float; 1 GiB each way) that
calibrates what FETCH_SIZE / WRITE_SIZE report per byte moved.  Under
`rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE) the per-dispatch averages of
the two kernels give the stage kernel's measured HBM traffic.
"""
from __future__ import annotations

import argparse
import sys


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=20)
    ap.add_argument("--q", type=int, default=3)
    ap.add_argument("--periods", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--trap2d", action="store_true")
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--scatterer", action="store_true",
                    help="one homogeneous period of the 1,572,864-tet P2 scatterer (FP32 fields)")
    ap.add_argument("--variant", type=int, default=-1,
                    help="stage-kernel variant for the field precision and order (default: the library's choice)")
    ap.add_argument("--batched", action="store_true",
                    help="the batched autotuner on the 64 members of the 10368-tet P2 mesh: every stage variant "
                         "timed on 8 steps with all members active (FP32 fields)")
    a = ap.parse_args()
    import torch

    from . import cmcg, inputs
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if a.trap2d:
        w = inputs.trap2d(75, 3, "disk")
        mesh = cmcg.cmcg_mesh2d_create(w.xy, w.tri, w.tags)
        s = cmcg.cmcg_space_create(mesh, 3, cmcg.CMCG_FP64 if a.fp64 else cmcg.CMCG_FP32)
        p = cmcg.cmcg_problem_create(s, w.eps, w.mu, None, w.omega,
                                     inputs.current_2d(w, cmcg.cmcg_space_nodes(s)))
        info = cmcg.cmcg_space_info(s)
        K, Np = info["K"], info["Np"]
        M, _ = cmcg.cmcg_problem_steps(p)
        print(f"2-D stage kernel: K={K} Np={Np} M={M}, {a.periods} periods = {4 * M * a.periods} launches",
              flush=True)
        U0 = torch.randn((K, 3, Np), dtype=torch.float64, device=dev) * 1e-3
        UT = torch.empty_like(U0)
        for _ in range(a.periods):
            cmcg.cmcg_debug_period(p, U0, UT, 1, False)
        torch.cuda.synchronize()
        return copy_calibration(a, dev)
    if a.batched:
        ws = inputs.batched_members(n=12, q=2, B=64)
        mesh = cmcg.cmcg_mesh_create(ws[0].xyz, ws[0].tet, ws[0].tags)
        s = cmcg.cmcg_space_create(mesh, 2, cmcg.CMCG_FP32)
        nodes = cmcg.cmcg_space_nodes(s)
        probs = [cmcg.cmcg_problem_create(s, w.eps, w.mu, None, w.omega,
                                          inputs.gaussian_current(nodes, w.centre, w.width, w.pol)) for w in ws]
        v, us = cmcg.cmcg_autotune_batch(probs)
        print(f"batched stage kernel: 64 members x {ws[0].K} tets, P2; variant {v}; us per launch "
              f"{[round(u, 2) for u in us]}", flush=True)
        torch.cuda.synchronize()
        return copy_calibration(a, dev)
    w = inputs.scatterer() if a.scatterer else inputs.large_single(n=a.n, q=a.q)
    if a.variant >= 0:
        cmcg.cmcg_tune_stage(w.q, cmcg.CMCG_FP64 if a.fp64 else cmcg.CMCG_FP32, a.variant)
    if a.scatterer:
        a.periods = 1
    mesh = cmcg.cmcg_mesh_create(w.xyz, w.tet, w.tags)
    s = cmcg.cmcg_space_create(mesh, w.q, cmcg.CMCG_FP64 if a.fp64 else cmcg.CMCG_FP32)
    nodes = cmcg.cmcg_space_nodes(s)
    j = torch.tensor(inputs.gaussian_current(nodes, w.centre, w.width, w.pol), dtype=torch.float64, device=dev)
    p = cmcg.cmcg_problem_create_device(s, w.eps, w.mu, w.sigma, w.omega, j)
    info = cmcg.cmcg_space_info(s)
    K, Np = info["K"], info["Np"]
    opts = cmcg.cmcg_options_default()
    M, _ = cmcg.cmcg_problem_steps(p, opts)
    print(f"stage kernel: K={K} Np={Np} M={M}, {a.periods} periods = {4 * M * a.periods} launches", flush=True)
    U0 = torch.randn((K, 6, Np), dtype=torch.float64, device=dev) * 1e-3
    UT = torch.empty_like(U0)
    for _ in range(a.periods):
        cmcg.cmcg_debug_period(p, U0, UT, 1, False, opts=opts)
    torch.cuda.synchronize()
    return copy_calibration(a, dev)


def copy_calibration(a, dev) -> int:
    """Plain elementwise copies of known size (torch.neg: read and write
    copy_mib MiB each): what FETCH_SIZE / WRITE_SIZE report per byte moved."""
    import torch
    n = a.copy_mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    for _ in range(a.copies):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(f"copy kernel: {a.copies} x (read {a.copy_mib} MiB, write {a.copy_mib} MiB)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
