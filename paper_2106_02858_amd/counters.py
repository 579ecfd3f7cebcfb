"""Counter workload for HBM-traffic measurement of the stage kernel.

    python -m paper_2106_02858_amd.counters [--n 20 --q 3 --periods 2]

Runs whole homogeneous periods (4 M stage launches each) of the large
single-solve problem (48000 tets, P3, FP32 fields), then a plain elementwise
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
    a = ap.parse_args()
    import torch

    from . import cmcg, inputs
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = inputs.large_single(n=a.n, q=a.q)
    mesh = cmcg.cmcg_mesh_create(w.xyz, w.tet, w.tags)
    s = cmcg.cmcg_space_create(mesh, w.q, cmcg.CMCG_FP32)
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
