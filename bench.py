"""Benchmark: CMCG for time-harmonic Maxwell on one MI355X.

Workload (default): unit cube 20^3 x 6 = 48000 tetrahedra, P3 (20 nodes), eps
per cube from {1,2,4} (seed 2), mu = 1, omega = 4 pi, impedance boundary,
Gaussian e_z current of width 0.05 at a seeded point of [0.3,0.7]^3.
Fields are stepped in FP32 with the CG vectors, inner products, alpha/beta
and the filter accumulator in FP64.

One step = one complete CMCG solve from the zero guess (Algorithm 1, CG
iterations until ||R||/||R0|| <= 1e-6, filter period), inputs resident in
HBM.  value = DG dof-updates per second over the timed steps (6 Np K per
time step, all periods).  Also reported: time-to-1e-6 of the FP32-field path
and of the plain FP64 path on the same problem, the roofline of the dominant
kernel (the fused RK4 stage kernel), and the FP64 CPU oracle on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=20)
    ap.add_argument("--q", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 reference solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default stage-kernel variant instead of autotuning it in the warm-up solve")
    ap.add_argument("--cpu-steps", type=int, default=4, help="RK steps of the CPU oracle sample")
    ap.add_argument("--kernel-periods", type=int, default=3)
    ap.add_argument("--workload", choices=["large_single", "batched", "serving", "scatterer", "fw", "trap2d",
                                           "curves2d", "lts"],
                    default="large_single",
                    help="large_single (default bench line), the 64-member batched configuration, or the "
                         "Poisson request stream through the serving engine")
    ap.add_argument("--trap", choices=["square", "disk"], default="disk", help="trap2d: shape of the trap")
    ap.add_argument("--exp", choices=["cavity", "cavity_near", "planewave", "waveguide", "trap"], default="cavity",
                    help="curves2d: which 2-D experiment")
    ap.add_argument("--max-periods", type=int, default=1024, help="curves2d: longest run in simulated periods")
    ap.add_argument("--n2d", type=int, default=75, help="trap2d: cells per side of the Cartesian mesh")
    ap.add_argument("--members2d", type=int, default=1, help="trap2d: dipole positions solved in one batch")
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--fp64-members", type=int, default=64,
                    help="batched: members also solved one by one with plain FP64 fields (0: none)")
    ap.add_argument("--cg-iters", type=int, default=6, help="scatterer: CG iterations of the timed solve")
    ap.add_argument("--fw-walls", choices=["impedance", "pec"], default="impedance",
                    help="fw: walls of the comparison problem (pec: closed cavity)")
    ap.add_argument("--requests", type=int, default=60, help="serving: requests taken from the stream")
    ap.add_argument("--rate", type=float, default=20.0, help="serving: Poisson arrival rate (req/s)")
    ap.add_argument("--slots", type=int, default=8, help="serving: engine slots")
    ap.add_argument("--serve-precision", choices=["fp32", "fp64"], default="fp32",
                    help="serving: field precision of the served solves (fp64: the plain form, for comparison)")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serving: engine memory budget")
    ap.add_argument("--cobatch", type=int, default=8,
                    help="serving: queued requests on one space (n, q) that may share a slot and run as one "
                         "batched solve (1: every request alone)")
    ap.add_argument("--cobatch-max-k", type=int, default=3072,
                    help="serving: co-batch only spaces of at most this many elements (0: any); the default "
                         "takes the n = 8 meshes, whose single launches fill an eighth of the chip")
    ap.add_argument("--lts-n", type=int, default=20, help="lts: cells per axis")
    ap.add_argument("--lts-r", type=int, default=32, help="lts: the thin layers are 1/r of a cell wide")
    ap.add_argument("--lts-m", type=int, default=8, help="lts: fine substeps per coarse step")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="default line: requests of the short served stream")
    ap.add_argument("--no-extra", action="store_true",
                    help="default line: skip the scatterer and batched kernel rooflines and the short served stream")
    return ap.parse_args()


# FETCH_SIZE / WRITE_SIZE per dispatch (KiB) of the stage kernel on the
# 48000-tet P3 FP32 problem, with the scales a 1 GiB copy gives each counter;
# valid only for the kernel source they were taken on (SHA-256 below).
MEASURED_TRAFFIC = [
    {"kernels_sha256": "95f2693eedc0bcfb1df99161361c7df1cf804e6b22fdb00f46db1035fc9af466",
     "kernel": "k_stage_mfma<float,3,true,false,2,false,true>", "K": 48000,
     "fetch_kib": 41696.72, "fetch_scale": 2.0000, "write_kib": 42197.84, "write_scale": 1.0000},
    {"kernels_sha256": "95f2693eedc0bcfb1df99161361c7df1cf804e6b22fdb00f46db1035fc9af466",
     "kernel": "k_stage_mfma<float,3,true,false,4>", "K": 48000,
     "fetch_kib": 41006.57, "fetch_scale": 2.0000, "write_kib": 42187.65, "write_scale": 1.0000},
]


# The same for the FP64 stage kernel of the plain FP64 solve (48000 tets, P3):
# the two forms its autotuner keeps (two and four waves per block).
MEASURED_TRAFFIC_FP64 = [
    {"kernels_sha256": "95f2693eedc0bcfb1df99161361c7df1cf804e6b22fdb00f46db1035fc9af466",
     "kernel": "k_stage_mfma<double,3,true,false,2>", "K": 48000,
     "fetch_kib": 81060.19, "fetch_scale": 2.0000, "write_kib": 78750.00, "write_scale": 1.0000},
    {"kernels_sha256": "95f2693eedc0bcfb1df99161361c7df1cf804e6b22fdb00f46db1035fc9af466",
     "kernel": "k_stage_mfma<double,3,true,false,4>", "K": 48000,
     "fetch_kib": 75600.09, "fetch_scale": 2.0000, "write_kib": 78750.00, "write_scale": 1.0000},
]


# The same for the P2 FP32 stage kernels of the large launches: the
# 1,572,864-tet scatterer (variants 3 and 2, the two its autotuner keeps) and the
# batched launch of 64 members on the 10368-tet mesh, every member active
# (K = members x elements; every variant the batched autotuner times).
_SHA_Q2 = "95f2693eedc0bcfb1df99161361c7df1cf804e6b22fdb00f46db1035fc9af466"
MEASURED_TRAFFIC_Q2 = [
    {"kernels_sha256": _SHA_Q2, "kernel": "k_stage_mfma<float,2,true,false,1>", "K": 1572864,
     "fetch_kib": 826087.99, "fetch_scale": 2.0000, "write_kib": 696403.27, "write_scale": 1.0000},
    {"kernels_sha256": _SHA_Q2, "kernel": "k_stage_mfma<float,2,false,false,1>", "K": 1572864,
     "fetch_kib": 841445.58, "fetch_scale": 2.0000, "write_kib": 696003.22, "write_scale": 1.0000},
] + [
    {"kernels_sha256": _SHA_Q2, "kernel": k, "K": 64 * 10368,
     "fetch_kib": fe, "fetch_scale": 2.0000, "write_kib": wr, "write_scale": 1.0000}
    for k, fe, wr in (("k_stage_mfma<float,2,true,false,1>", 261308.21, 293151.86),
                      ("k_stage_mfma<float,2,false,false,1>", 265477.60, 293033.53),
                      ("k_stage<float,2,false,false>", 284333.38, 292218.74),
                      ("k_stage<float,2,true,false>", 252748.48, 291670.07),
                      ("k_stage_mfma<float,2,true,false,2>", 247271.13, 291747.63),
                      ("k_stage_mfma<float,2,true,false,2,true>", 245780.23, 291612.83),
                      ("k_stage_mfma<float,2,true,false,4>", 245653.31, 291603.04),
                      ("k_stage_mfma<float,2,true,false,4,true>", 245600.44, 291600.09))
]


# The same for the 2-D stage kernel on the 22500-triangle disk trap (P3, FP32).
MEASURED_TRAFFIC_2D = {
    "kernels_sha256": "1e4fa0faed3d3bee44654fa8b73c89c99f3c0e16ad84b3f16579f81e44a68dfa",
    "kernel": "k_stage2d<float,3,true>", "K": 22500,
    "fetch_kib": 5077.52, "fetch_scale": 2.0000, "write_kib": 4944.12, "write_scale": 1.0000,
}


def measured_traffic(kernel: str, K: int, table=None, source: str = "kernels.hip"):
    """HBM bytes per launch from the committed counter runs (a table or a list
    of tables, one per measured kernel), or None when the kernel source or
    the workload differs from every one measured."""
    import hashlib
    tables = MEASURED_TRAFFIC if table is None else table
    tables = tables if isinstance(tables, list) else [tables]
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2106_02858_amd", "csrc", source)
    try:
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    for t in tables:
        if digest == t["kernels_sha256"] and kernel == t["kernel"] and K == t["K"]:
            return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024
    return None


# single-frequency instantiations (the MH template argument selects the several-frequency code)
STAGE_KERNEL = {0: "k_stage<float,{q},false,false>", 1: "k_stage<float,{q},true,false>",
                2: "k_stage_mfma<float,{q},false,false,1>", 3: "k_stage_mfma<float,{q},true,false,1>",
                4: "k_stage_mfma<float,{q},true,false,2>", 5: "k_stage_mfma<float,{q},true,false,2,true>",
                6: "k_stage_mfma<float,{q},true,false,2,false,true>",
                7: "k_stage_mfma<float,{q},true,false,2,true,true>",
                8: "k_stage_mfma<float,{q},true,false,4>", 9: "k_stage_mfma<float,{q},true,false,4,true>"}
STAGE_KERNEL64 = {v: k.replace("float", "double") for v, k in STAGE_KERNEL.items()}


def stage_bytes_per_element(q: int, esize: int) -> float:
    """Algorithmic HBM bytes of one average stage launch per element: the field
    vectors each stage must read or write once, plus the element's geometry
    (40 values) and connectivity (4 int32); neighbour traces are counted as
    cache hits.  RK4 per dof and step: stage 1 reads Y, writes Y', Acc;
    stages 2-3 read Y, U, Acc and write Y', Acc; stage 4 reads Y, Acc and
    writes U -- FP64: 16 passes of 8 B; FP32 with the compensated state also
    reads U and reads/writes the 2-byte low part in stage 4: 72 B.  RK2: FP64
    5 passes of 8 B; FP32 5 passes of 4 B + 2 x 2 B."""
    Np = (q + 1) * (q + 2) * (q + 3) // 6
    if q >= 2:
        per_dof = 72.0 / 4 if esize == 4 else 128.0 / 4
    else:
        per_dof = 24.0 / 2 if esize == 4 else 40.0 / 2
    return 6 * Np * per_dof + 40 * esize + 16


def method_bytes_per_dof_update(q: int, esize: int, members: int = 1) -> float:
    """The method's minimum HBM bytes per dof-update (one dof advanced one
    full time step): every field vector the Runge-Kutta form must read or
    write once per stage -- RK4 16 passes (stage 1 reads Y and writes Y',
    Acc; stages 2-3 read Y, U, Acc and write Y', Acc; stage 4 reads Y, Acc and
    writes U), RK2 5 passes -- plus each element's geometry and connectivity
    once per right-hand side (27 geometry scalars, 4 neighbour ids, 4 face
    codes: 128 B with FP32 fields, 236 B with FP64), shared by the members of
    a batched launch; neighbour traces are taken as cache hits.  The 48000-tet
    P3 FP32 solve: 68.27 B; the 64-member P2 batch: 64.13 B; the
    1,572,864-tet P2 scatterer: 72.53 B; FP64 P3: 135.87 B."""
    Np = (q + 1) * (q + 2) * (q + 3) // 6
    passes, stages = (16, 4) if q >= 2 else (5, 2)
    geo = 128.0 if esize == 4 else 236.0
    return passes * esize + stages * geo / (6 * Np) / members


def method_bytes_per_launch(q: int, esize: int, K: int, members: int = 1) -> float:
    """method_bytes_per_dof_update spread over the stage launches of a step
    (each launch advances 6 Np K dofs of every member by one stage)."""
    Np = (q + 1) * (q + 2) * (q + 3) // 6
    stages = 4 if q >= 2 else 2
    return method_bytes_per_dof_update(q, esize, members) * 6 * Np * K * members / stages


def compensation_bytes_per_launch(q: int, K: int, members: int = 1) -> float:
    """Extra traffic of the compensated FP32 state, beyond the method's
    minimum, per dof and step: the last stage reads and writes the 2-byte low
    part, and with RK4 also reads U (4 B) for the two-sum (RK2's last stage
    reads U anyway)."""
    Np = (q + 1) * (q + 2) * (q + 3) // 6
    stages, extra = (4, 8.0) if q >= 2 else (2, 4.0)
    return extra * 6 * Np * K * members / stages


def bytes_per_dof_update(q: int, esize: int, members: int = 1) -> float:
    """Algorithmic HBM bytes per dof-update (one dof advanced one full step):
    the field passes of stage_bytes_per_element over the stages of a step,
    geometry and connectivity shared by the members of a batched launch."""
    Np = (q + 1) * (q + 2) * (q + 3) // 6
    stages = 4 if q >= 2 else 2
    field = stage_bytes_per_element(q, esize) - (40 * esize + 16)
    return stages * (field + (40 * esize + 16) / members) / (6 * Np)


def cpu_baseline(w, steps: int):
    """The FP64 oracle (as is) on a bounded sample: `steps` RK4 steps of the
    full mesh without source, timed on the host cores."""
    import numpy as np
    import psutil

    from oracle import dg, timestep
    p = dg.make_problem(w.xyz, w.tet, w.tags, w.q, w.eps, w.mu, w.sigma, omega=w.omega)
    M = timestep.n_steps(p)
    dt = 2 * math.pi / w.omega / M
    U = np.random.default_rng(0).standard_normal((p.K, 6, p.Np))
    proc = psutil.Process()
    c0 = proc.cpu_times()
    t0 = time.perf_counter()
    for m in range(steps):
        U, _ = timestep.rk4_step(p, m * dt, U, dt, False) if w.q > 1 else timestep.rk2_step(p, m * dt, U, dt, False)
    el = time.perf_counter() - t0
    c1 = proc.cpu_times()
    cores = (c1.user - c0.user + c1.system - c0.system) / el
    ndof = p.K * 6 * p.Np
    return {"value": ndof * steps / el, "unit": "dof-updates/s", "cores": round(cores, 2), "kind": "oracle",
            "sample": f"{steps} RK{'4' if w.q > 1 else '2'} step(s) of the full {p.K}-tet P{w.q} mesh "
                      f"({ndof} dofs), FP64 numpy oracle, {el:.1f} s"}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline_child(args):
    fn, w, steps = args
    return fn(w, steps)


def cpu_baseline_threads(fn, w, steps: int, threads: int) -> dict:
    """fn(w, steps) in a fresh process whose BLAS / OpenMP pools hold
    `threads` threads (the oracle unchanged; only the thread count differs)."""
    import concurrent.futures as cf
    import multiprocessing
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: str(threads) for k in keys})
    try:
        with cf.ProcessPoolExecutor(max_workers=1, mp_context=multiprocessing.get_context("spawn")) as ex:
            return ex.submit(_cpu_baseline_child, (fn, w, steps)).result()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def batched(a):
    """64 independent solves on the 12^3 x 6 = 10368-tet P2 mesh (omega in
    [2 pi, 6 pi], seeded centres and polarisations, eps = mu = 1), FP32 fields,
    advanced by one batched CMCG; value = aggregate dof-updates/s."""
    import torch

    from paper_2106_02858_amd import cmcg, inputs
    torch.cuda.set_device(0)
    ws = inputs.batched_members(n=12 if a.n == 20 else a.n, q=2, B=a.members)
    w0 = ws[0]
    mesh = cmcg.cmcg_mesh_create(w0.xyz, w0.tet, w0.tags)
    s = cmcg.cmcg_space_create(mesh, w0.q, cmcg.CMCG_FP32)
    nodes = cmcg.cmcg_space_nodes(s)
    probs = [cmcg.cmcg_problem_create(s, w.eps, w.mu, None, w.omega,
                                      inputs.gaussian_current(nodes, w.centre, w.width, w.pol)) for w in ws]
    info = cmcg.cmcg_space_info(s)
    opts = cmcg.cmcg_options_default(tol=a.tol, max_iter=2000, autotune=0 if a.no_autotune else 1)
    t_ref = [time.perf_counter()]

    def progress(it, rel):
        if it % 10 == 0:
            log(f"  iter {it} worst rel {rel:.3e} t {time.perf_counter() - t_ref[0]:.1f}s")
        return False

    opts.set_progress(progress)
    for _ in range(a.warmup):
        t_ref[0] = time.perf_counter()
        cmcg.cmcg_solve_batch(probs, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dof = 0.0
    for _ in range(a.steps):
        t_ref[0] = time.perf_counter()
        res = cmcg.cmcg_solve_batch(probs, opts)
        sts = [cmcg.cmcg_result_stats(r) for r in res]
        dof += sum(st["dof_updates"] for st in sts)
        log(f"batched solve: max iters {max(st['iters'] for st in sts)} seconds {sts[0]['seconds']:.2f}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    Ms = [st["steps"] for st in sts]
    out = {"metric": "DG dof-updates/s; CMCG time-to-1e-6 residual vs FP64 plain; p50/p99 latency",
           "value": dof / el, "unit": "dof-updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": el / a.steps * 1e3, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"batched: {a.members} solves on the {info['K']}-tet P2 mesh, omega in [2pi,6pi], "
                                  f"FP32 fields, CMCG to {a.tol:g} + filter", "members": a.members, "K": info["K"],
                      "q": 2, "steps_per_period_min": min(Ms), "steps_per_period_max": max(Ms),
                      "stage_variant": cmcg.cmcg_tune_resolve_stage(2, cmcg.CMCG_FP32, info["K"], len(probs)),
                      "autotuned": not a.no_autotune},
           "cmcg": {"iters_min": min(st["iters"] for st in sts), "iters_max": max(st["iters"] for st in sts),
                    "time_to_1e-6_all_members_s": max(st["seconds_to_1e6"] for st in sts),
                    "seconds": sts[0]["seconds"]},
           "hbm_job": job_roofline(dof / el, method_bytes_per_dof_update(2, 4, a.members))}
    if a.fp64_members > 0:
        # the plain FP64 form on the same problems: one solve after another
        s64 = cmcg.cmcg_space_create(mesh, w0.q, cmcg.CMCG_FP64)
        nodes64 = cmcg.cmcg_space_nodes(s64)
        o64 = cmcg.cmcg_options_default(tol=a.tol, max_iter=2000, autotune=0 if a.no_autotune else 1)
        t6, tall, it64 = [], [], []
        for b, w in enumerate(ws[:a.fp64_members]):
            p64 = cmcg.cmcg_problem_create(s64, w.eps, w.mu, None, w.omega,
                                           inputs.gaussian_current(nodes64, w.centre, w.width, w.pol))
            st = cmcg.cmcg_result_stats(cmcg.cmcg_solve(p64, o64))
            t6.append(st["seconds_to_1e6"])
            tall.append(st["seconds"])
            it64.append(st["iters"])
            if b % 16 == 15:
                log(f"fp64 member {b + 1}: time-to-1e-6 so far {sum(t6):.2f} s")
        out["fp64_plain"] = {"members": len(t6), "mode": "one plain FP64 solve after another",
                             "time_to_1e-6_sum_s": sum(t6), "seconds_sum": sum(tall),
                             "iters_min": min(it64), "iters_max": max(it64)}
        log(f"fp64 plain, {len(t6)} members one by one: time-to-1e-6 {sum(t6):.2f} s "
            f"(batched FP32: {out['cmcg']['time_to_1e-6_all_members_s']:.2f} s)")
    print(json.dumps(out), flush=True)


def job_roofline(rate: float, bpd: float) -> dict:
    """Whole-job HBM fraction: dof-updates/s x algorithmic bytes per dof-update
    (CG vector work and idle members count as time, not as bytes)."""
    gbs = rate * bpd / 1e9
    cp = stream_copy_gbs()
    return {"bytes_per_dof_update": bpd, "achieved_GBs": gbs, "peak_GBs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS,
            "copy_GBs": cp, "frac_of_copy": gbs / cp}


_COPY_GBS = []


def stream_copy_gbs(nbytes: int = 1 << 30) -> float:
    """Bandwidth of a plain device-to-device copy of 1 GiB (read + write
    bytes over the best of 5 timed copies): the practical HBM ceiling."""
    if _COPY_GBS:
        return _COPY_GBS[0]
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    best = float("inf")
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del x, y
    _COPY_GBS.append(2 * nbytes / best / 1e9)
    return _COPY_GBS[0]


def scatterer(a):
    """The 64^3 x 6 = 1572864-tet P2 dielectric-sphere scatterer (eps = 4 in
    the sphere of radius 1/4, omega = 8 pi, source width 0.03 at
    (0.15, 0.5, 0.5)), FP32 fields: a CMCG solve of --cg-iters iterations plus
    the filter period (its working set is far beyond the on-die caches), and
    the stage kernel's rate at this size."""
    import torch

    from paper_2106_02858_amd import cmcg, inputs
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = inputs.scatterer()
    mesh = cmcg.cmcg_mesh_create(w.xyz, w.tet, w.tags)
    s = cmcg.cmcg_space_create(mesh, w.q, cmcg.CMCG_FP32)
    nodes = cmcg.cmcg_space_nodes(s)
    jd = torch.tensor(inputs.gaussian_current(nodes, w.centre, w.width, w.pol), dtype=torch.float64, device=dev)
    p = cmcg.cmcg_problem_create_device(s, w.eps, w.mu, w.sigma, w.omega, jd)
    del jd, nodes
    info = cmcg.cmcg_space_info(s)
    K, Np = info["K"], info["Np"]
    opts = cmcg.cmcg_options_default(fixed_iters=a.cg_iters, autotune=0 if a.no_autotune else 1)
    M, dt = cmcg.cmcg_problem_steps(p, opts)
    log(f"scatterer K={K} Np={Np} M={M}")
    t_ref = [time.perf_counter()]

    def progress(it, rel):
        log(f"  iter {it} rel {rel:.3e} t {time.perf_counter() - t_ref[0]:.1f}s")
        return False

    opts.set_progress(progress)
    if not a.no_autotune:  # outside the timed region (the solve reuses the cached choice)
        v, us = cmcg.cmcg_autotune_stage(p, opts)
        log(f"autotuned stage variant {v}: us per launch {[round(u, 1) for u in us]}")
    U0 = torch.randn((K, 6, Np), dtype=torch.float64, device=dev) * 1e-3
    UT = torch.empty_like(U0)
    cmcg.cmcg_debug_period(p, U0, UT, 1, False, opts=opts)  # builds the period's graph
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = cmcg.cmcg_solve(p, opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = cmcg.cmcg_result_stats(r)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    cmcg.cmcg_debug_period(p, U0, UT, 1, False, opts=opts)
    ev1.record(stream)
    torch.cuda.synchronize()
    per_launch = ev0.elapsed_time(ev1) / 1e3 / (4 * M)
    bpl = method_bytes_per_launch(w.q, 4, K)
    achieved = bpl / per_launch / 1e9
    kname = STAGE_KERNEL[cmcg.cmcg_tune_resolve_stage(w.q, cmcg.CMCG_FP32, K)].format(q=w.q)
    out = {"metric": "DG dof-updates/s; CMCG time-to-1e-6 residual vs FP64 plain; p50/p99 latency",
           "value": st["dof_updates"] / el, "unit": "dof-updates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": el * 1e3, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"scatterer: 64^3x6 = {K} tets, P2, eps = 4 in the sphere |x - c| < 1/4 "
                                  f"(103392 tets), omega = 8 pi, source width 0.03 at (0.15,0.5,0.5); "
                                  f"CMCG {a.cg_iters} iterations + filter period", "K": K, "q": w.q,
                      "steps_per_period": M, "stage_variant": cmcg.cmcg_tune_resolve_stage(w.q, cmcg.CMCG_FP32, K),
                      "autotuned": not a.no_autotune},
           "cmcg": {"iters": st["iters"], "periods": st["periods"], "rel_res": st["rel_res"]},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname, K, MEASURED_TRAFFIC_Q2),
                        "kernel": kname,
                        "avg_launch_us": per_launch * 1e6, "bytes_per_launch": bpl,
                        "copy_GBs": stream_copy_gbs(), "frac_of_copy": achieved / stream_copy_gbs()},
           "hbm_job": job_roofline(st["dof_updates"] / el, method_bytes_per_dof_update(w.q, 4))}
    print(json.dumps(out), flush=True)


def stage2d_bytes_per_element(q: int, esize: int) -> float:
    """Algorithmic HBM bytes of one average 2-D stage launch per triangle: the
    field passes of stage_bytes_per_element over 3 components, the geometry
    (25 values) and connectivity (3 int32)."""
    Np = (q + 1) * (q + 2) // 2
    if q >= 2:
        per_dof = 72.0 / 4 if esize == 4 else 128.0 / 4
    else:
        per_dof = 24.0 / 2 if esize == 4 else 40.0 / 2
    return 3 * Np * per_dof + 25 * esize + 12


def cpu_baseline_2d(w, steps: int):
    """The 2-D FP64 oracle (as is) on a bounded sample: `steps` RK steps of
    the full mesh without source, timed on the host cores."""
    import numpy as np
    import psutil

    from oracle import dg2d, timestep
    p = dg2d.make_problem(w.xy, w.tri, w.tags, w.q, w.eps, w.mu, w.sigma, omega=w.omega)
    M = timestep.n_steps(p)
    dt = 2 * math.pi / w.omega / M
    U = np.random.default_rng(0).standard_normal((p.K, 3, p.Np))
    proc = psutil.Process()
    c0 = proc.cpu_times()
    t0 = time.perf_counter()
    for m in range(steps):
        U, _ = timestep.rk4_step(p, m * dt, U, dt, False) if w.q > 1 else timestep.rk2_step(p, m * dt, U, dt, False)
    el = time.perf_counter() - t0
    c1 = proc.cpu_times()
    ndof = p.K * 3 * p.Np
    return {"value": ndof * steps / el, "unit": "dof-updates/s", "cores": round((c1.user - c0.user + c1.system -
                                                                               c0.system) / el, 2),
            "kind": "oracle", "sample": f"{steps} RK{'4' if w.q > 1 else '2'} step(s) of the full {p.K}-triangle "
                                        f"P{w.q} mesh ({ndof} dofs), FP64 numpy 2-D oracle, {el:.1f} s"}


def trap2d_batch(a):
    """--members2d B solves of the 2-D dipole-in-trap problem advanced by one
    batched CMCG (grid.y = member): the dipole at B seeded points of the trap,
    FP32 fields, shared mesh and media; value = aggregate dof-updates/s."""
    import numpy as np
    import torch

    from paper_2106_02858_amd import cmcg, inputs
    torch.cuda.set_device(0)
    w = inputs.trap2d(a.n2d, 3, a.trap)
    mesh = cmcg.cmcg_mesh2d_create(w.xy, w.tri, w.tags)
    s = cmcg.cmcg_space_create(mesh, w.q, cmcg.CMCG_FP32)
    nodes = cmcg.cmcg_space_nodes(s)
    info = cmcg.cmcg_space_info(s)
    K, Np = info["K"], info["Np"]
    rng = np.random.default_rng(12)
    probs = []
    for _ in range(a.members2d):
        r, t = 0.4 * math.sqrt(rng.uniform()), rng.uniform(0, 2 * math.pi)   # inside |x| < 0.4
        w.centre = np.array([r * math.cos(t), r * math.sin(t)])
        probs.append(cmcg.cmcg_problem_create(s, w.eps, w.mu, None, w.omega, inputs.current_2d(w, nodes)))
    opts = cmcg.cmcg_options_default(tol=a.tol, max_iter=3000)
    M, _ = cmcg.cmcg_problem_steps(probs[0], opts)
    for _ in range(a.warmup):
        cmcg.cmcg_solve_batch(probs, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        res = cmcg.cmcg_solve_batch(probs, opts)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / a.steps
    sts = [cmcg.cmcg_result_stats(r) for r in res]
    dof = sum(st["dof_updates"] for st in sts)
    log(f"2-D trap batch of {a.members2d}: K={K} M={M}, iterations {min(st['iters'] for st in sts)}-"
        f"{max(st['iters'] for st in sts)}, {el:.3f} s")
    bpd = bytes_per_dof_update_2d(3, 4, a.members2d)
    out = {"metric": "DG dof-updates/s; CMCG time-to-1e-6 residual vs FP64 plain; p50/p99 latency",
           "value": dof / el, "unit": "dof-updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": el * 1e3, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"2-D TM dipole in a trapping {a.trap}: {a.members2d} dipole positions (seed 12) "
                                  f"batched on the {K}-triangle P3 mesh, omega = {w.omega / math.pi:.0f} pi; "
                                  f"CMCG to {a.tol:g}", "K": K, "q": 3, "members": a.members2d,
                      "steps_per_period": M},
           "cmcg": {"iters_min": min(st["iters"] for st in sts), "iters_max": max(st["iters"] for st in sts),
                    "all_converged": all(st["status"] == cmcg.CMCG_OK for st in sts), "seconds": el},
           "hbm_job": job_roofline(dof / el, bpd)}
    print(json.dumps(out), flush=True)


def bytes_per_dof_update_2d(q: int, esize: int, members: int = 1) -> float:
    """Algorithmic HBM bytes per 2-D dof-update: the field passes of
    stage2d_bytes_per_element over the stages of a step, geometry and
    connectivity shared by the members of a batched launch."""
    Np = (q + 1) * (q + 2) // 2
    stages = 4 if q >= 2 else 2
    field = stage2d_bytes_per_element(q, esize) - (25 * esize + 12)
    return stages * (field + (25 * esize + 12) / members) / (3 * Np)


def trap2d_bench(a):
    """The paper's own 2-D workload (dipole in a trapping body, Section 6),
    transverse-magnetic fields on triangles, P3: CMCG to --tol with FP32
    fields, timed, beside the plain FP64 solve; the 2-D stage kernel's
    launch time over a period (HIP events on the solve's stream)."""
    import numpy as np
    import torch

    from paper_2106_02858_amd import cmcg, inputs
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = inputs.trap2d(a.n2d, 3, a.trap)
    mesh = cmcg.cmcg_mesh2d_create(w.xy, w.tri, w.tags)

    def make(prec):
        s = cmcg.cmcg_space_create(mesh, w.q, prec)
        j = inputs.current_2d(w, cmcg.cmcg_space_nodes(s))
        return s, cmcg.cmcg_problem_create(s, w.eps, w.mu, None, w.omega, j)

    res = {}
    for prec in (cmcg.CMCG_FP32, cmcg.CMCG_FP64):
        s, p = make(prec)
        info = cmcg.cmcg_space_info(s)
        K, Np = info["K"], info["Np"]
        opts = cmcg.cmcg_options_default(tol=a.tol, max_iter=3000)
        M, dt = cmcg.cmcg_problem_steps(p, opts)
        U0 = torch.randn((K, 3, Np), dtype=torch.float64, device=dev) * 1e-3
        UT = torch.empty_like(U0)
        cmcg.cmcg_debug_period(p, U0, UT, 1, False, opts=opts)  # builds the period's graph (untimed)
        for _ in range(a.warmup):
            cmcg.cmcg_solve(p, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            r = cmcg.cmcg_solve(p, opts)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / a.steps
        st = cmcg.cmcg_result_stats(r)
        stream = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(a.kernel_periods):
            cmcg.cmcg_debug_period(p, U0, UT, 1, False, opts=opts)
        ev1.record(stream)
        torch.cuda.synchronize()
        per_launch = ev0.elapsed_time(ev1) / 1e3 / (a.kernel_periods * 4 * M)
        res[prec] = dict(el=el, st=st, K=K, Np=Np, M=M, per_launch=per_launch,
                         rate=st["dof_updates"] / st["seconds"] if st["seconds"] > 0 else 0.0)
        log(f"2-D trap prec={prec} K={K} M={M}: {st['iters']} iters, {el:.3f} s, stage launch "
            f"{per_launch * 1e6:.2f} us (includes the field conversions of the period)")
    f32, f64 = res[cmcg.CMCG_FP32], res[cmcg.CMCG_FP64]
    K = f32["K"]
    bpe = stage2d_bytes_per_element(3, 4)
    achieved = bpe * K / f32["per_launch"] / 1e9
    out = {"metric": "DG dof-updates/s; CMCG time-to-1e-6 residual vs FP64 plain; p50/p99 latency",
           "value": f32["st"]["dof_updates"] / f32["el"], "unit": "dof-updates/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": f32["el"] * 1e3, "higher_is_better": True, "scaling": "strong",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"2-D TM dipole in a trapping {a.trap} (Section 6): (-1,1)^2 Cartesian "
                                  f"{a.n2d}x{a.n2d} mesh, {K} triangles, P3, eps = 4 in the trap, impedance walls, "
                                  f"omega = {w.omega / math.pi:.0f} pi, Gaussian j (s = 0.05); CMCG to {a.tol:g}",
                      "K": K, "q": 3, "steps_per_period": f32["M"]},
           "cmcg": {"iters": f32["st"]["iters"], "periods": f32["st"]["periods"], "rel_res": f32["st"]["rel_res"],
                    "seconds": f32["el"], "fp64_iters": f64["st"]["iters"], "fp64_seconds": f64["el"],
                    "speedup_vs_fp64": f64["el"] / f32["el"]},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS,
                        "traffic": measured_traffic("k_stage2d<float,3,true>", K, MEASURED_TRAFFIC_2D, "kernels2d.hip"),
                        "kernel": "k_stage2d<float,3,true>",
                        "avg_launch_us": f32["per_launch"] * 1e6, "bytes_per_launch": bpe * K,
                        "fp64_avg_launch_us": f64["per_launch"] * 1e6}}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline_2d(w, max(a.cpu_steps, 20))
    print(json.dumps(out), flush=True)


def curves2d(a):
    """CMCG against the limiting-amplitude iteration (FW) on the paper's 2-D
    experiments (Section 6), FP64 fields: error of the filtered field after a
    given number of simulated periods, relative to the CMCG solution at
    1e-10 (eps-mu norm; Section 6 measures the trapping-medium case the same
    way).  CMCG after k iterations has simulated 2 k + 3 periods (two for
    Algorithm 1, two per iteration, one filter period); FW after L periods
    has simulated L."""
    import torch

    from paper_2106_02858_amd import cmcg, inputs
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    exps = {
        "cavity": lambda: inputs.cavity2d(32, 1, 3 * math.sqrt(2) * math.pi, 1 / 8),
        "cavity_near": lambda: inputs.cavity2d(32, 1, 3 * math.sqrt(2) * math.pi, 1 / 64),
        "planewave": lambda: inputs.planewave2d(32, 1, 10 * math.pi),
        "waveguide": lambda: inputs.waveguide2d(32, 3, 6 * math.pi),
        "trap": lambda: inputs.trap2d(30, 3, "square"),
    }
    w = exps[a.exp]()
    mesh = cmcg.cmcg_mesh2d_create(w.xy, w.tri, w.tags)
    s = cmcg.cmcg_space_create(mesh, w.q, cmcg.CMCG_FP64)
    info = cmcg.cmcg_space_info(s)
    K, Np = info["K"], info["Np"]
    nodes = cmcg.cmcg_space_nodes(s)
    g = None
    if w.source in ("planewave", "wallwave"):
        import numpy as np
        # edge nodes in the library's node order (edge f opposite vertex f, from its lower vertex)
        q = w.q
        lab = [(i, j) for j in range(q + 1) for i in range(q + 1 - j)]
        idx = {l: n for n, l in enumerate(lab)}
        edges = [[idx[(q - k, k)] for k in range(q + 1)], [idx[(0, k)] for k in range(q + 1)],
                 [idx[(k, 0)] for k in range(q + 1)]]
        fp = nodes[:, np.array(edges)]
        fn = inputs.planewave_boundary_data if w.source == "planewave" else inputs.waveguide_boundary_data
        g = fn(w, fp)
    p = cmcg.cmcg_problem_create(s, w.eps, w.mu, None, w.omega, inputs.current_2d(w, nodes), g)
    M, _ = cmcg.cmcg_problem_steps(p)

    def field(r):
        fr = torch.zeros((K, 3, Np), dtype=torch.float64, device=dev)
        fi = torch.zeros_like(fr)
        cmcg.cmcg_result_filtered_device(r, fr, fi)
        return fr, fi

    t0 = time.perf_counter()
    ref = cmcg.cmcg_solve(p, cmcg.cmcg_options_default(tol=1e-10, max_iter=4000))
    st = cmcg.cmcg_result_stats(ref)
    Rr, Ri = field(ref)
    den = cmcg.cmcg_debug_dot(p, Rr, Rr) + cmcg.cmcg_debug_dot(p, Ri, Ri)
    log(f"{a.exp}: K={K} q={w.q} M={M}; reference CMCG {st['iters']} iterations ({st['status']}) "
        f"{time.perf_counter() - t0:.1f}s")

    def err(r):
        fr, fi = field(r)
        dr, di = fr - Rr, fi - Ri
        return math.sqrt((cmcg.cmcg_debug_dot(p, dr, dr) + cmcg.cmcg_debug_dot(p, di, di)) / den)

    cm, fw = [], []
    k = 1
    while 2 * k + 3 <= a.max_periods and k <= st["iters"]:
        cm.append([2 * k + 3, err(cmcg.cmcg_solve(p, cmcg.cmcg_options_default(fixed_iters=k)))])
        k *= 2
    L = 2
    while L <= a.max_periods:
        fw.append([L, err(cmcg.cmcg_fw_solve(p, cmcg.cmcg_options_default(fixed_iters=L)))])
        L *= 2
    for (pc, e1) in cm:
        log(f"  CMCG {pc:5d} periods: {e1:.3e}")
    for (pf, e2) in fw:
        log(f"  FW   {pf:5d} periods: {e2:.3e}")
    out = {"metric": "relative error of the filtered field against the CMCG solution at 1e-10 vs simulated periods",
           "value": None, "unit": "curves", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": (time.perf_counter() - t0) * 1e3, "higher_is_better": False, "scaling": "strong",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"2-D {a.exp} ({w.name}), {K} triangles, P{w.q}, {M} steps per period",
                      "reference_iters": st["iters"], "reference_periods": st["periods"]},
           "curves": {"cmcg": cm, "fw": fw}}
    print(json.dumps(out), flush=True)


def fw_compare(a):
    """CMCG against the limiting-amplitude (FW) iteration on the 48000-tet P3
    problem with FP32 fields: CMCG to --tol, then FW for 1/8, 1/4, 1/2 and 1
    times the periods CMCG used; each FW result is compared with the CMCG solution
    (relative eps-mu norm of the filtered fields), cost in periods and time.
    With impedance walls also CMCG after 4, 8 and 16 run-up periods."""
    import torch

    from paper_2106_02858_amd import cmcg, inputs
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = inputs.large_single(n=a.n, q=a.q,
                            boundary_tag=inputs.TAG_PEC if a.fw_walls == "pec" else inputs.TAG_IMPEDANCE)
    mesh = cmcg.cmcg_mesh_create(w.xyz, w.tet, w.tags)
    s = cmcg.cmcg_space_create(mesh, w.q, cmcg.CMCG_FP32)
    nodes = cmcg.cmcg_space_nodes(s)
    jd = torch.tensor(inputs.gaussian_current(nodes, w.centre, w.width, w.pol), dtype=torch.float64, device=dev)
    p = cmcg.cmcg_problem_create_device(s, w.eps, w.mu, w.sigma, w.omega, jd)
    info = cmcg.cmcg_space_info(s)
    K, Np = info["K"], info["Np"]

    def fields(r):
        f = [torch.empty((K, 6, Np), dtype=torch.float64, device=dev) for _ in range(2)]
        cmcg.cmcg_result_filtered_device(r, *f)
        return f

    t_ref = [time.perf_counter()]

    def progress(it, rel):
        if it % 20 == 0:
            log(f"  cmcg iter {it} rel {rel:.3e} t {time.perf_counter() - t_ref[0]:.1f}s")
        return False

    oc = cmcg.cmcg_options_default(tol=a.tol, max_iter=2000)
    oc.set_progress(progress)
    rc = cmcg.cmcg_solve(p, oc)
    stc = cmcg.cmcg_result_stats(rc)
    Fc = fields(rc)
    den = sum(cmcg.cmcg_debug_dot(p, x, x) for x in Fc)
    log(f"cmcg: {stc['iters']} iterations, {stc['periods']} periods, {stc['seconds']:.2f} s")
    rows = []
    for frac in ((0.125, 0.25, 0.5, 1.0) if a.fw_walls == "impedance" else (0.5, 1.0, 2.0, 4.0)):
        L = max(2, int(round(frac * stc["periods"])))
        t0 = time.perf_counter()
        of = cmcg.cmcg_options_default(fixed_iters=L)
        t_ref[0] = time.perf_counter()

        def fw_progress(it, rel):
            if it % 200 == 0:
                log(f"  fw period {it} change {rel:.3e} t {time.perf_counter() - t_ref[0]:.1f}s")
            return False

        of.set_progress(fw_progress)
        rf = cmcg.cmcg_fw_solve(p, of)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        d = [x - y for x, y in zip(fields(rf), Fc)]
        err = math.sqrt(sum(cmcg.cmcg_debug_dot(p, x, x) for x in d) / den)
        last = float(cmcg.cmcg_result_history(rf)[-1])
        rows.append({"periods": L, "seconds": el, "rel_diff_to_cmcg": err, "last_rel_change": last})
        log(f"fw {L} periods: {el:.2f} s, rel. difference to CMCG {err:.3e}, last change {last:.3e}")
    # CMCG after a run-up of l limiting-amplitude periods (open problem only:
    # in a closed cavity the run-up state does not approach the solution).
    # The stop rule is relative to the first residual, which the run-up makes
    # smaller: each run-up solve stops at the same absolute residual as the
    # zero-start one (its ||R_0|| is read from an untimed solve with no CG step).
    runup_rows = []
    for l in ((4, 8, 16) if a.fw_walls == "impedance" else ()):
        res0 = cmcg.cmcg_result_stats(cmcg.cmcg_solve(p, cmcg.cmcg_options_default(max_iter=0, runup=l)))["res0"]
        tol_l = a.tol * stc["res0"] / res0
        o_r = cmcg.cmcg_options_default(tol=tol_l, max_iter=2000, runup=l)
        r_r = cmcg.cmcg_solve(p, o_r)
        st_r = cmcg.cmcg_result_stats(r_r)
        d = [x - y for x, y in zip(fields(r_r), Fc)]
        err = math.sqrt(sum(cmcg.cmcg_debug_dot(p, x, x) for x in d) / den)
        runup_rows.append({"runup": l, "tol": tol_l, "iters": st_r["iters"], "periods": st_r["periods"],
                           "seconds": st_r["seconds"], "rel_diff_to_cmcg": err})
        log(f"cmcg after {l} run-up periods: {st_r['iters']} iterations, {st_r['periods']} periods, "
            f"{st_r['seconds']:.2f} s, rel. difference to CMCG from zero {err:.3e}")
    out = {"metric": "DG dof-updates/s; CMCG time-to-1e-6 residual vs FP64 plain; p50/p99 latency",
           "value": stc["dof_updates"] / stc["seconds"], "unit": "dof-updates/s", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": stc["seconds"] * 1e3, "higher_is_better": True, "scaling": "strong",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"CMCG vs limiting amplitude (FW) on the 48000-tet P3 problem with "
                                  f"{a.fw_walls} walls, FP32 fields, CMCG to {a.tol:g}"},
           "cmcg": {"iters": stc["iters"], "periods": stc["periods"], "seconds": stc["seconds"]},
           "fw": rows, "cmcg_after_runup": runup_rows}
    print(json.dumps(out), flush=True)


def lts_compare(a):
    """Local time stepping against global stepping on a locally refined mesh:
    the unit cube with --lts-n cells per axis whose middle x-cell is split so
    that two of its layers are --lts-r times thinner than a cell (a slab of
    elements with a much shorter CFL step), P2, eps = mu = 1, omega = 4 pi,
    impedance walls, Gaussian source at the centre.  Both CMCG solves to --tol with FP64 fields: time per period
    (forward, HIP events) and per solve, and the difference of the two
    filtered fields (each carries its own time-discretisation error)."""
    import numpy as np
    import torch

    from paper_2106_02858_amd import cmcg, inputs
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n, r = a.lts_n, a.lts_r
    c = n // 2
    # the middle x-cell split into two thin cells of width 1/(r n) around its
    # centre and two ordinary ones
    mid = np.array([c, c + 0.5 - 1.0 / r, c + 0.5, c + 0.5 + 1.0 / r]) / n
    xs = np.concatenate([np.arange(c) / n, mid, np.arange(c + 1, n + 1) / n])
    ys = np.arange(n + 1) / n
    xyz, tet, tags = inputs.graded_cube_mesh(xs, ys, ys)
    K = tet.shape[0]
    mesh = cmcg.cmcg_mesh_create(xyz, tet, tags)
    s = cmcg.cmcg_space_create(mesh, 2, cmcg.CMCG_FP64)
    nodes = cmcg.cmcg_space_nodes(s)
    omega = 4 * math.pi
    jd = torch.tensor(inputs.gaussian_current(nodes, (0.5, 0.5, 0.5), 0.1, 2), dtype=torch.float64, device=dev)
    p = cmcg.cmcg_problem_create_device(s, np.ones(K), np.ones(K), None, omega, jd)
    info = cmcg.cmcg_space_info(s)
    Np = info["Np"]
    stream = torch.cuda.current_stream()
    U0 = torch.randn((K, 6, Np), dtype=torch.float64, device=dev) * 1e-3
    UT = torch.empty_like(U0)
    rows = {}
    fields = {}
    for name, ratio in (("global", 0), ("lts", a.lts_m)):
        o = cmcg.cmcg_options_default(tol=a.tol, max_iter=2000, lts_ratio=ratio, autotune=0 if a.no_autotune else 1)
        M, dt = cmcg.cmcg_problem_steps(p, o)
        cmcg.cmcg_debug_period(p, U0, UT, 1, False, opts=o)  # warm-up (graphs, buffers)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        cmcg.cmcg_debug_period(p, U0, UT, 1, False, opts=o)
        ev1.record(stream)
        torch.cuda.synchronize()
        per_fwd = ev0.elapsed_time(ev1) / 1e3
        ev0.record(stream)
        cmcg.cmcg_debug_period(p, U0, UT, -1, False, opts=o)
        ev1.record(stream)
        torch.cuda.synchronize()
        per_bwd = ev0.elapsed_time(ev1) / 1e3
        # the same periods from eager launches (no graph replay)
        oe = cmcg.cmcg_options_default(tol=a.tol, max_iter=2000, lts_ratio=ratio, use_graph=0,
                                       autotune=0 if a.no_autotune else 1)
        eager = []
        for direction in (1, -1):
            ev0.record(stream)
            cmcg.cmcg_debug_period(p, U0, UT, direction, False, opts=oe)
            ev1.record(stream)
            torch.cuda.synchronize()
            eager.append(ev0.elapsed_time(ev1) / 1e3)
        res = cmcg.cmcg_solve(p, o)
        st = cmcg.cmcg_result_stats(res)
        f = [torch.empty((K, 6, Np), dtype=torch.float64, device=dev) for _ in range(2)]
        cmcg.cmcg_result_filtered_device(res, *f)
        fields[name] = f
        rows[name] = {"steps_per_period": M, "dt": dt, "period_forward_s": per_fwd, "period_backward_s": per_bwd,
                      "period_forward_eager_s": eager[0], "period_backward_eager_s": eager[1],
                      "iters": st["iters"], "rel_res": st["rel_res"], "seconds": st["seconds"],
                      "time_to_1e-6_s": st["seconds_to_1e6"]}
        if ratio > 1:
            rows[name]["fine_elements"] = int(cmcg.cmcg_problem_lts_fine(p, K, o).sum())
            rows[name]["substeps"] = ratio
        log(f"{name}: M = {M}, period fwd {per_fwd * 1e3:.2f} ms bwd {per_bwd * 1e3:.2f} ms "
            f"(eager {eager[0] * 1e3:.2f} / {eager[1] * 1e3:.2f} ms), "
            f"{st['iters']} iterations, {st['seconds']:.2f} s")
    d = [x - y for x, y in zip(fields["lts"], fields["global"])]
    den = sum(cmcg.cmcg_debug_dot(p, x, x) for x in fields["global"])
    diff = math.sqrt(sum(cmcg.cmcg_debug_dot(p, x, x) for x in d) / den)
    g, l = rows["global"], rows["lts"]
    out = {"metric": "CMCG time with local time stepping vs global stepping on a locally refined mesh",
           "value": g["seconds"] / l["seconds"], "unit": "speedup", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": l["seconds"] * 1e3, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"unit cube, {n} cells per axis, the middle x-cell split into {r} (a thin slab), "
                                  f"{K} tets, P2, omega = 4 pi, impedance walls; CMCG to {a.tol:g}, FP64 fields",
                      "K": K, "q": 2},
           "global": g, "lts": l, "filtered_rel_diff": diff,
           "period_speedup": g["period_forward_s"] / l["period_forward_s"]}
    print(json.dumps(out), flush=True)


def served(a):
    """The request stream (n in {8,12,16,24}, q in {1,2,3}, omega in [2pi,8pi],
    eps per cube in {1,2,4}, Poisson arrivals) through the serving engine."""
    import numpy as np
    import torch

    from paper_2106_02858_amd import cmcg, inputs, serving
    torch.cuda.set_device(0)
    reqs = inputs.serving_stream(n_requests=2000, rate=a.rate)[: a.requests]
    fp64 = a.serve_precision == "fp64"
    out = serving.serve(reqs, budget_bytes=int(a.budget_gb * 2 ** 30), max_slots=a.slots, tol=a.tol,
                        precision=cmcg.CMCG_FP64 if fp64 else cmcg.CMCG_FP32, log=log, cobatch=a.cobatch,
                        cobatch_max_elements=a.cobatch_max_k or None)
    svc = np.array([r["done"] - r["admitted"] for r in out["records"]])
    res = {"metric": "DG dof-updates/s; CMCG time-to-1e-6 residual vs FP64 plain; p50/p99 latency",
           "value": out["dof_updates_per_s"], "unit": "dof-updates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": out["elapsed"] * 1e3, "higher_is_better": True, "scaling": "strong",
           "vs_baseline": None, "dtype": "f64" if fp64 else "f32", "data": "synthetic",
           "config": {"workload": f"serving: first {a.requests} requests of the 2000-request Poisson stream at "
                                  f"{a.rate:g} req/s (n in 8,12,16,24; q in 1,2,3), {a.slots} slots, "
                                  f"{a.budget_gb:g} GB budget, CMCG to {a.tol:g}, "
                                  f"{'plain FP64' if fp64 else 'FP32'} fields, co-batching up to {a.cobatch}"
                                  + (f" (spaces of at most {a.cobatch_max_k} elements)" if a.cobatch_max_k else "")},
           "serving": {**{k: out[k] for k in ("completed", "elapsed", "throughput", "p50", "p99", "offered_rate",
                                              "engine_steps")},
                       "co_batched_requests": sum(1 for r in out["records"] if r["members"] > 1),
                       "service_p50": float(np.percentile(svc, 50)), "service_p99": float(np.percentile(svc, 99))}}
    byts = sum(r["dof_updates"] * method_bytes_per_dof_update(r["q"], 8 if fp64 else 4) for r in out["records"])
    res["hbm_job"] = job_roofline(out["dof_updates_per_s"], byts / max(1.0, sum(r["dof_updates"] for r in out["records"])))
    print(json.dumps(res), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "single-GPU implementation: --gpus must be 1"}))
        sys.exit(2)
    if a.workload == "batched":
        batched(a)
        return
    if a.workload == "serving":
        served(a)
        return
    if a.workload == "scatterer":
        scatterer(a)
        return
    if a.workload == "curves2d":
        curves2d(a)
        return
    if a.workload == "trap2d":
        if a.members2d > 1:
            trap2d_batch(a)
        else:
            trap2d_bench(a)
        return
    if a.workload == "fw":
        fw_compare(a)
        return
    if a.workload == "lts":
        lts_compare(a)
        return
    import numpy as np
    import torch

    from paper_2106_02858_amd import cmcg, inputs

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = inputs.large_single(n=a.n, q=a.q)
    mesh = cmcg.cmcg_mesh_create(w.xyz, w.tet, w.tags)

    def make(prec):
        s = cmcg.cmcg_space_create(mesh, w.q, prec)
        nodes = cmcg.cmcg_space_nodes(s)
        j = inputs.gaussian_current(nodes, w.centre, w.width, w.pol)
        jd = torch.tensor(j, dtype=torch.float64, device=dev)
        p = cmcg.cmcg_problem_create_device(s, w.eps, w.mu, w.sigma, w.omega, jd)
        return s, p

    s32, p32 = make(cmcg.CMCG_FP32)
    info = cmcg.cmcg_space_info(s32)
    K, Np, ndof = info["K"], info["Np"], info["ndof"]
    opts = cmcg.cmcg_options_default(tol=a.tol, max_iter=2000, autotune=0 if a.no_autotune else 1)
    M, dt = cmcg.cmcg_problem_steps(p32, opts)
    stream = torch.cuda.current_stream()

    log(f"K={K} Np={Np} ndof={ndof} M={M}")
    t_ref = [time.perf_counter()]

    def progress(it, rel):
        if it % 10 == 0:
            log(f"  iter {it} rel {rel:.3e} t {time.perf_counter() - t_ref[0]:.1f}s")
        return False

    opts.set_progress(progress)
    for _ in range(a.warmup):
        t_ref[0] = time.perf_counter()
        r = cmcg.cmcg_solve(p32, opts)
        log(f"warmup solve: {cmcg.cmcg_result_stats(r)}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dof_updates = 0.0
    stats = []
    for _ in range(a.steps):
        t_ref[0] = time.perf_counter()
        r = cmcg.cmcg_solve(p32, opts)
        st = cmcg.cmcg_result_stats(r)
        stats.append(st)
        dof_updates += st["dof_updates"]
        log(f"timed solve: {st}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = dof_updates / elapsed

    # dominant kernel: average stage-launch duration from HIP events around
    # whole homogeneous periods (4 M stage launches each) on the same stream
    U0 = torch.randn((K, 6, Np), dtype=torch.float64, device=dev) * 1e-3
    UT = torch.empty_like(U0)
    cmcg.cmcg_debug_period(p32, U0, UT, 1, False, opts=opts)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(a.kernel_periods):
        cmcg.cmcg_debug_period(p32, U0, UT, 1, False, opts=opts)
    ev1.record(stream)
    torch.cuda.synchronize()
    per_launch_s = ev0.elapsed_time(ev1) / 1e3 / (a.kernel_periods * 4 * M)
    bpl = method_bytes_per_launch(w.q, 4, K)
    kname = STAGE_KERNEL[cmcg.cmcg_tune_resolve_stage(w.q, cmcg.CMCG_FP32, K)].format(q=w.q)
    achieved = bpl / per_launch_s / 1e9

    out = {
        "metric": "DG dof-updates/s; CMCG time-to-1e-6 residual vs FP64 plain; p50/p99 latency",
        "value": value,
        "unit": "dof-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"unit cube {a.n}^3x6 = {K} tets, P{w.q}, eps per cube in {{1,2,4}} (seed 2), "
                               f"mu=1, omega=4pi, impedance boundary, Gaussian e_z source width 0.05; "
                               f"CMCG to rel. residual {a.tol:g} + filter period",
                   "K": K, "q": w.q, "ndof": ndof, "steps_per_period": M, "fields": "fp32",
                   "cg": "fp64", "stage_variant": cmcg.cmcg_tune_resolve_stage(w.q, cmcg.CMCG_FP32, K),
                   "autotuned": not a.no_autotune},
        "cmcg": {"iters": stats[-1]["iters"], "periods": stats[-1]["periods"],
                 "rel_res": stats[-1]["rel_res"], "seconds": stats[-1]["seconds"],
                 "time_to_1e-6_fp32_s": stats[-1]["seconds_to_1e6"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname, K),
                     "kernel": kname,
                     "avg_launch_us": per_launch_s * 1e6,
                     "bytes_per_launch": bpl,
                     "bytes_per_dof_update": method_bytes_per_dof_update(w.q, 4),
                     "compensation_overhead_bytes_per_launch": compensation_bytes_per_launch(w.q, K),
                     "implementation_bytes_per_launch": stage_bytes_per_element(w.q, 4) * K,
                     "copy_GBs": stream_copy_gbs(), "frac_of_copy": achieved / stream_copy_gbs()},
    }
    if not a.no_fp64:
        s64, p64 = make(cmcg.CMCG_FP64)
        t_ref[0] = time.perf_counter()
        r64 = cmcg.cmcg_solve(p64, opts)
        st64 = cmcg.cmcg_result_stats(r64)
        log(f"fp64 solve: {st64}")
        out["cmcg"]["time_to_1e-6_fp64_s"] = st64["seconds_to_1e6"]
        out["cmcg"]["iters_fp64"] = st64["iters"]
        # FP32-field result against the FP64 result (relative eps,mu norm via the library's inner product)
        f32 = [torch.empty((K, 6, Np), dtype=torch.float64, device=dev) for _ in range(2)]
        f64 = [torch.empty((K, 6, Np), dtype=torch.float64, device=dev) for _ in range(2)]
        cmcg.cmcg_result_filtered_device(r, *f32)
        cmcg.cmcg_result_filtered_device(r64, *f64)
        d = [x - y for x, y in zip(f32, f64)]
        num = sum(cmcg.cmcg_debug_dot(p64, x, x) for x in d)
        den = sum(cmcg.cmcg_debug_dot(p64, x, x) for x in f64)
        out["cmcg"]["fp32_vs_fp64_rel_l2"] = math.sqrt(num / den)
        # the plain FP64 path's stage kernel (the variant its autotuned solve kept)
        ev0.record(stream)
        for _ in range(a.kernel_periods):
            cmcg.cmcg_debug_period(p64, U0, UT, 1, False, opts=opts)
        ev1.record(stream)
        torch.cuda.synchronize()
        pl64 = ev0.elapsed_time(ev1) / 1e3 / (a.kernel_periods * 4 * M)
        bpl64 = method_bytes_per_launch(w.q, 8, K)
        v64 = cmcg.cmcg_tune_resolve_stage(w.q, cmcg.CMCG_FP64, K)
        out["roofline_fp64"] = {"workload": f"the same {K}-tet P{w.q} problem with FP64 fields",
                                "bound": "hbm", "achieved": bpl64 / pl64 / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": bpl64 / pl64 / 1e9 / HBM_PEAK_GBS,
                                "kernel": STAGE_KERNEL64[v64].format(q=w.q), "avg_launch_us": pl64 * 1e6,
                                "bytes_per_launch": bpl64, "bytes_per_dof_update": method_bytes_per_dof_update(w.q, 8),
                                "traffic": measured_traffic(STAGE_KERNEL64[v64].format(q=w.q), K,
                                                            MEASURED_TRAFFIC_FP64)}
        log(f"fp64 stage launch {pl64 * 1e6:.1f} us ({out['roofline_fp64']['kernel']})")
    del s32, p32, r
    if not a.no_extra:
        # the stage kernel where the working set exceeds the on-die caches, the
        # batched launch with every member active, and a short served stream
        out["roofline_scatterer"] = scatterer_kernel(a)
        out["roofline_batched"] = batched_kernel(a)
        out["serving"] = serving_short(a, 1)
    if not a.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_steps)
        # the same oracle on one thread (half the sample: the same per-step rate)
        log("cpu baseline, one thread")
        one = cpu_baseline_threads(cpu_baseline, w, max(1, a.cpu_steps // 2), 1)
        out["cpu_baseline"]["single_thread"] = {k: one[k] for k in ("value", "cores", "sample")}
        out["cpu_baseline"]["cpu_model"] = _cpu_model()
        out["cpu_baseline"]["host_threads"] = os.cpu_count()
    print(json.dumps(out), flush=True)


def _free_device():
    import gc

    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def scatterer_kernel(a) -> dict:
    """Stage-launch roofline on the 1,572,864-tet P2 scatterer (FP32 fields;
    its field vectors far exceed the 256 MB Infinity Cache): HIP events around
    one homogeneous period (4 M launches) on the launch stream."""
    import torch

    from paper_2106_02858_amd import cmcg, inputs
    _free_device()
    dev = torch.device("cuda:0")
    w = inputs.scatterer()
    mesh = cmcg.cmcg_mesh_create(w.xyz, w.tet, w.tags)
    s = cmcg.cmcg_space_create(mesh, w.q, cmcg.CMCG_FP32)
    jd = torch.tensor(inputs.gaussian_current(cmcg.cmcg_space_nodes(s), w.centre, w.width, w.pol),
                      dtype=torch.float64, device=dev)
    p = cmcg.cmcg_problem_create_device(s, w.eps, w.mu, w.sigma, w.omega, jd)
    del jd
    K, Np = w.K, 10
    opts = cmcg.cmcg_options_default()
    if not a.no_autotune:
        v, us = cmcg.cmcg_autotune_stage(p, opts)
        log(f"scatterer: autotuned variant {v}, us per launch {[round(u, 1) for u in us]}")
    M, _ = cmcg.cmcg_problem_steps(p, opts)
    U0 = torch.randn((K, 6, Np), dtype=torch.float64, device=dev) * 1e-3
    UT = torch.empty_like(U0)
    cmcg.cmcg_debug_period(p, U0, UT, 1, False, opts=opts)  # builds the period's graph
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    cmcg.cmcg_debug_period(p, U0, UT, 1, False, opts=opts)
    ev1.record(stream)
    torch.cuda.synchronize()
    per_launch = ev0.elapsed_time(ev1) / 1e3 / (4 * M)
    bpl = method_bytes_per_launch(w.q, 4, K)
    achieved = bpl / per_launch / 1e9
    kname = STAGE_KERNEL[cmcg.cmcg_tune_resolve_stage(w.q, cmcg.CMCG_FP32, K)].format(q=w.q)
    log(f"scatterer stage launch {per_launch * 1e6:.1f} us = {achieved:.0f} GB/s ({kname})")
    del p, s, mesh, U0, UT
    _free_device()
    return {"workload": f"scatterer: 64^3x6 = {K} tets, P2, FP32 fields, one homogeneous period of {M} steps",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "kernel": kname, "avg_launch_us": per_launch * 1e6,
            "bytes_per_launch": bpl, "bytes_per_dof_update": method_bytes_per_dof_update(w.q, 4),
            "compensation_overhead_bytes_per_launch": compensation_bytes_per_launch(w.q, K),
            "traffic": measured_traffic(kname, K, MEASURED_TRAFFIC_Q2)}


def batched_kernel(a) -> dict:
    """Batched stage-launch roofline: the 64 solves on the 10368-tet P2 mesh,
    one launch per Runge-Kutta stage for all members, timed by the library's
    batched autotuner (HIP events on its stream) over 8 homogeneous steps in
    which every member is active."""
    from paper_2106_02858_amd import cmcg, inputs
    _free_device()
    ws = inputs.batched_members(n=12, q=2, B=a.members)
    w0 = ws[0]
    mesh = cmcg.cmcg_mesh_create(w0.xyz, w0.tet, w0.tags)
    s = cmcg.cmcg_space_create(mesh, w0.q, cmcg.CMCG_FP32)
    nodes = cmcg.cmcg_space_nodes(s)
    probs = [cmcg.cmcg_problem_create(s, w.eps, w.mu, None, w.omega,
                                      inputs.gaussian_current(nodes, w.centre, w.width, w.pol)) for w in ws]
    old = cmcg.cmcg_tune_get_stage(2, cmcg.CMCG_FP32)
    v, us = cmcg.cmcg_autotune_batch(probs)
    if a.no_autotune:
        cmcg.cmcg_tune_stage(2, cmcg.CMCG_FP32, old)
        v = old
    per_launch = us[v] * 1e-6
    K = w0.K
    bpl = method_bytes_per_launch(2, 4, K, a.members)
    achieved = bpl / per_launch / 1e9
    kname = STAGE_KERNEL[v].format(q=2)
    log(f"batched stage launch (all {a.members} members active) {us[v]:.1f} us = {achieved:.0f} GB/s ({kname}); "
        f"variants {[round(u, 1) for u in us]}")
    del probs, s, mesh
    _free_device()
    return {"workload": f"batched: {a.members} members on the {K}-tet P2 mesh, FP32 fields, every member active",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "kernel": kname, "avg_launch_us": us[v],
            "bytes_per_launch": bpl, "bytes_per_dof_update": method_bytes_per_dof_update(2, 4, a.members),
            "compensation_overhead_bytes_per_launch": compensation_bytes_per_launch(2, K, a.members),
            "variant_us": us, "traffic": measured_traffic(kname, K * a.members, MEASURED_TRAFFIC_Q2)}


def serving_short(a, cobatch: int) -> dict:
    """The head of the 20 req/s request stream through the serving engine
    (FP32 fields, CMCG to 1e-6): latency p50 / p99 and throughput; up to
    `cobatch` queued requests on one space share a slot."""
    import numpy as np

    from paper_2106_02858_amd import cmcg, inputs, serving
    _free_device()
    reqs = inputs.serving_stream(n_requests=2000, rate=a.rate)[: a.serve_requests]
    out = serving.serve(reqs, budget_bytes=int(a.budget_gb * 2 ** 30), max_slots=a.slots, tol=a.tol,
                        precision=cmcg.CMCG_FP32, log=log, cobatch=cobatch)
    svc = np.array([r["done"] - r["admitted"] for r in out["records"]])
    byts = sum(r["dof_updates"] * method_bytes_per_dof_update(r["q"], 4) for r in out["records"])
    dofs = max(1.0, sum(r["dof_updates"] for r in out["records"]))
    _free_device()
    return {"workload": f"first {a.serve_requests} requests of the 2000-request Poisson stream at {a.rate:g} req/s "
                        f"(n in 8,12,16,24; q in 1,2,3), {a.slots} slots, FP32 fields, CMCG to {a.tol:g}, "
                        f"co-batching up to {cobatch}",
            **{k: out[k] for k in ("completed", "elapsed", "throughput", "p50", "p99", "offered_rate")},
            "co_batched_requests": sum(1 for r in out["records"] if r["members"] > 1),
            "rejected": len(out["rejected"]), "service_p50": float(np.percentile(svc, 50)),
            "service_p99": float(np.percentile(svc, 99)), "dof_updates_per_s": out["dof_updates_per_s"],
            "hbm_job": job_roofline(out["dof_updates_per_s"], byts / dofs)}


if __name__ == "__main__":
    main()
