"""Parity at the full sizes of the benchmarked configurations, in the launch
configuration bench.py times.

* one right-hand side on the 48000-tet P3 mesh, the 1,572,864-tet P2
  scatterer and the largest served mesh (24^3 x 6 tets, P3), compared with the
  FP64 oracle on sampled elements: the oracle evaluates each sampled element
  on the submesh of it and its face neighbours (global boundary tags kept),
  where its right-hand side is exactly the full mesh's;
* the 64-member batched configuration: members equal their single solves
  bit for bit;
* the head of the 2000-request stream through the serving engine: each
  served result equals the same request solved alone, bit for bit;
* whole solves at full size: FP32 fields against FP64 fields (the FP64
  path is itself pinned to the oracle) at the same CG iteration count, on the
  48000-tet P3 configuration and the 1,572,864-tet P2 scatterer, 1e-5
  relative in the eps,mu norm.
"""
import math

import numpy as np
import pytest

from paper_2106_02858_amd import inputs
from tests._sampled import sample_elements, sampled_oracle_rhs

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


WORKLOADS = {
    "large_single_p3": lambda: (inputs.large_single(), (0, 1)),
    "scatterer_p2": lambda: (inputs.scatterer(), (1,)),
    "served_n24_p3": lambda: (inputs.serving_request_workload(
        next(r for r in inputs.serving_stream() if r["n"] == 24 and r["q"] == 3)), (1,)),
}


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_sampled_rhs_at_full_size(lib, name):
    import torch
    w, precisions = WORKLOADS[name]()
    print(f"full-size rhs {name}: K={w.K} q={w.q}", flush=True)
    m = lib.cmcg_mesh_create(w.xyz, w.tet, w.tags)
    rng = np.random.default_rng(11)
    extra = []
    if name == "scatterer_p2":  # elements on the dielectric interface
        inside = np.nonzero(w.eps == 4.0)[0]
        extra = rng.choice(inside, 4, replace=False)
    samples = sample_elements(w, rng, extra)
    t = 0.37 * 2 * math.pi / w.omega
    for precision in precisions:
        s = lib.cmcg_space_create(m, w.q, precision)
        nodes = lib.cmcg_space_nodes(s)
        jd = torch.tensor(inputs.gaussian_current(nodes, w.centre, w.width, w.pol), dtype=torch.float64,
                          device="cuda")
        p = lib.cmcg_problem_create_device(s, w.eps, w.mu, w.sigma, w.omega, jd)
        del jd
        info = lib.cmcg_space_info(s)
        U = np.random.default_rng(5).standard_normal((w.K, 6, info["Np"]))
        Ud = torch.tensor(U, dtype=torch.float64, device="cuda")
        out = torch.empty_like(Ud)
        lib.cmcg_debug_rhs(p, Ud, out, t=t, with_source=True)
        got = out[torch.tensor(samples, device="cuda")].cpu().numpy()
        del Ud, out
        ref = sampled_oracle_rhs(w, nodes, U, samples, t)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"  precision {precision}: {len(samples)} sampled elements, max rel err {err:.2e}", flush=True)
        assert err < TOL[precision]


def filtered(lib, r, K, Np):
    import torch
    fr = torch.zeros((K, 6, Np), dtype=torch.float64, device="cuda")
    fi = torch.zeros_like(fr)
    lib.cmcg_result_filtered_device(r, fr, fi)
    return fr.cpu().numpy() + 1j * fi.cpu().numpy()


def test_batched_configuration_members_equal_single(lib):
    ws = inputs.batched_members()
    w0 = ws[0]
    print(f"batched full size: {len(ws)} members, K={w0.K}", flush=True)
    m = lib.cmcg_mesh_create(w0.xyz, w0.tet, w0.tags)
    s = lib.cmcg_space_create(m, w0.q, lib.CMCG_FP32)
    nodes = lib.cmcg_space_nodes(s)
    probs = [lib.cmcg_problem_create(s, w.eps, w.mu, None, w.omega,
                                     inputs.gaussian_current(nodes, w.centre, w.width, w.pol)) for w in ws]
    o = lib.cmcg_options_default(tol=1e-6, max_iter=2000)
    res = lib.cmcg_solve_batch(probs, o)
    info = lib.cmcg_space_info(s)
    for b in (0, 21, 42, 63):
        single = lib.cmcg_solve(probs[b], o)
        a, c = lib.cmcg_result_stats(res[b]), lib.cmcg_result_stats(single)
        print(f"  member {b}: iters {a['iters']} M {a['steps']}", flush=True)
        assert a["iters"] == c["iters"] and a["status"] == c["status"] == lib.CMCG_OK
        assert np.array_equal(filtered(lib, res[b], info["K"], info["Np"]),
                              filtered(lib, single, info["K"], info["Np"]))


def test_serving_stream_head_equal_alone(lib):
    from paper_2106_02858_amd import serving
    reqs = inputs.serving_stream()[:6]
    out = serving.serve(reqs, budget_bytes=64 << 30, max_slots=8, tol=1e-6, keep_results=True)
    assert out["completed"] == len(reqs)
    cache = serving.SpaceCache(lib.CMCG_FP32)
    for rec in out["records"]:
        req = next(r for r in reqs if r["id"] == rec["id"])
        prob = serving.build_problem(cache, req)
        alone = lib.cmcg_solve(prob, lib.cmcg_options_default(tol=1e-6, max_iter=2000))
        s, _ = cache.get(req["n"], req["q"])
        info = lib.cmcg_space_info(s)
        print(f"  request {rec['id']}: n={req['n']} q={req['q']} iters {rec['iters']}", flush=True)
        assert lib.cmcg_result_stats(alone)["iters"] == rec["iters"]
        assert np.array_equal(filtered(lib, out["results"][rec["id"]], info["K"], info["Np"]),
                              filtered(lib, alone, info["K"], info["Np"]))


def _weighted_rel(lib, p64, a, b):
    """||a - b|| / ||b|| in the eps,mu norm (complex dof vectors on the
    device), with the FP64 problem's inner product."""
    d = a - b
    num = lib.cmcg_debug_dot(p64, d.real.contiguous(), d.real.contiguous()) + \
        lib.cmcg_debug_dot(p64, d.imag.contiguous(), d.imag.contiguous())
    den = lib.cmcg_debug_dot(p64, b.real.contiguous(), b.real.contiguous()) + \
        lib.cmcg_debug_dot(p64, b.imag.contiguous(), b.imag.contiguous())
    return math.sqrt(num / den)


def _filtered_dev(lib, r, K, Np):
    import torch
    fr = torch.zeros((K, 6, Np), dtype=torch.float64, device="cuda")
    fi = torch.zeros_like(fr)
    lib.cmcg_result_filtered_device(r, fr, fi)
    return torch.complex(fr, fi)


@pytest.mark.parametrize("name,iters", [("large_single_p3", 0), ("scatterer_p2", 6)])
def test_fp32_solve_against_fp64_solve_at_full_size(lib, name, iters):
    """One CMCG solve with FP32 fields (FP64 CG scalars and vectors) against
    the same solve with FP64 fields at the same iteration count: the FP32
    error stated per result stays within 1e-5.  48000-tet P3: the FP64
    solve's own count at 1e-6 (the benchmarked solve); 1,572,864-tet P2
    scatterer: a fixed count of 6 iterations."""
    import torch
    w = inputs.large_single() if name == "large_single_p3" else inputs.scatterer()
    print(f"full-size solve {name}: K={w.K} q={w.q}", flush=True)
    m = lib.cmcg_mesh_create(w.xyz, w.tet, w.tags)
    res = {}
    for precision in (0, 1):
        s = lib.cmcg_space_create(m, w.q, precision)
        jd = torch.tensor(inputs.gaussian_current(lib.cmcg_space_nodes(s), w.centre, w.width, w.pol),
                          dtype=torch.float64, device="cuda")
        p = lib.cmcg_problem_create_device(s, w.eps, w.mu, w.sigma, w.omega, jd)
        del jd
        if precision == 0 and iters == 0:
            o = lib.cmcg_options_default(tol=1e-6, max_iter=2000)
        else:
            o = lib.cmcg_options_default(fixed_iters=iters)
        r = lib.cmcg_solve(p, o)
        st = lib.cmcg_result_stats(r)
        if precision == 0:
            iters = st["iters"]
        info = lib.cmcg_space_info(s)
        res[precision] = (p, _filtered_dev(lib, r, info["K"], info["Np"]))
        print(f"  precision {precision}: {st['iters']} iterations, rel res {st['rel_res']:.2e}, "
              f"{st['seconds']:.2f} s", flush=True)
        del r
    err = _weighted_rel(lib, res[0][0], res[1][1], res[0][1])
    print(f"  FP32 vs FP64 filtered fields: {err:.2e}", flush=True)
    assert err < 1e-5
