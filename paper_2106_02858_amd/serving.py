"""Request-serving loop over the engine of the C ABI (continuous batching).

Requests arrive on a wall clock (arrival times in seconds, e.g. a Poisson
stream).  Arrived requests wait in a FIFO queue; the head is admitted into an
engine slot as soon as a slot is free and its device footprint fits the
budget (a request that cannot fit even an empty engine is rejected and
listed in the returned "rejected"); every engine step advances all running solves (their periods overlap
on the device); finished solves are collected and their latency (result
ready - arrival) recorded.  All numerical work runs in the HIP library; this
loop only schedules.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from . import cmcg, inputs


class SpaceCache:
    """Meshes and spaces shared by requests of the same (n, q)."""

    def __init__(self, precision):
        self.precision = precision
        self.meshes = {}
        self.spaces = {}

    def get(self, n, q):
        if n not in self.meshes:
            xyz, tet, tags = inputs.cube_mesh(n)
            self.meshes[n] = cmcg.cmcg_mesh_create(xyz, tet, tags)
        key = (n, q)
        if key not in self.spaces:
            s = cmcg.cmcg_space_create(self.meshes[n], q, self.precision)
            self.spaces[key] = (s, cmcg.cmcg_space_nodes(s))
        return self.spaces[key]


def build_problem(cache: SpaceCache, req):
    w = inputs.serving_request_workload(req)
    s, nodes = cache.get(w.n, w.q)
    j = inputs.gaussian_current(nodes, w.centre, w.width, w.pol)
    return cmcg.cmcg_problem_create(s, w.eps, w.mu, None, w.omega, j)


def serve(requests, budget_bytes: int, max_slots: int, precision=cmcg.CMCG_FP32, tol: float = 1e-6,
          max_iter: int = 2000, time_scale: float = 1.0, log=None, keep_results: bool = False,
          cobatch: int = 1, cobatch_max_elements: int | None = None):
    """Serve `requests` (dicts with "arrival" and the recipe fields of
    inputs.serving_stream).  time_scale > 1 compresses the arrival clock.
    cobatch > 1: when the head of the queue has queued requests on the same
    space (n, q), up to `cobatch` of them share one slot and are solved
    together by the batched launches (each result equals its solo solve);
    cobatch_max_elements limits that to spaces of at most that many elements
    (small meshes, whose single launches leave most of the chip idle).
    Returns a dict with latencies, throughput and per-request records."""
    engine = cmcg.cmcg_engine_create(budget_bytes, max_slots)
    cache = SpaceCache(precision)
    opts = cmcg.cmcg_options_default(tol=tol, max_iter=max_iter)
    pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
    queue = collections.deque()
    slots = {}  # slot -> (request, problem, admit time)
    records = []
    rejected = []
    results = {}
    t0 = time.perf_counter()

    def now():
        return (time.perf_counter() - t0) * time_scale

    steps = 0
    while pending or queue or slots:
        t = now()
        while pending and pending[0]["arrival"] <= t:
            queue.append(pending.popleft())
        # FIFO admission while the head fits.  A head that can never fit (its
        # footprint exceeds the whole budget, or it does not fit an engine that
        # holds nothing else) is rejected and recorded, so the loop neither
        # spins on it nor holds back the requests behind it.
        while queue:
            req = queue[0]
            prob = req.get("_problem") or build_problem(cache, req)
            req["_problem"] = prob
            small = cobatch_max_elements is None or \
                cmcg.cmcg_space_info(cache.get(req["n"], req["q"])[0])["K"] <= cobatch_max_elements
            if cobatch > 1 and small:
                group = [r for r in queue if (r["n"], r["q"]) == (req["n"], req["q"])][:cobatch]
                if len(group) > 1:
                    for r in group:
                        r["_problem"] = r.get("_problem") or build_problem(cache, r)
                    try:
                        slot = cmcg.cmcg_engine_admit_batch(engine, [r["_problem"] for r in group], opts)
                    except cmcg.CmcgError as err:
                        if err.code != cmcg.CMCG_ERR_TOO_LARGE:
                            raise
                        slot = None  # too large together: admit the head alone
                    else:
                        if slot is None and slots:
                            break
                    if slot is not None:
                        for r in group:
                            queue.remove(r)
                        slots[slot] = (group, [r["_problem"] for r in group], now())
                        continue
            try:
                slot = cmcg.cmcg_engine_admit(engine, prob, opts)
            except cmcg.CmcgError as err:
                if err.code != cmcg.CMCG_ERR_TOO_LARGE:
                    raise
                slot = None
            else:
                if slot is None and slots:
                    break  # fits later, once a running solve has finished
            if slot is None:
                queue.popleft()
                req.pop("_problem", None)
                rejected.append(dict(id=req["id"], n=req["n"], q=req["q"], arrival=req["arrival"],
                                     footprint=cmcg.cmcg_problem_footprint(prob)))
                if log:
                    log(f"rejected {req['id']} n={req['n']} q={req['q']}: does not fit the budget")
                continue
            queue.popleft()
            slots[slot] = ([req], [prob], now())
        if not slots:
            if pending:  # idle until the next arrival
                wait = (pending[0]["arrival"] - now()) / time_scale
                if wait > 0:
                    time.sleep(min(wait, 0.05))
            continue
        cmcg.cmcg_engine_step(engine)
        steps += 1
        for slot in list(slots):
            if cmcg.cmcg_engine_poll(engine, slot) >= 2:
                reqs_in, probs_in, t_adm = slots.pop(slot)
                if len(reqs_in) > 1:
                    res_list = cmcg.cmcg_engine_collect_batch(engine, slot, probs_in)
                else:
                    res_list = [cmcg.cmcg_engine_collect(engine, slot, probs_in[0])]
                t_done = now()
                for req, res in zip(reqs_in, res_list):
                    st = cmcg.cmcg_result_stats(res)
                    rec = dict(id=req["id"], n=req["n"], q=req["q"], omega=req["omega"], arrival=req["arrival"],
                               admitted=t_adm, done=t_done, latency=t_done - req["arrival"], iters=st["iters"],
                               rel_res=st["rel_res"], dof_updates=st["dof_updates"], members=len(reqs_in))
                    records.append(rec)
                    if keep_results:
                        results[req["id"]] = res
                    req.pop("_problem", None)
                    if log:
                        log(f"done {req['id']} n={req['n']} q={req['q']} iters={st['iters']} "
                            f"members={len(reqs_in)} latency={rec['latency']:.2f}s queue={len(queue)} "
                            f"running={len(slots)}")
    elapsed = now()
    lat = np.array([r["latency"] for r in records])
    out = dict(completed=len(records), elapsed=elapsed, engine_steps=steps,
               throughput=len(records) / elapsed if elapsed > 0 else 0.0,
               dof_updates_per_s=sum(r["dof_updates"] for r in records) / elapsed if elapsed > 0 else 0.0,
               p50=float(np.percentile(lat, 50)) if len(lat) else None,
               p99=float(np.percentile(lat, 99)) if len(lat) else None,
               offered_rate=(len(requests) / max(r["arrival"] for r in requests)) if requests else 0.0,
               records=records, rejected=rejected)
    if keep_results:
        out["results"] = results
    return out
