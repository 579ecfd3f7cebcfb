"""Indexing beyond 2^31 in one field vector: the 144^3 x 6 = 17,915,904-tet
cube at P3 carries 2,149,908,480 dofs per vector.  One right-hand side with
FP32 fields is compared with the FP64 oracle at sampled elements, among them
the last ones, whose dof indices lie beyond 2^31.  The field is a formula of
the indices, evaluated alike on the device and on the host.

Needs about 120 GB of device memory (two FP64 vectors held by torch, 34 GB;
the library's FP32 stage buffers, low parts, FP64 filter accumulators,
right-hand-side buffer and geometry, 85 GB), skipped when less than 130 GB
are free once the memory cached by earlier tests is released, and about 10 GB
of host memory; about half a minute on one MI355X."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2106_02858_amd import inputs
from tests._sampled import sampled_oracle_rhs

pytestmark = pytest.mark.gpu

N, Q = 144, 3


def field_host(elems, Np):
    """U[e][c][i] = sin(1e-3 e + 0.37 c + 0.11 i), the device formula below."""
    e = np.asarray(elems, dtype=np.float64)[:, None, None]
    c = np.arange(6, dtype=np.float64)[None, :, None]
    i = np.arange(Np, dtype=np.float64)[None, None, :]
    return np.sin((e * 1e-3 + c * 0.37) + i * 0.11)


def fill_device(U, chunk=1 << 20):
    import torch
    K, _, Np = U.shape
    c = torch.arange(6, dtype=torch.float64, device=U.device).view(1, 6, 1) * 0.37
    i = torch.arange(Np, dtype=torch.float64, device=U.device).view(1, 1, Np) * 0.11
    for s in range(0, K, chunk):
        e = torch.arange(s, min(K, s + chunk), dtype=torch.float64, device=U.device).view(-1, 1, 1)
        U[s:s + e.shape[0]] = torch.sin((e * 1e-3 + c) + i)


@pytest.mark.timeout(1500)
def test_rhs_beyond_2_31_dofs(lib):
    import gc

    import torch
    # release what earlier tests left: library objects no longer referenced
    # and the blocks torch's caching allocator still holds
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    print(f"huge: {free / 1e9:.0f} GB of {total / 1e9:.0f} GB free", flush=True)
    if free < 130e9:
        pytest.skip(f"needs ~130 GB free device memory, {free / 1e9:.0f} GB free")
    print(f"huge: building the {N}^3 x 6 cube", flush=True)
    xyz, tet, tags = inputs.cube_mesh(N)
    K = tet.shape[0]
    print(f"huge: K={K} q={Q}", flush=True)
    m = lib.cmcg_mesh_create(xyz, tet, tags)
    print("  mesh built", flush=True)
    s = lib.cmcg_space_create(m, Q, lib.CMCG_FP32)
    info = lib.cmcg_space_info(s)
    Np, ndof = info["Np"], info["ndof"]
    assert ndof > 2 ** 31
    print(f"  space built: {ndof} dofs", flush=True)
    p = lib.cmcg_problem_create(s, np.ones(K), np.ones(K), None, 4 * math.pi, None)
    print("  problem built", flush=True)
    U = torch.empty((K, 6, Np), dtype=torch.float64, device="cuda")
    fill_device(U)
    out = torch.empty_like(U)
    t = 0.1
    lib.cmcg_debug_rhs(p, U, out, t=t, with_source=False)
    torch.cuda.synchronize()
    print(f"  rhs done: {ndof} dofs", flush=True)
    rng = np.random.default_rng(17)
    first_beyond = (2 ** 31) // (6 * Np) + 1   # first element whose dofs all lie beyond 2^31
    samples = np.unique(np.concatenate([[0, 1, K // 2, K - 1, K - 2, K - 3, first_beyond],
                                        rng.integers(first_beyond, K, 6), rng.integers(0, K, 12)]))
    got = out[torch.tensor(samples, device="cuda")].cpu().numpy()
    del U, out
    print("  oracle at the sampled elements", flush=True)
    w = SimpleNamespace(xyz=xyz, tet=tet, tags=tags, q=Q, K=K, eps=np.ones(K), mu=np.ones(K),
                        sigma=np.zeros(K), omega=4 * math.pi)
    ref = sampled_oracle_rhs(w, None, lambda el: field_host(el, Np), samples, t, with_source=False)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"  {len(samples)} sampled elements (indices up to {samples.max()}), max rel err {err:.2e}", flush=True)
    assert err < 1e-5
