"""Several frequencies in one solve on the GPU against the FP64 oracle: a
three-harmonic current (k = 1, 2, 3 times omega0), CMCG at a fixed iteration
count over the base period, every harmonic filtered at its own frequency
(trapezoid for P1, Hermite for P2); argument checks."""
import numpy as np
import pytest

from oracle import dg, multifreq
from paper_2106_02858_amd import inputs
from tests._pairs import rel_norm_c

pytestmark = pytest.mark.gpu


def setup(lib, q, precision):
    xyz, tet, tags = inputs.cube_mesh(2)
    K = tet.shape[0]
    rng = np.random.default_rng(12)
    eps = rng.choice([1.0, 2.0], K)
    omega0 = 1.5 * np.pi
    base = dg.make_problem(xyz, tet, tags, q, eps, np.ones(K), omega=omega0)
    ks = [1, 2, 3]
    js = [inputs.gaussian_current(base.geo.x, c, 0.35, pol) * (1.0 + 0.5j * h)
          for h, (c, pol) in enumerate((((0.4, 0.5, 0.5), 2), ((0.6, 0.4, 0.5), 0), ((0.5, 0.5, 0.6), 1)))]
    mp = multifreq.make(base, ks, js)
    m = lib.cmcg_mesh_create(xyz, tet, tags)
    s = lib.cmcg_space_create(m, q, precision)
    lp = lib.cmcg_problem_create_harmonics(s, eps, np.ones(K), None, omega0, ks, np.stack(js))
    return base, mp, s, lp


def harmonic(lib, r, h, K, Np):
    import torch
    fr = torch.zeros((K, 6, Np), dtype=torch.float64, device="cuda")
    fi = torch.zeros_like(fr)
    lib.cmcg_result_filtered_harmonic_device(r, h, fr, fi)
    return fr.cpu().numpy() + 1j * fi.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 2])
def test_harmonics_against_oracle(lib, q, precision):
    base, mp, s, lp = setup(lib, q, precision)
    M0 = 6 * ((lib.cmcg_problem_steps(lp, lib.cmcg_options_default())[0] + 5) // 6)
    iters = 10
    ref = multifreq.solve(mp, M=M0, fixed_iters=iters)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=iters, steps=M0))
    assert lib.cmcg_result_harmonics(r) == 3
    for h in range(3):
        err = rel_norm_c(base, harmonic(lib, r, h, base.K, base.Np), ref.Fs[h])
        print(f"q={q} prec={precision} harmonic k={mp.ks[h]}: {err:.2e}", flush=True)
        assert err < (1e-11 if precision == 0 else 1e-5)


def test_harmonic_arguments(lib):
    xyz, tet, tags = inputs.cube_mesh(1)
    K = tet.shape[0]
    m = lib.cmcg_mesh_create(xyz, tet, tags)
    s = lib.cmcg_space_create(m, 1, 0)
    j = np.zeros((9, K, 4, 3))
    for ks in ([], [1, 1], [0, 2], list(range(1, 10))):
        with pytest.raises(lib.CmcgError) as e:
            lib.cmcg_problem_create_harmonics(s, np.ones(K), np.ones(K), None, 1.0, ks, j[:max(1, len(ks))])
        assert e.value.code == lib.CMCG_ERR_ARG, ks
    p = lib.cmcg_problem_create_harmonics(s, np.ones(K), np.ones(K), None, 1.0, [1, 3], j[:2] + 1.0)
    with pytest.raises(lib.CmcgError) as e:
        lib.cmcg_solve_batch([p])
    assert e.value.code == lib.CMCG_ERR_ARG
    r = lib.cmcg_solve(p, lib.cmcg_options_default(fixed_iters=2))
    with pytest.raises(lib.CmcgError) as e:
        harmonic(lib, r, 2, K, 4)
    assert e.value.code == lib.CMCG_ERR_ARG
