"""Thin Python binding of libcmcg.so (include/cmcg.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device arrays are torch tensors on the current HIP device (PyTorch supplies
device memory and streams); host arrays are numpy arrays.  Functions keep the
C names; the small classes only attach the matching *_destroy call to the
handle's lifetime.  Importing this module fails loudly when the library has
not been built.

A program that also uses torch on the device initialises torch first (for
instance torch.cuda.set_device(0)): the HIP runtime that is loaded first
serves both, and torch cannot start on one the library loaded before it.
Without torch, host arrays and the default stream suffice.
"""
from __future__ import annotations

import ctypes as C
import sys
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmcg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2106_02858_amd.build`")

_lib = C.CDLL(LIB_PATH)

CMCG_OK = 0
CMCG_STAGE_VARIANTS = 10  # include/cmcg.h
CMCG_NOT_CONVERGED = 1
CMCG_ERR_ARG = -1
CMCG_ERR_MESH = -2
CMCG_ERR_NOMEM = -3
CMCG_ERR_DEVICE = -4
CMCG_ERR_UNSTABLE = -5
CMCG_ERR_BREAKDOWN = -6
CMCG_ERR_STATE = -7
CMCG_ERR_TOO_LARGE = -8
CMCG_FP64, CMCG_FP32 = 0, 1
CMCG_TAG_INTERIOR, CMCG_TAG_PEC, CMCG_TAG_IMPEDANCE = 0, 1, 2
CMCG_SCHEME_AUTO, CMCG_SCHEME_RK2, CMCG_SCHEME_RK4 = 0, 2, 4
CMCG_FLUX_UPWIND, CMCG_FLUX_CENTRED = 0, 1

EXPORTED = [
    "cmcg_last_error", "cmcg_version", "cmcg_options_default",
    "cmcg_mesh_create", "cmcg_mesh2d_create", "cmcg_mesh_dim", "cmcg_mesh_destroy", "cmcg_mesh_info",
    "cmcg_space_create", "cmcg_space_destroy", "cmcg_space_info", "cmcg_space_nodes",
    "cmcg_problem_create", "cmcg_problem_create_device", "cmcg_problem_destroy", "cmcg_problem_steps", "cmcg_problem_lts_fine",
    "cmcg_problem_create_harmonics", "cmcg_result_harmonics", "cmcg_result_filtered_harmonic_device",
    "cmcg_solve", "cmcg_fw_solve", "cmcg_solve_batch", "cmcg_result_fields", "cmcg_result_filtered_device", "cmcg_result_initial_device",
    "cmcg_result_stats", "cmcg_result_history", "cmcg_result_destroy",
    "cmcg_debug_rhs", "cmcg_debug_period", "cmcg_debug_step", "cmcg_debug_dot", "cmcg_debug_dot_noalloc", "cmcg_debug_mfma", "cmcg_tune_stage", "cmcg_tune_get_stage", "cmcg_tune_resolve_stage",
    "cmcg_autotune_stage", "cmcg_autotune_batch", "cmcg_mesh_locality_order",
    "cmcg_problem_footprint", "cmcg_engine_create", "cmcg_engine_destroy", "cmcg_engine_admit",
    "cmcg_engine_step", "cmcg_engine_poll", "cmcg_engine_collect", "cmcg_engine_cancel", "cmcg_engine_info",
    "cmcg_engine_admit_batch", "cmcg_engine_slot_members", "cmcg_engine_collect_batch",
]


PROGRESS_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_double)


class cmcg_options(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("fixed_iters", C.c_int), ("cfl", C.c_double),
                ("steps", C.c_int), ("scheme", C.c_int), ("flux", C.c_int), ("use_graph", C.c_int),
                ("residual_refresh", C.c_int), ("progress", PROGRESS_FN), ("progress_ctx", C.c_void_p),
                ("runup", C.c_int), ("autotune", C.c_int), ("lts_ratio", C.c_int)]

    def set_progress(self, fn):
        """fn(iter, rel_res) -> bool (True stops the iteration)."""
        self._cb = PROGRESS_FN(lambda ctx, it, rel: int(bool(fn(it, rel))))
        self.progress = self._cb


class cmcg_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("periods", C.c_int), ("steps", C.c_int), ("status", C.c_int),
                ("dt", C.c_double), ("rel_res", C.c_double), ("J0", C.c_double), ("seconds", C.c_double),
                ("seconds_to_1e6", C.c_double), ("dof_updates", C.c_double), ("res0", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


P = C.c_void_p
D = C.POINTER(C.c_double)
_sig = {
    "cmcg_last_error": (C.c_char_p, []),
    "cmcg_version": (C.c_char_p, []),
    "cmcg_options_default": (None, [C.POINTER(cmcg_options)]),
    "cmcg_mesh_create": (C.c_int, [C.c_int64, P, C.c_int64, P, P, C.POINTER(P)]),
    "cmcg_mesh_destroy": (None, [P]),
    "cmcg_mesh2d_create": (C.c_int, [C.c_int64, P, C.c_int64, P, P, C.POINTER(P)]),
    "cmcg_mesh_dim": (C.c_int, [P, C.POINTER(C.c_int)]),
    "cmcg_mesh_info": (C.c_int, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), D]),
    "cmcg_space_create": (C.c_int, [P, C.c_int, C.c_int, C.POINTER(P)]),
    "cmcg_space_destroy": (None, [P]),
    "cmcg_space_info": (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "cmcg_space_nodes": (C.c_int, [P, P]),
    "cmcg_problem_create": (C.c_int, [P, P, P, P, C.c_double, P, P, P, P, C.POINTER(P)]),
    "cmcg_problem_create_device": (C.c_int, [P, P, P, P, C.c_double, P, P, P, P, P, C.POINTER(P)]),
    "cmcg_debug_step": (C.c_int, [P, C.POINTER(cmcg_options), C.c_int, C.c_int, C.c_int, P, P, P]),
    "cmcg_debug_dot_noalloc": (C.c_int, [P, P, P, P, P]),
    "cmcg_debug_mfma": (C.c_int, [C.c_int, P, P, P, P]),
    "cmcg_problem_lts_fine": (C.c_int, [P, C.POINTER(cmcg_options), P, C.POINTER(C.c_int64)]),
    "cmcg_problem_destroy": (None, [P]),
    "cmcg_problem_steps": (C.c_int, [P, C.POINTER(cmcg_options), C.POINTER(C.c_int), D]),
    "cmcg_solve": (C.c_int, [P, C.POINTER(cmcg_options), P, P, C.POINTER(P)]),
    "cmcg_fw_solve": (C.c_int, [P, C.POINTER(cmcg_options), P, P, C.POINTER(P)]),
    "cmcg_problem_create_harmonics": (C.c_int, [P, P, P, P, C.c_double, C.c_int, P, P, P, C.POINTER(P)]),
    "cmcg_result_harmonics": (C.c_int, [P, C.POINTER(C.c_int)]),
    "cmcg_result_filtered_harmonic_device": (C.c_int, [P, C.c_int, P, P, P]),
    "cmcg_solve_batch": (C.c_int, [C.POINTER(P), C.c_int, C.POINTER(cmcg_options), P, C.POINTER(P)]),
    "cmcg_result_fields": (C.c_int, [P, P, P, P, P]),
    "cmcg_result_filtered_device": (C.c_int, [P, P, P, P]),
    "cmcg_result_initial_device": (C.c_int, [P, P, P]),
    "cmcg_result_stats": (C.c_int, [P, C.POINTER(cmcg_stats)]),
    "cmcg_result_history": (C.c_int, [P, P, C.c_int, C.POINTER(C.c_int)]),
    "cmcg_result_destroy": (None, [P]),
    "cmcg_debug_rhs": (C.c_int, [P, C.POINTER(cmcg_options), C.c_double, C.c_int, P, P, P]),
    "cmcg_debug_period": (C.c_int, [P, C.POINTER(cmcg_options), C.c_int, C.c_int, P, P, P, P, P]),
    "cmcg_debug_dot": (C.c_int, [P, P, P, D, P]),
    "cmcg_tune_stage": (C.c_int, [C.c_int, C.c_int, C.c_int]),
    "cmcg_problem_footprint": (C.c_int, [P, C.POINTER(C.c_size_t)]),
    "cmcg_engine_create": (C.c_int, [C.c_size_t, C.c_int, C.POINTER(P)]),
    "cmcg_engine_destroy": (None, [P]),
    "cmcg_engine_admit": (C.c_int, [P, P, C.POINTER(cmcg_options), C.POINTER(C.c_int)]),
    "cmcg_engine_step": (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "cmcg_engine_poll": (C.c_int, [P, C.c_int, C.POINTER(C.c_int)]),
    "cmcg_engine_collect": (C.c_int, [P, C.c_int, C.POINTER(P)]),
    "cmcg_engine_cancel": (C.c_int, [P, C.c_int]),
    "cmcg_engine_info": (C.c_int, [P, C.POINTER(C.c_size_t), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "cmcg_engine_admit_batch": (C.c_int, [P, P, C.c_int, C.POINTER(cmcg_options), C.POINTER(C.c_int)]),
    "cmcg_engine_slot_members": (C.c_int, [P, C.c_int, C.POINTER(C.c_int)]),
    "cmcg_engine_collect_batch": (C.c_int, [P, C.c_int, P, C.c_int]),
    "cmcg_mesh_locality_order": (C.c_int, [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "cmcg_tune_get_stage": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int)]),
    "cmcg_tune_resolve_stage": (C.c_int, [C.c_int, C.c_int, C.c_int64, C.c_int, C.POINTER(C.c_int)]),
    "cmcg_autotune_stage": (C.c_int, [P, C.POINTER(cmcg_options), C.c_void_p, C.POINTER(C.c_int),
                                      C.POINTER(C.c_double)]),
    "cmcg_autotune_batch": (C.c_int, [P, C.c_int, C.POINTER(cmcg_options), C.c_void_p, C.POINTER(C.c_int),
                                      C.POINTER(C.c_double)]),
}
for _n, (_r, _a) in _sig.items():
    _f = getattr(_lib, _n)
    _f.restype = _r
    _f.argtypes = _a


class CmcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cmcg error {code}: {msg}")
        self.code = code


def _check(rc, allow=(CMCG_OK,)):
    if rc not in allow:
        raise CmcgError(rc, _lib.cmcg_last_error().decode())
    return rc


def _ptr(a):
    """Address of a contiguous numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous
        return a.ctypes.data
    assert a.is_contiguous()
    return a.data_ptr()


def _stream(stream=None):
    """A raw HIP stream handle, a torch stream, or None: torch's current
    stream when torch has already initialised the device, else the default
    stream.  (Initialising torch here, after the library has started the HIP
    runtime on its own, would fail: the device runtime is set up by whichever
    comes first.)"""
    if stream is not None:
        return getattr(stream, "cuda_stream", stream)
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        return torch.cuda.current_stream().cuda_stream
    return None


def cmcg_version():
    return _lib.cmcg_version().decode()


def cmcg_last_error():
    return _lib.cmcg_last_error().decode()


def cmcg_options_default(**kw) -> cmcg_options:
    o = cmcg_options()
    _lib.cmcg_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class _Handle:
    _destroy = None

    def __init__(self, h, keep=()):
        self.h = h
        self._keep = keep

    def __del__(self):
        h = getattr(self, "h", None)
        if h and self._destroy and _lib is not None:
            try:
                getattr(_lib, self._destroy)(h)
            except Exception:
                pass
            self.h = None


class Mesh(_Handle):
    _destroy = "cmcg_mesh_destroy"


class Space(_Handle):
    _destroy = "cmcg_space_destroy"

    def info(self):
        return cmcg_space_info(self)


class Problem(_Handle):
    _destroy = "cmcg_problem_destroy"


class Result(_Handle):
    _destroy = "cmcg_result_destroy"


def cmcg_mesh_create(xyz, tet, face_tag=None) -> Mesh:
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tet = np.ascontiguousarray(tet, dtype=np.int64)
    tags = None if face_tag is None else np.ascontiguousarray(face_tag, dtype=np.int8)
    h = P()
    _check(_lib.cmcg_mesh_create(xyz.shape[0], _ptr(xyz), tet.shape[0], _ptr(tet), _ptr(tags), C.byref(h)))
    return Mesh(h)


def cmcg_mesh2d_create(xy, tri, edge_tag=None) -> Mesh:
    """Triangle mesh of the 2-D transverse-magnetic setting: xy [nv,2],
    tri [K,3], edge_tag [K,3] (edge f opposite vertex f)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int64)
    tags = None if edge_tag is None else np.ascontiguousarray(edge_tag, dtype=np.int8)
    h = P()
    _check(_lib.cmcg_mesh2d_create(xy.shape[0], _ptr(xy), tri.shape[0], _ptr(tri), _ptr(tags), C.byref(h)))
    return Mesh(h)


def cmcg_mesh_dim(m: Mesh) -> int:
    d = C.c_int()
    _check(_lib.cmcg_mesh_dim(m.h, C.byref(d)))
    return d.value


def cmcg_mesh_info(m: Mesh):
    K, nb, rho = C.c_int64(), C.c_int64(), C.c_double()
    _check(_lib.cmcg_mesh_info(m.h, C.byref(K), C.byref(nb), C.byref(rho)))
    return dict(K=K.value, n_boundary=nb.value, min_rho=rho.value)


def cmcg_space_create(m: Mesh, q: int, precision: int = CMCG_FP64) -> Space:
    h = P()
    _check(_lib.cmcg_space_create(m.h, q, precision, C.byref(h)))
    s = Space(h)
    s.dim = cmcg_mesh_dim(m)
    return s


def cmcg_space_info(s: Space):
    q, Np, Nfp, K, nd = C.c_int(), C.c_int(), C.c_int(), C.c_int64(), C.c_int64()
    _check(_lib.cmcg_space_info(s.h, C.byref(q), C.byref(Np), C.byref(Nfp), C.byref(K), C.byref(nd)))
    dim = getattr(s, "dim", 3)
    return dict(q=q.value, Np=Np.value, Nfp=Nfp.value, K=K.value, ndof=nd.value, dim=dim,
                ncomp=3 if dim == 2 else 6)


def cmcg_space_nodes(s: Space) -> np.ndarray:
    i = cmcg_space_info(s)
    out = np.empty((i["K"], i["Np"], i["dim"]))
    _check(_lib.cmcg_space_nodes(s.h, _ptr(out)))
    return out


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def cmcg_problem_create(s: Space, eps, mu, sigma=None, omega=2 * np.pi, j=None, g=None) -> Problem:
    """j: complex [K,Np,3] nodal current density; g: complex [K,4,Nfp,3].
    2-D spaces: j [K,Np] (the e component), g [K,3,Nfp]."""
    eps, mu, sigma = _f64(eps), _f64(mu), _f64(sigma)
    jr = ji = gr = gi = None
    if j is not None:
        j = np.asarray(j)
        jr = _f64(np.real(j))
        ji = _f64(np.imag(j)) if np.iscomplexobj(j) else None
    if g is not None:
        g = np.asarray(g)
        gr = _f64(np.real(g))
        gi = _f64(np.imag(g)) if np.iscomplexobj(g) else None
    h = P()
    _check(_lib.cmcg_problem_create(s.h, _ptr(eps), _ptr(mu), _ptr(sigma), float(omega), _ptr(jr), _ptr(ji),
                                    _ptr(gr), _ptr(gi), C.byref(h)))
    return Problem(h, keep=(s,))


def cmcg_problem_create_device(s: Space, eps, mu, sigma, omega, j_re_dev, j_im_dev=None, stream=None,
                               g_re_dev=None, g_im_dev=None) -> Problem:
    eps, mu, sigma = _f64(eps), _f64(mu), _f64(sigma)
    h = P()
    _check(_lib.cmcg_problem_create_device(s.h, _ptr(eps), _ptr(mu), _ptr(sigma), float(omega), _ptr(j_re_dev),
                                           _ptr(j_im_dev), _ptr(g_re_dev), _ptr(g_im_dev), _stream(stream),
                                           C.byref(h)))
    return Problem(h, keep=(s,))


def cmcg_problem_lts_fine(p: Problem, K: int, opts: cmcg_options):
    """Boolean [K]: the elements local time stepping with `opts` treats as fine."""
    f = np.zeros(K, dtype=np.int8)
    nf = C.c_int64()
    _check(_lib.cmcg_problem_lts_fine(p.h, C.byref(opts), _ptr(f), C.byref(nf)))
    return f.astype(bool)


def cmcg_problem_steps(p: Problem, opts: cmcg_options | None = None):
    o = opts or cmcg_options_default()
    M, dt = C.c_int(), C.c_double()
    _check(_lib.cmcg_problem_steps(p.h, C.byref(o), C.byref(M), C.byref(dt)))
    return M.value, dt.value


def cmcg_solve(p: Problem, opts: cmcg_options | None = None, u0_dev=None, stream=None) -> Result:
    o = opts or cmcg_options_default()
    h = P()
    _check(_lib.cmcg_solve(p.h, C.byref(o), _ptr(u0_dev), _stream(stream), C.byref(h)),
           allow=(CMCG_OK, CMCG_NOT_CONVERGED))
    return Result(h, keep=(p,))


def cmcg_problem_create_harmonics(s: Space, eps, mu, sigma, omega0: float, ks, js) -> Problem:
    """js: complex [nh, K, Np, 3] nodal currents of the harmonics k_h omega0."""
    eps, mu, sigma = _f64(eps), _f64(mu), _f64(sigma)
    js = np.asarray(js)
    jr = _f64(np.real(js))
    ji = _f64(np.imag(js)) if np.iscomplexobj(js) else None
    karr = np.ascontiguousarray(np.asarray(ks, dtype=np.int32))
    h = P()
    _check(_lib.cmcg_problem_create_harmonics(s.h, _ptr(eps), _ptr(mu), _ptr(sigma), float(omega0), len(karr),
                                              _ptr(karr), _ptr(jr), _ptr(ji), C.byref(h)))
    return Problem(h, keep=(s,))


def cmcg_result_harmonics(r: Result) -> int:
    n = C.c_int()
    _check(_lib.cmcg_result_harmonics(r.h, C.byref(n)))
    return n.value


def cmcg_result_filtered_harmonic_device(r: Result, h: int, f_re_dev, f_im_dev, stream=None):
    _check(_lib.cmcg_result_filtered_harmonic_device(r.h, int(h), _ptr(f_re_dev), _ptr(f_im_dev), _stream(stream)))


def cmcg_fw_solve(p: Problem, opts: cmcg_options | None = None, u0_dev=None, stream=None) -> Result:
    o = opts or cmcg_options_default()
    h = P()
    _check(_lib.cmcg_fw_solve(p.h, C.byref(o), _ptr(u0_dev), _stream(stream), C.byref(h)),
           allow=(CMCG_OK, CMCG_NOT_CONVERGED))
    return Result(h, keep=(p,))


def cmcg_solve_batch(problems, opts: cmcg_options | None = None, stream=None):
    o = opts or cmcg_options_default()
    n = len(problems)
    arr = (P * n)(*[p.h for p in problems])
    res = (P * n)()
    _check(_lib.cmcg_solve_batch(arr, n, C.byref(o), _stream(stream), res), allow=(CMCG_OK, CMCG_NOT_CONVERGED))
    return [Result(P(res[b]), keep=(problems[b],)) for b in range(n)]


def cmcg_result_fields(r: Result, K: int, Np: int, dim: int = 3):
    """(e, h) complex at the nodes: [K,Np,3] each, or in 2-D e [K,Np], h [K,Np,2]."""
    shapes = [(K, Np, 3)] * 4 if dim == 3 else [(K, Np), (K, Np), (K, Np, 2), (K, Np, 2)]
    out = [np.empty(sh) for sh in shapes]
    _check(_lib.cmcg_result_fields(r.h, *[_ptr(a) for a in out]))
    e = out[0] + 1j * out[1]
    h = out[2] + 1j * out[3]
    return e, h


def cmcg_result_filtered_device(r: Result, f_re, f_im, stream=None):
    _check(_lib.cmcg_result_filtered_device(r.h, _ptr(f_re), _ptr(f_im), _stream(stream)))


def cmcg_result_initial_device(r: Result, u0, stream=None):
    _check(_lib.cmcg_result_initial_device(r.h, _ptr(u0), _stream(stream)))


def cmcg_result_stats(r: Result) -> dict:
    st = cmcg_stats()
    _check(_lib.cmcg_result_stats(r.h, C.byref(st)))
    return st.as_dict()


def cmcg_result_history(r: Result) -> np.ndarray:
    n = C.c_int()
    _check(_lib.cmcg_result_history(r.h, None, 0, C.byref(n)))
    out = np.empty(n.value)
    _check(_lib.cmcg_result_history(r.h, _ptr(out), n.value, C.byref(n)))
    return out


def cmcg_debug_rhs(p: Problem, u_dev, out_dev, t: float = 0.0, with_source: bool = True,
                   opts: cmcg_options | None = None, stream=None):
    o = opts or cmcg_options_default()
    _check(_lib.cmcg_debug_rhs(p.h, C.byref(o), float(t), int(with_source), _ptr(u_dev), _ptr(out_dev),
                               _stream(stream)))


def cmcg_debug_period(p: Problem, u0_dev, ut_dev, direction: int = 1, with_source: bool = False,
                      f_re_dev=None, f_im_dev=None, opts: cmcg_options | None = None, stream=None):
    o = opts or cmcg_options_default()
    _check(_lib.cmcg_debug_period(p.h, C.byref(o), int(direction), int(with_source), _ptr(u0_dev), _ptr(ut_dev),
                                  _ptr(f_re_dev), _ptr(f_im_dev), _stream(stream)))


def cmcg_debug_step(p: Problem, u_dev, out_dev, m: int = 0, direction: int = 1, with_source: bool = False,
                    opts: cmcg_options | None = None, stream=None):
    o = opts or cmcg_options_default()
    _check(_lib.cmcg_debug_step(p.h, C.byref(o), int(m), int(direction), int(with_source), _ptr(u_dev),
                                _ptr(out_dev), _stream(stream)))


def cmcg_debug_dot(p: Problem, u_dev, v_dev, stream=None) -> float:
    out = C.c_double()
    _check(_lib.cmcg_debug_dot(p.h, _ptr(u_dev), _ptr(v_dev), C.byref(out), _stream(stream)))
    return out.value


def cmcg_debug_dot_noalloc(p: Problem, u_dev, v_dev, out_dev, stream=None):
    """(U, V)_{eps,mu} into out_dev[0] (device), asynchronous on `stream`,
    with no allocation (fixed per-GPU scratch array)."""
    _check(_lib.cmcg_debug_dot_noalloc(p.h, _ptr(u_dev), _ptr(v_dev), _ptr(out_dev), _stream(stream)))


def cmcg_debug_mfma(precision: int, a_dev, b_dev, d_dev, stream=None):
    """D [16,16] = A [16,4] B [4,16] on one matrix-core instruction (device FP64 arrays)."""
    _check(_lib.cmcg_debug_mfma(int(precision), _ptr(a_dev), _ptr(b_dev), _ptr(d_dev), _stream(stream)))


def cmcg_tune_stage(q: int, precision: int, variant: int):
    _check(_lib.cmcg_tune_stage(q, precision, variant))


def cmcg_tune_get_stage(q: int, precision: int) -> int:
    """The current choice for (q, precision); -1 = chosen per launch from its size."""
    v = C.c_int()
    _check(_lib.cmcg_tune_get_stage(q, precision, C.byref(v)))
    return v.value


def cmcg_tune_resolve_stage(q: int, precision: int, K: int, members: int = 1) -> int:
    """The variant a launch over K elements and `members` members runs now."""
    v = C.c_int()
    _check(_lib.cmcg_tune_resolve_stage(q, precision, int(K), int(members), C.byref(v)))
    return v.value


def cmcg_mesh_locality_order(xyz, tet) -> np.ndarray:
    """Permutation of the elements along a Morton curve of their centroids:
    build the mesh from tet[order] (and permute every per-element input alike)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tet = np.ascontiguousarray(tet, dtype=np.int64)
    order = np.empty(tet.shape[0], dtype=np.int64)
    _check(_lib.cmcg_mesh_locality_order(xyz.shape[0], _ptr(xyz), tet.shape[0], _ptr(tet), _ptr(order)))
    return order


def cmcg_autotune_stage(p: Problem, opts: cmcg_options | None = None, stream=None):
    """(chosen variant, [microseconds per stage launch of every variant, 0 = not applicable])."""
    o = opts or cmcg_options_default()
    v = C.c_int()
    us = (C.c_double * CMCG_STAGE_VARIANTS)()
    _check(_lib.cmcg_autotune_stage(p.h, C.byref(o), _stream(stream), C.byref(v), us))
    return v.value, list(us)


def cmcg_autotune_batch(problems, opts: cmcg_options | None = None, stream=None):
    """(chosen variant, [microseconds per batched stage launch of every
    variant with all members active, 0 = not applicable])."""
    o = opts or cmcg_options_default()
    n = len(problems)
    arr = (P * n)(*[p.h for p in problems])
    v = C.c_int()
    us = (C.c_double * CMCG_STAGE_VARIANTS)()
    _check(_lib.cmcg_autotune_batch(arr, n, C.byref(o), _stream(stream), C.byref(v), us))
    return v.value, list(us)


class Engine(_Handle):
    _destroy = "cmcg_engine_destroy"


def cmcg_problem_footprint(p: Problem) -> int:
    b = C.c_size_t()
    _check(_lib.cmcg_problem_footprint(p.h, C.byref(b)))
    return b.value


def cmcg_engine_create(hbm_budget: int, max_slots: int) -> Engine:
    h = P()
    _check(_lib.cmcg_engine_create(int(hbm_budget), int(max_slots), C.byref(h)))
    return Engine(h)


def cmcg_engine_admit(e: Engine, p: Problem, opts: cmcg_options | None = None):
    """Slot index, or None when the request does not fit now (keep it queued).
    Raises CmcgError with code CMCG_ERR_TOO_LARGE when it never can."""
    o = opts or cmcg_options_default()
    slot = C.c_int(-1)
    rc = _lib.cmcg_engine_admit(e.h, p.h, C.byref(o), C.byref(slot))
    if rc == CMCG_ERR_NOMEM:
        return None
    _check(rc)
    return slot.value


def cmcg_engine_step(e: Engine):
    r, f = C.c_int(), C.c_int()
    _check(_lib.cmcg_engine_step(e.h, C.byref(r), C.byref(f)))
    return r.value, f.value


def cmcg_engine_poll(e: Engine, slot: int) -> int:
    st = C.c_int()
    _check(_lib.cmcg_engine_poll(e.h, slot, C.byref(st)))
    return st.value


def cmcg_engine_collect(e: Engine, slot: int, problem: Problem | None = None) -> Result:
    h = P()
    _check(_lib.cmcg_engine_collect(e.h, slot, C.byref(h)), allow=(CMCG_OK, CMCG_NOT_CONVERGED))
    return Result(h, keep=(problem,) if problem is not None else ())


def cmcg_engine_admit_batch(e: Engine, problems, opts: cmcg_options | None = None):
    """Slot index of a co-batched slot holding `problems` (one space), or None
    when it does not fit now.  Raises CmcgError (CMCG_ERR_TOO_LARGE) when it
    never can."""
    o = opts or cmcg_options_default()
    n = len(problems)
    arr = (P * n)(*[p.h for p in problems])
    slot = C.c_int(-1)
    rc = _lib.cmcg_engine_admit_batch(e.h, arr, n, C.byref(o), C.byref(slot))
    if rc == CMCG_ERR_NOMEM:
        return None
    _check(rc)
    return slot.value


def cmcg_engine_slot_members(e: Engine, slot: int) -> int:
    n = C.c_int()
    _check(_lib.cmcg_engine_slot_members(e.h, slot, C.byref(n)))
    return n.value


def cmcg_engine_collect_batch(e: Engine, slot: int, problems) -> list:
    n = len(problems)
    res = (P * n)()
    _check(_lib.cmcg_engine_collect_batch(e.h, slot, res, n), allow=(CMCG_OK, CMCG_NOT_CONVERGED))
    return [Result(P(res[b]), keep=(problems[b],)) for b in range(n)]


def cmcg_engine_cancel(e: Engine, slot: int):
    _check(_lib.cmcg_engine_cancel(e.h, slot))


def cmcg_engine_info(e: Engine):
    u, r, f = C.c_size_t(), C.c_int(), C.c_int()
    _check(_lib.cmcg_engine_info(e.h, C.byref(u), C.byref(r), C.byref(f)))
    return dict(used=u.value, running=r.value, finished=f.value)
