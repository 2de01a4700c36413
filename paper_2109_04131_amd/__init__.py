"""Python binding of the MI355X usFFT library (C ABI in include/usfft.h).

Argument marshalling only: every step runs in the HIP kernels of
libusfft.so.  Device buffers are torch tensors on the GPU (their data
pointers are passed), host arrays are numpy arrays.  Importing this module
fails loudly when the built library is missing; there is no CPU path.
"""
import ctypes as C
import os
import sys

import numpy as np
# PyTorch ships its own HIP runtime under the soname the library links
# against.  Loading torch first lets the library bind to that runtime, so the
# process holds one HIP runtime; loaded the other way round, both runtimes end
# up mapped and torch then finds no GPU.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libusfft.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libusfft.so is not built: run __graft_entry__.build() (hipcc, gfx950)")
_lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ELATTICE = 0, -1, -2, -3, -4, -5
SAMPLER_PDE, SAMPLER_TRIG_POLY, SAMPLER_PDE_MESH = 0, 1, 2
FP64, FP32_REFINE = 0, 1
OUT_MAG2, OUT_COMPLEX = 0, 1
PRECOND_DST, PRECOND_JACOBI = 0, 1
MODEL_PERIODIC, MODEL_AFFINE, MODEL_LOGNORMAL = 0, 1, 2
KIND_LAT2, KIND_LAT3 = 3, 4

_P32 = C.POINTER(C.c_int32)
_PD = C.POINTER(C.c_double)


class _Problem(C.Structure):
    _fields_ = [("d", C.c_int32), ("k_lo", _P32), ("k_hi", _P32), ("sampler", C.c_int32),
                ("mesh_n", C.c_int32), ("a0", C.c_double), ("amp", _PD), ("mode1", _P32), ("mode2", _P32),
                ("G_poly", C.c_int64), ("n_poly", C.c_int64), ("poly_k", _P32), ("poly_c", _PD),
                ("model", C.c_int32), ("alpha", C.c_double), ("beta", C.c_double), ("delta", C.c_double),
                ("basis1", C.c_int32), ("basis2", C.c_int32),
                ("mesh_nv", C.c_int32), ("mesh_nt", C.c_int32), ("mesh_xy", _PD), ("mesh_tri", _P32),
                ("mesh_boundary", C.POINTER(C.c_uint8)), ("n_nodes", C.c_int64), ("nodes_xy", _PD)]


class _Params(C.Structure):
    _fields_ = [("s", C.c_int32), ("s_local", C.c_int32), ("r", C.c_int32), ("theta", C.c_double),
                ("theta_relative", C.c_int32), ("tie_rel", C.c_double), ("precision", C.c_int32),
                ("lattice_c", C.c_double), ("lattice_tries", C.c_int32), ("lattice_max", C.c_int32),
                ("lattice_mmax", C.c_int32), ("pcg_rtol", C.c_double), ("pcg_maxit", C.c_int32),
                ("inner_rtol", C.c_double), ("refine_every", C.c_int32), ("solver_config", C.c_int32),
                ("precond", C.c_int32), ("trace", C.c_int32), ("autotune", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("samples", C.c_int64), ("samples_step1", C.c_int64), ("samples_step2", C.c_int64),
                ("samples_step3", C.c_int64), ("lattices", C.c_int64), ("max_candidates", C.c_int64),
                ("pcg_iterations", C.c_int64), ("sample_launches", C.c_int64), ("dft_launches", C.c_int64),
                ("solver_block", C.c_int64), ("solver_npt", C.c_int64), ("solver_kind", C.c_int64),
                ("theta_abs", C.c_double), ("ms_sample", C.c_double),
                ("ms_dft", C.c_double), ("ms_select", C.c_double), ("ms_total", C.c_double),
                ("dft_bytes", C.c_double), ("max_batch", C.c_int64), ("max_family", C.c_int64),
                ("workspace_bytes", C.c_int64), ("plan_reused", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = C.c_void_p
_sigs = {
    "usfft_last_error": (C.c_char_p, []),
    "usfft_version": (C.c_char_p, []),
    "usfft_plan_create": (C.c_int, [C.POINTER(_Problem), C.POINTER(_Params), C.POINTER(_vp)]),
    "usfft_plan_destroy": (None, [_vp]),
    "usfft_tune_save": (C.c_int, [C.c_char_p]),
    "usfft_tune_load": (C.c_int, [C.c_char_p]),
    "usfft_tune_clear": (C.c_int, []),
    "usfft_plan_nodes": (C.c_int64, [_vp]),
    "usfft_detect": (C.c_int, [_vp, C.c_uint64, _vp, C.POINTER(_vp)]),
    "usfft_detect_batch": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, _vp]),
    "usfft_plan_workspace": (C.c_int, [_vp, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "usfft_detect_ws": (C.c_int, [_vp, C.c_uint64, C.c_int64, C.c_int64, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "usfft_coefficients_ws": (C.c_int, [_vp, _vp, C.c_int64, C.c_uint64, C.c_int64, C.c_int64, _vp, C.c_size_t,
                                        _vp, C.POINTER(_vp)]),
    "usfft_result_info": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                    C.POINTER(Stats)]),
    "usfft_result_copy": (C.c_int, [_vp, _vp, _vp]),
    "usfft_result_destroy": (None, [_vp]),
    "usfft_result_trace": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int64), _vp]),
    "usfft_eval": (C.c_int, [_vp, _vp, C.c_int64, _vp, _vp]),
    "usfft_eval_noalloc": (C.c_int, [_vp, _vp, C.c_int64, _vp, _vp]),
    "usfft_statistics": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "usfft_coefficients": (C.c_int, [_vp, _vp, C.c_int64, C.c_uint64, _vp, _vp]),
    "usfft_errors": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.c_double, _vp, _vp, _vp]),
    "usfft_sample": (C.c_int, [_vp, _vp, C.c_int64, _vp, C.c_int32, C.c_int64, C.c_int64, _vp, _vp]),
    "usfft_nodes": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp]),
    "usfft_line_dft": (C.c_int, [_vp, C.c_int32, C.c_int64, C.c_int64, C.c_int64, C.c_int32, _vp, C.c_int32,
                                 C.c_int32, _vp, C.c_int64, _vp]),
    "usfft_lattice_dft": (C.c_int, [_vp, C.c_int32, C.c_int64, C.c_int64, C.c_int64, C.c_int32, _vp, _vp,
                                    C.c_int32, C.c_int32, _vp, C.c_int64, _vp]),
    "usfft_lattice_coeffs": (C.c_int, [_vp, C.c_int32, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32, _vp,
                                       _vp, C.c_int64, _vp, _vp]),
    "usfft_select": (C.c_int, [_vp, C.c_int64, C.c_int64, C.c_int64, C.c_int32, _vp, C.c_double, _vp, _vp, _vp]),
    "usfft_product": (C.c_int, [_vp, C.c_int64, C.c_int32, _vp, C.c_int64, _vp, _vp]),
    "usfft_compact": (C.c_int, [_vp, _vp, C.c_int64, C.c_int32, _vp, C.POINTER(C.c_int64), _vp]),
    "usfft_server_create": (C.c_int, [_vp, C.POINTER(_vp)]),
    "usfft_server_submit": (C.c_int, [_vp, _vp, _vp, C.c_uint64, C.POINTER(C.c_uint64)]),
    "usfft_server_poll": (C.c_int, [_vp, C.c_uint64, C.c_int32, C.POINTER(_vp), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "usfft_server_destroy": (None, [_vp]),
    "usfft_family": (C.c_int, [_vp, C.c_int64, C.c_int32, C.c_double, C.c_int32, C.c_int32, C.c_int32,
                               C.c_uint64, C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_sigs)


class UsfftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("usfft status %d: %s" % (status, msg))
        self.status = status


def _check(st):
    if st != OK:
        raise UsfftError(st, _lib.usfft_last_error().decode())


def _ptr(x):
    """Device pointer of a torch tensor, host pointer of a numpy array, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        # torch's current stream when the caller works with torch on the GPU,
        # else the default stream (torch's default stream is that stream too)
        torch = sys.modules.get("torch")
        if torch is None or not torch.cuda.is_initialized():
            return 0
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def version():
    return _lib.usfft_version().decode()


DEFAULT_PARAMS = dict(s=50, s_local=50, r=5, theta=1e-12, theta_relative=False, tie_rel=2.0 ** -30,
                      precision=FP64, lattice_c=2.0, lattice_tries=8, lattice_max=64, lattice_mmax=9601,
                      pcg_rtol=1e-12, pcg_maxit=4000, inner_rtol=2e-4, refine_every=200, solver_config=-1,
                      precond=0, trace=False, autotune=False)


def _marshal(problem, params):
    """Problem and params structures plus the numpy arrays they point into."""
    p = dict(DEFAULT_PARAMS)
    p.update({k: v for k, v in params.items() if k in DEFAULT_PARAMS})
    keep = []

    def arr(v, dt):
        a = np.ascontiguousarray(np.asarray(v, dtype=dt))
        keep.append(a)
        return a.ctypes.data_as(_P32 if dt == np.int32 else _PD)

    pr = _Problem()
    pr.d = int(problem["d"])
    pr.k_lo = arr(problem["k_lo"], np.int32)
    pr.k_hi = arr(problem["k_hi"], np.int32)
    kind = problem.get("sampler", "pde")
    if kind in ("pde", "pde_mesh"):
        if kind == "pde":
            pr.sampler = SAMPLER_PDE
            pr.mesh_n = int(problem["mesh_n"])
        else:
            pr.sampler = SAMPLER_PDE_MESH
            xy = np.ascontiguousarray(np.asarray(problem["mesh_xy"], dtype=np.float64))
            tri = np.ascontiguousarray(np.asarray(problem["mesh_tri"], dtype=np.int32))
            bnd = np.ascontiguousarray(np.asarray(problem["mesh_boundary"], dtype=np.uint8))
            keep.extend([xy, tri, bnd])
            pr.mesh_nv, pr.mesh_nt = len(xy), len(tri)
            pr.mesh_xy = xy.ctypes.data_as(_PD)
            pr.mesh_tri = tri.ctypes.data_as(_P32)
            pr.mesh_boundary = bnd.ctypes.data_as(C.POINTER(C.c_uint8))
        pr.a0 = float(problem.get("a0", 1.0))
        pr.amp = arr(problem["amp"], np.float64)
        pr.mode1 = arr(problem["mode1"], np.int32)
        pr.mode2 = arr(problem["mode2"], np.int32)
        pr.model = int(problem.get("model", MODEL_PERIODIC))
        pr.alpha = float(problem.get("alpha", -1.0))
        pr.beta = float(problem.get("beta", 1.0))
        pr.delta = float(problem.get("delta", 0.0))
        pr.basis1 = int(problem.get("basis1", 0))
        pr.basis2 = int(problem.get("basis2", 0))
        if problem.get("nodes_xy") is not None:
            pts = np.ascontiguousarray(np.asarray(problem["nodes_xy"], dtype=np.float64).reshape(-1, 2))
            keep.append(pts)
            pr.n_nodes = len(pts)
            pr.nodes_xy = pts.ctypes.data_as(_PD)
    else:
        pr.sampler = SAMPLER_TRIG_POLY
        K = np.asarray(problem["poly_k"])
        P = np.asarray(problem["poly_c"], dtype=np.complex128)
        pr.n_poly, pr.G_poly = P.shape
        pr.poly_k = arr(K, np.int32)
        pr.poly_c = arr(np.stack([P.real, P.imag], -1), np.float64)
    pa = _Params()
    for k in DEFAULT_PARAMS:
        setattr(pa, k, type(DEFAULT_PARAMS[k])(p[k]) if not isinstance(DEFAULT_PARAMS[k], bool) else int(p[k]))
    return pr, pa, keep, p


class Plan:
    """usfft_plan_create / usfft_plan_destroy."""

    def __init__(self, problem, params):
        pr, pa, keep, p = _marshal(problem, params)
        self.d = pr.d
        h = _vp()
        _check(_lib.usfft_plan_create(C.byref(pr), C.byref(pa), C.byref(h)))
        self.handle = h
        self.params = p
        self.G = int(_lib.usfft_plan_nodes(h))

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.usfft_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()


class _ServerCfg(C.Structure):
    _fields_ = [("max_active", C.c_int32), ("hbm_budget", C.c_uint64)]


class Server:
    """usfft_server_*: continuous batching of whole jobs on worker streams."""

    def __init__(self, max_active=4, hbm_budget=0):
        cfg = _ServerCfg(max_active, hbm_budget)
        h = _vp()
        _check(_lib.usfft_server_create(C.byref(cfg), C.byref(h)))
        self.handle = h

    def submit(self, problem, params, seed):
        pr, pa, keep, _ = _marshal(problem, params)
        job = C.c_uint64()
        _check(_lib.usfft_server_submit(self.handle, C.byref(pr), C.byref(pa), C.c_uint64(seed), C.byref(job)))
        return job.value

    def poll(self, job, wait=False):
        """(Result or None, status, latency_s, queue_s); status 1 = pending."""
        h = _vp()
        st = C.c_int32()
        lat = C.c_double()
        q = C.c_double()
        _check(_lib.usfft_server_poll(self.handle, C.c_uint64(job), int(wait), C.byref(h), C.byref(st),
                                      C.byref(lat), C.byref(q)))
        res = Result(h) if h.value else None
        err = _lib.usfft_last_error().decode() if st.value not in (OK, 1) else ""
        return res, st.value, lat.value, q.value, err

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.usfft_server_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()


class Result:
    """usfft_result_info / usfft_result_copy / usfft_result_destroy."""

    def __init__(self, handle):
        self.handle = handle
        n = C.c_int64()
        d = C.c_int32()
        G = C.c_int64()
        st = Stats()
        _check(_lib.usfft_result_info(handle, C.byref(n), C.byref(d), C.byref(G), C.byref(st)))
        self.n, self.d, self.G = n.value, d.value, G.value
        self.stats = st.as_dict()

    def freqs(self):
        out = np.zeros((self.n, self.d), dtype=np.int32)
        _check(_lib.usfft_result_copy(self.handle, out.ctypes.data if self.n else None, None))
        return out

    def coeffs(self):
        out = np.zeros((self.n, self.G, 2), dtype=np.float64)
        _check(_lib.usfft_result_copy(self.handle, None, out.ctypes.data if self.n else None))
        return out[..., 0] + 1j * out[..., 1]

    def trace(self):
        """usfft_result_trace: [(set (n x width int32), n_cand)] for the d
        step-1 sets I^(t), then the d - 1 step-2 sets I^(1..t)."""
        out = []
        for stage in range(2 * self.d - 1):
            n = C.c_int64()
            w = C.c_int32()
            nc = C.c_int64()
            _check(_lib.usfft_result_trace(self.handle, stage, C.byref(n), C.byref(w), C.byref(nc), None))
            a = np.zeros((n.value, w.value), dtype=np.int32)
            _check(_lib.usfft_result_trace(self.handle, stage, C.byref(n), C.byref(w), C.byref(nc),
                                           a.ctypes.data if a.size else None))
            out.append((a, nc.value))
        return out

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.usfft_result_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()


def tune_save(path):
    """usfft_tune_save: the tuning cache as JSON."""
    _check(_lib.usfft_tune_save(os.fsencode(path)))


def tune_load(path):
    """usfft_tune_load: merge a saved tuning cache."""
    _check(_lib.usfft_tune_load(os.fsencode(path)))


def tune_clear():
    _check(_lib.usfft_tune_clear())


def plan_create(problem, params):
    return Plan(problem, params)


def detect(plan, seed, stream=None):
    h = _vp()
    _check(_lib.usfft_detect(plan.handle, C.c_uint64(seed), _stream(stream), C.byref(h)))
    return Result(h)


def plan_workspace(plan, n_cand_max, samples_max):
    """usfft_plan_workspace: device bytes of the _ws calls for these bounds."""
    b = C.c_size_t()
    _check(_lib.usfft_plan_workspace(plan.handle, int(n_cand_max), int(samples_max), C.byref(b)))
    return b.value


def detect_ws(plan, seed, n_cand_max, samples_max, ws, ws_bytes=None, stream=None):
    """usfft_detect_ws: usfft_detect inside the caller's workspace (a device
    tensor); the result's coefficients live in that workspace."""
    nb = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    h = _vp()
    _check(_lib.usfft_detect_ws(plan.handle, C.c_uint64(seed), int(n_cand_max), int(samples_max), _ptr(ws), nb,
                                _stream(stream), C.byref(h)))
    return Result(h)


def coefficients_ws(plan, freqs, seed, n_cand_max, samples_max, ws, ws_bytes=None, stream=None):
    """usfft_coefficients_ws: usfft_coefficients inside the caller's workspace."""
    F = np.ascontiguousarray(np.asarray(freqs, dtype=np.int32).reshape(-1, plan.d))
    nb = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    h = _vp()
    _check(_lib.usfft_coefficients_ws(plan.handle, F.ctypes.data if F.size else None, F.shape[0], C.c_uint64(seed),
                                      int(n_cand_max), int(samples_max), _ptr(ws), nb, _stream(stream), C.byref(h)))
    return Result(h)


def detect_batch(plans, seeds):
    """usfft_detect_batch: jobs run together with their solver launches fused.
    Returns ([Result or None], [status], (launches, fused launches, segments))."""
    n = len(plans)
    hs = (_vp * n)(*[p.handle.value for p in plans])
    sd = (C.c_uint64 * n)(*seeds)
    outs = (_vp * n)()
    sts = (C.c_int * n)()
    fs = (C.c_int64 * 3)()
    st = _lib.usfft_detect_batch(hs, n, sd, outs, sts, fs)
    res = [Result(_vp(outs[i])) if outs[i] else None for i in range(n)]
    if st != OK and all(r is None for r in res):
        _check(st)
    return res, list(sts), tuple(fs)


def coefficients(plan, freqs, seed, stream=None):
    """usfft_coefficients: step 3 alone on the given frequencies (n x d)."""
    F = np.ascontiguousarray(np.asarray(freqs, dtype=np.int32).reshape(-1, plan.d))
    h = _vp()
    _check(_lib.usfft_coefficients(plan.handle, F.ctypes.data if F.size else None, F.shape[0], C.c_uint64(seed),
                                   _stream(stream), C.byref(h)))
    return Result(h)


def eval(result, y, out, stream=None):
    _check(_lib.usfft_eval(result.handle, _ptr(y), y.shape[0], _ptr(out), _stream(stream)))


def eval_noalloc(result, y, out, stream=None):
    """usfft_eval_noalloc: usfft_eval with the library's fixed device scratch."""
    _check(_lib.usfft_eval_noalloc(result.handle, _ptr(y), y.shape[0], _ptr(out), _stream(stream)))


def statistics(result, mean=None, var=None, gsi=None, stream=None):
    """usfft_statistics: mean (G x 2 float64), var (G), gsi (d x G); any may be None."""
    _check(_lib.usfft_statistics(result.handle, _ptr(mean), _ptr(var), _ptr(gsi), _stream(stream)))


def errors(plan, result, y, p, errp, errinf, stream=None):
    """usfft_errors: err_p and err_inf per node over the test parameters y (n x d)."""
    _check(_lib.usfft_errors(plan.handle, result.handle, _ptr(y), y.shape[0], float(p), _ptr(errp), _ptr(errinf),
                             _stream(stream)))


def sample(plan, y, u, out_fp32, ld, col0=0, iters=None, stream=None):
    _check(_lib.usfft_sample(plan.handle, _ptr(y), y.shape[0], _ptr(u), int(out_fp32), ld, col0, _ptr(iters),
                             _stream(stream)))


def nodes(d, line, t, M, z, tail, y, stream=None):
    M = np.ascontiguousarray(np.asarray(M, dtype=np.int32).reshape(-1))
    z = np.ascontiguousarray(np.asarray(z if z is not None else [0], dtype=np.int32).reshape(-1))
    tail = np.ascontiguousarray(np.asarray(tail, dtype=np.float64))
    _check(_lib.usfft_nodes(d, line, t, len(M), M.ctypes.data, z.ctypes.data, tail.ctypes.data, _ptr(y),
                            _stream(stream)))


def line_dft(u, u_fp32, G, ld, col0, K, bins, out_kind, out, ldo, stream=None):
    bins = np.ascontiguousarray(np.asarray(bins, dtype=np.int32))
    _check(_lib.usfft_line_dft(_ptr(u), int(u_fp32), G, ld, col0, K, bins.ctypes.data, len(bins), out_kind,
                               _ptr(out), ldo, _stream(stream)))


def lattice_dft(u, u_fp32, G, ld, col0, M, bins, pos, out_kind, out, ldo, stream=None):
    _check(_lib.usfft_lattice_dft(_ptr(u), int(u_fp32), G, ld, col0, M, _ptr(bins), _ptr(pos), bins.shape[0],
                                  out_kind, _ptr(out), ldo, _stream(stream)))


def lattice_coeffs(u, u_fp32, G, ld, col0, M, z, J, out, stream=None):
    """usfft_lattice_coeffs: Algorithm A on one lattice (M, z) for the candidates J (device, n x t)."""
    z = np.ascontiguousarray(np.asarray(z, dtype=np.int64).reshape(-1))
    _check(_lib.usfft_lattice_coeffs(_ptr(u), int(u_fp32), G, ld, col0, int(M), len(z), z.ctypes.data, _ptr(J),
                                     J.shape[0], _ptr(out), _stream(stream)))


def select(v, G, n, ld, s_tilde, theta2, tie_rel, mask, thr=None, stream=None):
    _check(_lib.usfft_select(_ptr(v), G, n, ld, s_tilde, _ptr(theta2), tie_rel, _ptr(mask), _ptr(thr),
                             _stream(stream)))


def product(parent, np_, t, child, nc, out, stream=None):
    _check(_lib.usfft_product(_ptr(parent), np_, t, _ptr(child), nc, _ptr(out), _stream(stream)))


def compact(J, mask, n, t, out, stream=None):
    cnt = C.c_int64()
    _check(_lib.usfft_compact(_ptr(J), _ptr(mask), n, t, _ptr(out), C.byref(cnt), _stream(stream)))
    return cnt.value


def family(J, n, t, c, mmax, tries, lmax, seed, kind, tcode, assign, bins, cap=256, stream=None):
    nl = C.c_int32()
    Ms = np.zeros(cap, dtype=np.int32)
    zs = np.zeros(cap * t, dtype=np.int32)
    _check(_lib.usfft_family(_ptr(J), n, t, c, mmax, tries, lmax, C.c_uint64(seed), kind, tcode, cap,
                             C.byref(nl), Ms.ctypes.data, zs.ctypes.data, _ptr(assign), _ptr(bins),
                             _stream(stream)))
    L = nl.value
    return [int(m) for m in Ms[:L]], zs[: L * t].reshape(L, t).tolist()
