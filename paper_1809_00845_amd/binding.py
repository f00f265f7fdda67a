"""ctypes binding of libbemfft.so -- argument marshalling only.

Every step of the operator and the solve runs in the HIP library; this
module converts numpy/torch arguments to pointers and status codes to
exceptions.  It raises if the library is missing: there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbemfft.so")

LAPLACE2D, LAPLACE3D, NAVIER3D, HALFSPACE = 0, 1, 2, 3
FP64, FP32, BF16_MFMA = 0, 1, 2
C_HALF, C_USER, C_IMPLICIT = 0, 1, 2
OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EBREAKDOWN, ENOCONV = 0, -1, -2, -3, -4, -5, 1


class bemfft_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double),
                ("origin", ctypes.c_double * 3), ("pad", ctypes.c_int64 * 3)]


class bemfft_plan_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("c_mode", ctypes.c_int),
                ("c_user", ctypes.POINTER(ctypes.c_double)), ("stream", ctypes.c_void_p),
                ("keep_fp64", ctypes.c_int), ("autotune", ctypes.c_int), ("cell_quad", ctypes.c_int)]


class bemfft_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
                ("precond", ctypes.c_int), ("use_x0", ctypes.c_int), ("refine", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int)]


class bemfft_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("true_relres", ctypes.c_double),
                ("status", ctypes.c_int), ("seconds", ctypes.c_double), ("outer", ctypes.c_int),
                ("applies64", ctypes.c_int), ("x0_used", ctypes.c_int), ("x0_relres", ctypes.c_double)]


class bemfft_plan_info(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("kernel", ctypes.c_int), ("precision", ctypes.c_int),
                ("c_mode", ctypes.c_int), ("m", ctypes.c_int64), ("ncomp", ctypes.c_int64),
                ("n", ctypes.c_int64 * 3), ("pad", ctypes.c_int64 * 3), ("z_lo", ctypes.c_int64),
                ("z_count", ctypes.c_int64), ("nfields", ctypes.c_int64), ("nspectra", ctypes.c_int64),
                ("noutputs", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("spectra_bytes", ctypes.c_int64), ("spectrum_parity_residual", ctypes.c_double),
                ("plan_seconds", ctypes.c_double), ("zsched", ctypes.c_int), ("tune_us", ctypes.c_double * 3),
                ("fwd_xg", ctypes.c_int), ("fwd_tune_us", ctypes.c_double * 2)]


EXPORTS = [
    "bemfft_plan_create", "bemfft_apply", "bemfft_apply_profile", "bemfft_solve", "bemfft_plan_get_info", "bemfft_plan_get_c",
    "bemfft_plan_destroy", "bemfft_fft3d_c2c_f64", "bemfft_strerror", "bemfft_last_error",
    "bemfft_supported_sizes", "bemfft_batch_create", "bemfft_batch_apply", "bemfft_batch_solve",
    "bemfft_batch_members", "bemfft_batch_destroy", "bemfft_net_create", "bemfft_net_destroy",
    "bemfft_net_num_params", "bemfft_net_get_params", "bemfft_net_set_params", "bemfft_net_input",
    "bemfft_net_forward", "bemfft_net_infer", "bemfft_net_gradients", "bemfft_net_train_step", "bemfft_net_guess",
    "bemfft_plan_node_voxels", "bemfft_eval_grid", "bemfft_solve_cg", "bemfft_solve_noalloc",
]

NOALLOC_SCRATCH_BYTES = 32 << 20  # BEMFFT_NOALLOC_SCRATCH_BYTES

_lib = None


class BemfftError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status}): {last_error()}")


def load():
    """Load the HIP library (built by paper_1809_00845_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_1809_00845_amd.build.build() first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    L.bemfft_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(bemfft_grid), i64, dp, dp, dp,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.POINTER(bemfft_plan_opts)]
    L.bemfft_apply.argtypes = [vp, vp, vp, vp, vp]
    L.bemfft_eval_grid.argtypes = [vp, vp, vp, vp, vp]
    L.bemfft_apply_profile.argtypes = [vp, vp, vp, vp, ctypes.c_int, dp, vp]
    L.bemfft_solve.argtypes = [vp, vp, vp, vp, ctypes.POINTER(bemfft_solve_opts),
                               ctypes.POINTER(bemfft_solve_info), vp]
    L.bemfft_solve_noalloc.argtypes = [vp, vp, vp, vp, ctypes.POINTER(bemfft_solve_opts),
                                       ctypes.POINTER(bemfft_solve_info), vp]
    L.bemfft_solve_cg.argtypes = [vp, vp, vp, ctypes.POINTER(bemfft_solve_opts), ctypes.POINTER(bemfft_solve_info),
                                  vp]
    L.bemfft_plan_get_info.argtypes = [vp, ctypes.POINTER(bemfft_plan_info)]
    L.bemfft_plan_get_c.argtypes = [vp, dp]
    L.bemfft_plan_destroy.argtypes = [vp]
    L.bemfft_fft3d_c2c_f64.argtypes = [vp, i64, i64, i64, ctypes.c_int, vp]
    L.bemfft_strerror.argtypes = [ctypes.c_int]
    L.bemfft_strerror.restype = ctypes.c_char_p
    L.bemfft_last_error.restype = ctypes.c_char_p
    L.bemfft_supported_sizes.argtypes = [ctypes.POINTER(i64), ctypes.c_int]
    L.bemfft_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, vp]
    L.bemfft_batch_apply.argtypes = [vp, vp, vp, vp, vp]
    L.bemfft_batch_solve.argtypes = [vp, vp, vp, vp, ctypes.POINTER(bemfft_solve_opts),
                                     ctypes.POINTER(bemfft_solve_info), vp]
    L.bemfft_batch_members.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.bemfft_batch_destroy.argtypes = [vp]
    fp = ctypes.POINTER(ctypes.c_float)
    L.bemfft_net_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), ctypes.c_uint64, vp]
    L.bemfft_net_destroy.argtypes = [vp]
    L.bemfft_net_num_params.argtypes = [vp]
    L.bemfft_net_num_params.restype = i64
    L.bemfft_net_get_params.argtypes = [vp, fp]
    L.bemfft_net_set_params.argtypes = [vp, fp]
    L.bemfft_net_input.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, vp]
    L.bemfft_net_forward.argtypes = [vp, vp, vp, vp]
    L.bemfft_net_infer.argtypes = [vp, vp, vp, vp]
    L.bemfft_net_gradients.argtypes = [vp, vp, i64, vp, vp, vp, dp, fp, vp]
    L.bemfft_net_train_step.argtypes = [vp, vp, i64, vp, vp, vp, ctypes.c_float, dp, vp]
    L.bemfft_net_guess.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.bemfft_plan_node_voxels.argtypes = [vp, ctypes.POINTER(ctypes.c_int), dp]
    _lib = L
    return L


def strerror(status: int) -> str:
    return load().bemfft_strerror(status).decode()


def last_error() -> str:
    return load().bemfft_last_error().decode()


def _check(status, where):
    if status < 0:
        raise BemfftError(status, where)
    return status


def _ptr(t, n=None, dtype=None, name="tensor"):
    """Device pointer of a torch tensor.  The tensor must be a contiguous
    GPU tensor; with ``dtype`` it must have that torch dtype, with ``n``
    exactly n elements.  Checked here, before any library call, because the
    library trusts the sizes it is given."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t, n, name):
    import torch

    return _ptr(t, n, torch.float64, name)


def _u8(t, n, name):
    import torch

    return _ptr(t, n, torch.uint8, name)


def _plan_len(plan, n):
    """ncomp * m of a plan handle (looked up when the caller did not say)."""
    if n is not None:
        return int(n)
    inf = bemfft_plan_get_info(plan)
    return int(inf["ncomp"]) * int(inf["m"])


def _stream_ptr(stream):
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def supported_sizes():
    buf = (ctypes.c_int64 * 32)()
    n = load().bemfft_supported_sizes(buf, 32)
    return [int(buf[i]) for i in range(n)]


def bemfft_plan_create(dim, n, h, nodes, normals, weights, kernel, nu=0.3, mu=1.0, origin=(0.0, 0.0, 0.0),
                       pad=(0, 0, 0), precision=FP64, c_mode=C_IMPLICIT, c_user=None, stream=None, keep_fp64=False, autotune=0,
                       cell_quad=0):
    """Returns an opaque plan handle (ctypes.c_void_p)."""
    L = load()
    g = bemfft_grid()
    g.dim = dim
    for a in range(3):
        g.n[a] = int(n[a]) if a < len(n) else 1
        g.origin[a] = float(origin[a]) if a < len(origin) else 0.0
        g.pad[a] = int(pad[a]) if a < len(pad) else 0
    g.h = float(h)
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    m = nodes.shape[0]
    nptr = None
    if normals is not None:
        normals = np.ascontiguousarray(normals, dtype=np.float64)
        nptr = normals.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    wptr = None
    if weights is not None:
        weights = np.ascontiguousarray(weights, dtype=np.float64)
        wptr = weights.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    opts = bemfft_plan_opts()
    opts.precision = precision
    opts.c_mode = c_mode
    if c_user is not None:
        c_user = np.ascontiguousarray(c_user, dtype=np.float64)
        opts.c_user = c_user.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    opts.stream = _stream_ptr(stream) if stream is not None else None
    opts.keep_fp64 = 1 if keep_fp64 else 0
    opts.autotune = int(autotune)
    opts.cell_quad = int(cell_quad)
    h_ = ctypes.c_void_p()
    st = L.bemfft_plan_create(ctypes.byref(h_), ctypes.byref(g), m,
                              nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              nptr, wptr, kernel,
                              float(nu), float(mu), ctypes.byref(opts))
    _check(st, "bemfft_plan_create")
    return h_


def bemfft_apply(plan, q, u, r, stream=None, n=None):
    """n: ncomp * m of the plan (looked up if None)."""
    n = _plan_len(plan, n)
    return _check(load().bemfft_apply(plan, _f64(q, n, "q"), _f64(u, n, "u"), _f64(r, n, "r"),
                                      _stream_ptr(stream)), "bemfft_apply")


def bemfft_eval_grid(plan, q, u, out, stream=None, n=None):
    inf = bemfft_plan_get_info(plan)
    n = _plan_len(plan, n)
    nout = int(inf["ncomp"]) * int(inf["z_count"]) * int(inf["n"][1]) * int(inf["n"][0])
    return _check(load().bemfft_eval_grid(plan, _f64(q, n, "q"), _f64(u, n, "u"), _f64(out, nout, "out"),
                                          _stream_ptr(stream)), "bemfft_eval_grid")


def bemfft_apply_profile(plan, q, u, r, reps=10, stream=None, n=None):
    """Mean per-stage milliseconds (fwd_xy, zpass, inv_y, gather)."""
    n = _plan_len(plan, n)
    ms = (ctypes.c_double * 4)()
    _check(load().bemfft_apply_profile(plan, _f64(q, n, "q"), _f64(u, n, "u"), _f64(r, n, "r"), int(reps), ms,
                                       _stream_ptr(stream)), "bemfft_apply_profile")
    return [float(v) for v in ms]


def bemfft_solve(plan, bc, known, unknown, tol=1e-6, restart=100, maxit=1000, precond=1, use_x0=0,
                 refine=0, inner_tol=1e-4, max_outer=20, stream=None, n=None):
    n = _plan_len(plan, n)
    o = bemfft_solve_opts(tol, restart, maxit, precond, use_x0, refine, inner_tol, max_outer)
    info = bemfft_solve_info()
    st = load().bemfft_solve(plan, _u8(bc, n, "bc"), _f64(known, n, "known"), _f64(unknown, n, "unknown"),
                             ctypes.byref(o), ctypes.byref(info), _stream_ptr(stream))
    _check(st, "bemfft_solve")
    return {"status": st, "iters": info.iters, "restarts": info.restarts, "true_relres": info.true_relres,
            "seconds": info.seconds, "outer": info.outer, "applies64": info.applies64,
            "x0_used": info.x0_used, "x0_relres": info.x0_relres}


def bemfft_solve_noalloc(plan, bc, known, unknown, tol=1e-6, restart=100, maxit=1000, precond=1, use_x0=0,
                         refine=0, inner_tol=1e-4, max_outer=20, stream=None, n=None):
    """bemfft_solve with its workspace in the library's fixed device array
    (no allocation); same results."""
    n = _plan_len(plan, n)
    o = bemfft_solve_opts(tol, restart, maxit, precond, use_x0, refine, inner_tol, max_outer)
    info = bemfft_solve_info()
    st = load().bemfft_solve_noalloc(plan, _u8(bc, n, "bc"), _f64(known, n, "known"), _f64(unknown, n, "unknown"),
                                     ctypes.byref(o), ctypes.byref(info), _stream_ptr(stream))
    _check(st, "bemfft_solve_noalloc")
    return {"status": st, "iters": info.iters, "restarts": info.restarts, "true_relres": info.true_relres,
            "seconds": info.seconds, "outer": info.outer, "applies64": info.applies64,
            "x0_used": info.x0_used, "x0_relres": info.x0_relres}


def bemfft_solve_cg(plan, u, q, tol=1e-6, maxit=1000, precond=1, use_x0=0, stream=None, n=None):
    n = _plan_len(plan, n)
    o = bemfft_solve_opts(tol, 100, maxit, precond, use_x0, 0, 1e-4, 20)
    info = bemfft_solve_info()
    st = load().bemfft_solve_cg(plan, _f64(u, n, "u"), _f64(q, n, "q"), ctypes.byref(o), ctypes.byref(info),
                                _stream_ptr(stream))
    _check(st, "bemfft_solve_cg")
    return {"status": st, "iters": info.iters, "true_relres": info.true_relres, "seconds": info.seconds}


def bemfft_plan_get_info(plan):
    info = bemfft_plan_info()
    _check(load().bemfft_plan_get_info(plan, ctypes.byref(info)), "bemfft_plan_get_info")
    out = {}
    for name, _ in bemfft_plan_info._fields_:
        v = getattr(info, name)
        out[name] = list(v) if not isinstance(v, (int, float)) else v
    return out


def bemfft_plan_get_c(plan, m, ncomp):
    buf = np.zeros(m * ncomp * ncomp)
    _check(load().bemfft_plan_get_c(plan, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "bemfft_plan_get_c")
    return buf if ncomp == 1 else buf.reshape(m, ncomp, ncomp)


def bemfft_plan_destroy(plan):
    if plan is not None and plan.value:
        load().bemfft_plan_destroy(plan)


def bemfft_fft3d_c2c_f64(data, px, py, pz, direction, stream=None):
    import torch

    return _check(load().bemfft_fft3d_c2c_f64(_ptr(data, 2 * px * py * pz, torch.float64, "data"), px, py, pz,
                                              direction, _stream_ptr(stream)),
                  "bemfft_fft3d_c2c_f64")


class Plan:
    """Owns one plan; geometry from any object with dim/n/h/origin/nodes/
    normals/weights attributes."""

    def __init__(self, geom, kernel, precision=FP64, c_mode=C_IMPLICIT, c_user=None, nu=0.3, mu=1.0,
                 pad=(0, 0, 0), stream=None, keep_fp64=False, autotune=0, cell_quad=0):
        self.kernel = kernel
        self.ncomp = 3 if kernel in (NAVIER3D, HALFSPACE) else 1
        self.m = int(np.asarray(geom.weights).shape[0])
        self.handle = bemfft_plan_create(geom.dim, geom.n, geom.h, geom.nodes, geom.normals, geom.weights,
                                         kernel, nu, mu, origin=geom.origin, pad=pad, precision=precision,
                                         c_mode=c_mode, c_user=c_user, stream=stream, keep_fp64=keep_fp64,
                                         autotune=autotune, cell_quad=cell_quad)

    def apply(self, q, u, r=None, stream=None):
        import torch

        if r is None:
            r = torch.empty_like(u)
        bemfft_apply(self.handle, q, u, r, stream, n=self.ncomp * self.m)
        return r

    def eval_grid(self, q, u, out=None, stream=None):
        """S[q] - D[u] on the grid box [0, n0) x [0, n1) x [z_lo, z_lo + z_count):
        shape (ncomp, z_count, n1, n0) in 3D, (n1, n0) in 2D."""
        import torch

        inf = self.info()
        shape = (self.ncomp, inf["z_count"], inf["n"][1], inf["n"][0])
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=u.device)
        elif out.dtype != torch.float64 or out.numel() != int(np.prod(shape)):
            raise ValueError(f"eval_grid: out needs {shape} float64 values")
        bemfft_eval_grid(self.handle, q, u, out, stream, n=self.ncomp * self.m)
        if inf["dim"] == 2:
            return out[:, 0] if self.ncomp > 1 else out[0, 0]
        return out

    def solve(self, bc, known, unknown=None, **kw):
        import torch

        if unknown is None:
            unknown = torch.zeros_like(known, memory_format=torch.contiguous_format)
            kw.setdefault("use_x0", 0)
        info = bemfft_solve(self.handle, bc, known, unknown, n=self.ncomp * self.m, **kw)
        return unknown, info

    def solve_cg(self, u, q=None, **kw):
        """Dirichlet Laplace problem by CG on the symmetrised single-layer
        system: q with S[q] = c u + D[u]."""
        import torch

        if q is None:
            q = torch.zeros_like(u, memory_format=torch.contiguous_format)
            kw.setdefault("use_x0", 0)
        info = bemfft_solve_cg(self.handle, u, q, n=self.ncomp * self.m, **kw)
        return q, info

    def info(self):
        return bemfft_plan_get_info(self.handle)

    def c(self):
        return bemfft_plan_get_c(self.handle, self.m, self.ncomp)

    def close(self):
        bemfft_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None) is not None:
                self.close()
        except Exception:
            pass


class Batch:
    """Many plans x right-hand sides applied/solved together (concatenated
    device vectors; see bemfft_batch_* in include/bemfft.h)."""

    def __init__(self, plans, nrhs=1, use_graph=True, stream=None):
        self.plans = list(plans)  # keep the plans alive
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        self.handle = ctypes.c_void_p()
        _check(load().bemfft_batch_create(ctypes.byref(self.handle), arr, len(self.plans), int(nrhs),
                                          1 if use_graph else 0, _stream_ptr(stream)), "bemfft_batch_create")
        nm = len(self.plans) * nrhs
        off = (ctypes.c_int64 * nm)()
        ln = (ctypes.c_int64 * nm)()
        load().bemfft_batch_members(self.handle, off, ln)
        self.offsets = [int(v) for v in off]
        self.lengths = [int(v) for v in ln]
        self.total = self.offsets[-1] + self.lengths[-1]
        self.nrhs = nrhs

    def apply(self, q, u, r, stream=None):
        n = self.total
        return _check(load().bemfft_batch_apply(self.handle, _f64(q, n, "q"), _f64(u, n, "u"), _f64(r, n, "r"),
                                                _stream_ptr(stream)), "bemfft_batch_apply")

    def solve(self, bc, known, unknown, tol=1e-6, restart=100, maxit=1000, precond=1, use_x0=0, stream=None):
        nm = len(self.offsets)
        o = bemfft_solve_opts(tol, restart, maxit, precond, use_x0, 0, 1e-4, 20)
        info = (bemfft_solve_info * nm)()
        n = self.total
        st = load().bemfft_batch_solve(self.handle, _u8(bc, n, "bc"), _f64(known, n, "known"),
                                       _f64(unknown, n, "unknown"), ctypes.byref(o), info, _stream_ptr(stream))
        _check(st, "bemfft_batch_solve")
        return st, [{"iters": i.iters, "true_relres": i.true_relres, "status": i.status, "seconds": i.seconds}
                    for i in info]

    def close(self):
        if self.handle is not None and self.handle.value:
            load().bemfft_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_node_voxels(plan, m):
    """(voxel index int32[m], weight float64[m]) of each node, caller's order."""
    vox = np.zeros(m, dtype=np.int32)
    w = np.zeros(m)
    _check(load().bemfft_plan_node_voxels(plan, vox.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                          w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "bemfft_plan_node_voxels")
    return vox, w


class Net:
    """The learned-start network (bemfft_net_* in include/bemfft.h)."""

    def __init__(self, grid, dilations=(1, 2, 4, 8), width=16, seed=0, stream=None):
        self.grid = int(grid)
        self.dilations = list(dilations)
        dil = (ctypes.c_int * len(self.dilations))(*self.dilations)
        self.handle = ctypes.c_void_p()
        _check(load().bemfft_net_create(ctypes.byref(self.handle), self.grid, int(width), len(self.dilations), dil,
                                        ctypes.c_uint64(seed), _stream_ptr(stream) if stream is not None else None),
               "bemfft_net_create")
        self.nparam = int(load().bemfft_net_num_params(self.handle))
        self.V = self.grid ** 3

    def _targets(self, x, vox, tgt, wt):
        """Check the training arguments; returns the target count."""
        import torch

        nt = int(vox.numel())
        _ptr(x, 6 * self.V, torch.float32, "x")
        _ptr(vox, nt, torch.int32, "vox")
        _ptr(tgt, nt, torch.float32, "tgt")
        _ptr(wt, nt, torch.float32, "wt")
        return nt

    def params(self):
        buf = np.zeros(self.nparam, dtype=np.float32)
        _check(load().bemfft_net_get_params(self.handle, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "bemfft_net_get_params")
        return buf

    def set_params(self, params):
        params = np.ascontiguousarray(params, dtype=np.float32)
        if params.shape != (self.nparam,):
            raise ValueError(f"expected {self.nparam} parameters")
        _check(load().bemfft_net_set_params(self.handle, params.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "bemfft_net_set_params")

    def input(self, plan, bc, known, scale, x, stream=None):
        import torch

        n = plan.ncomp * plan.m
        _check(load().bemfft_net_input(self.handle, plan.handle, _u8(bc, n, "bc") if bc is not None else None,
                                       _f64(known, n, "known"), float(scale),
                                       _ptr(x, 6 * self.V, torch.float32, "x"), _stream_ptr(stream)),
               "bemfft_net_input")
        return x

    def forward(self, x, y, stream=None):
        import torch

        _check(load().bemfft_net_forward(self.handle, _ptr(x, 6 * self.V, torch.float32, "x"),
                                         _ptr(y, self.V, torch.float32, "y"), _stream_ptr(stream)),
               "bemfft_net_forward")
        return y

    def infer(self, x, y, stream=None):
        import torch

        _check(load().bemfft_net_infer(self.handle, _ptr(x, 6 * self.V, torch.float32, "x"),
                                       _ptr(y, self.V, torch.float32, "y"), _stream_ptr(stream)),
               "bemfft_net_infer")
        return y

    def gradients(self, x, vox, tgt, wt, stream=None):
        loss = ctypes.c_double()
        g = np.zeros(self.nparam, dtype=np.float32)
        nt = self._targets(x, vox, tgt, wt)
        _check(load().bemfft_net_gradients(self.handle, _ptr(x), nt, _ptr(vox), _ptr(tgt), _ptr(wt),
                                           ctypes.byref(loss), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                           _stream_ptr(stream)), "bemfft_net_gradients")
        return loss.value, g

    def train_step(self, x, vox, tgt, wt, lr, stream=None):
        loss = ctypes.c_double()
        nt = self._targets(x, vox, tgt, wt)
        _check(load().bemfft_net_train_step(self.handle, _ptr(x), nt, _ptr(vox), _ptr(tgt), _ptr(wt),
                                            float(lr), ctypes.byref(loss), _stream_ptr(stream)),
               "bemfft_net_train_step")
        return loss.value

    def guess(self, plan, bc, known, xbuf, x0, stream=None):
        import torch

        n = plan.ncomp * plan.m
        _check(load().bemfft_net_guess(self.handle, plan.handle, _u8(bc, n, "bc") if bc is not None else None,
                                       _f64(known, n, "known"), _ptr(xbuf, 6 * self.V, torch.float32, "xbuf"),
                                       _f64(x0, n, "x0"), _stream_ptr(stream)), "bemfft_net_guess")
        return x0

    def close(self):
        if self.handle is not None and self.handle.value:
            load().bemfft_net_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
