"""MI355X Sakurai-Sugiura complex-band-structure library: Python binding.

A thin ctypes layer over ``libcbs.so`` (the C ABI in ``include/cbs.h``).  It
only marshals arguments: every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory (tensors passed by ``data_ptr()``)
and streams (``torch.cuda.current_stream()``).  If the library is not built,
every call raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcbs.so")

CBS_OK, CBS_EINVAL, CBS_ENOMEM, CBS_EHIP, CBS_ENOCONV, CBS_EBREAKDOWN, CBS_ERANK, CBS_ETOOMANY, \
    CBS_ENONFINITE, CBS_EEIG = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
CBS_C128, CBS_C64 = 0, 1
CBS_FP64, CBS_MIXED = 0, 1
CBS_RR, CBS_HANKEL = 0, 1

# every function the header declares
EXPORTS = [
    "cbs_strerror", "cbs_last_error", "cbs_system_create", "cbs_system_destroy",
    "cbs_system_set_vloc", "cbs_system_npoints", "cbs_system_solve_id", "cbs_system_tiling",
    "cbs_params_default", "cbs_apply", "cbs_apply_noalloc",
    "cbs_apply_parts", "cbs_bicg", "cbs_bicg_history", "cbs_solve", "cbs_solve_batched", "cbs_lambda_to_k",
    "cbs_bands", "cbs_connect_branches",
    "cbs_grad_vloc",
]


class CbsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("fd_order", ctypes.c_int32), ("h", ctypes.c_double)]


class Proj(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_proj", ctypes.c_int32),
                ("ball_off", ctypes.c_void_p), ("ball_idx", ctypes.c_void_p),
                ("ball_w", ctypes.c_void_p), ("ball_val", ctypes.c_void_p),
                ("coeff", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("lambda_min", ctypes.c_double), ("n_q", ctypes.c_int32), ("n_rhs", ctypes.c_int32),
                ("n_mom", ctypes.c_int32), ("delta", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("extraction", ctypes.c_int32), ("half_stop", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("conj_nodes", ctypes.c_int32), ("block", ctypes.c_int32),
                ("lo_window", ctypes.c_int32)]

    def __repr__(self):
        return "Params(" + ", ".join(f"{n}={getattr(self, n)}" for n, _ in self._fields_) + ")"


class Info(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("n_eigs", ctypes.c_int32), ("iters_max", ctypes.c_int32),
                ("refine_steps", ctypes.c_int32), ("iters_mean", ctypes.c_double),
                ("max_solve_resid", ctypes.c_double), ("max_eig_resid", ctypes.c_double),
                ("sigma_first", ctypes.c_double), ("sigma_ratio", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_moments_ms", ctypes.c_double),
                ("t_extract_ms", ctypes.c_double), ("matvecs", ctypes.c_int64),
                ("stencil_launches", ctypes.c_int64), ("stencil_ms", ctypes.c_double),
                ("stencil_bytes", ctypes.c_double), ("stencil_lo_launches", ctypes.c_int64),
                ("stencil_lo_ms", ctypes.c_double), ("stencil_lo_bytes", ctypes.c_double),
                ("nodes_solved", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("status", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_LIB = None


def lib():
    """Load libcbs.so (raises if it is not built: the HIP path is the only path)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # PyTorch ships its own HIP runtime with the same soname (libamdhip64.so.7).  Loaded
        # first, it is the copy the library binds to, so tensors, streams and the library's
        # kernels share one runtime; loaded after the library, a second runtime would come
        # in beside the one the library found and the library would see no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.cbs_strerror.restype = ctypes.c_char_p
        L.cbs_strerror.argtypes = [i32]
        L.cbs_last_error.restype = ctypes.c_char_p
        L.cbs_last_error.argtypes = []
        L.cbs_system_create.restype = i32
        L.cbs_system_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(Grid), vp,
                                        ctypes.POINTER(Proj)]
        L.cbs_system_destroy.restype = None
        L.cbs_system_destroy.argtypes = [vp]
        L.cbs_system_set_vloc.restype = i32
        L.cbs_system_set_vloc.argtypes = [vp, vp]
        L.cbs_system_npoints.restype = i64
        L.cbs_system_npoints.argtypes = [vp]
        L.cbs_system_solve_id.restype = i64
        L.cbs_system_solve_id.argtypes = [vp]
        L.cbs_system_tiling.restype = ctypes.c_char_p
        L.cbs_system_tiling.argtypes = [vp, vp]
        L.cbs_params_default.restype = None
        L.cbs_params_default.argtypes = [ctypes.POINTER(Params)]
        L.cbs_apply.restype = i32
        L.cbs_apply.argtypes = [vp, dbl, i32, vp, i32, vp, vp, vp]
        L.cbs_apply_noalloc.restype = i32
        L.cbs_apply_noalloc.argtypes = [vp, dbl, i32, vp, i32, vp, vp, vp]
        L.cbs_apply_parts.restype = i32
        L.cbs_apply_parts.argtypes = [vp, dbl, i32, vp, vp, vp, vp, vp, vp]
        L.cbs_bicg.restype = i32
        L.cbs_bicg.argtypes = [vp, dbl, i32, vp, i32, vp, ctypes.POINTER(Params), vp, vp, vp, vp,
                               ctypes.POINTER(Info), vp]
        L.cbs_bicg_history.restype = i32
        L.cbs_bicg_history.argtypes = [vp, dbl, i32, vp, i32, vp, ctypes.POINTER(Params), i32, i32, vp, vp, vp,
                                       vp, vp, ctypes.POINTER(Info), vp]
        L.cbs_solve.restype = i32
        L.cbs_solve.argtypes = [vp, dbl, ctypes.POINTER(Params), vp, i32, vp, vp, vp,
                                ctypes.POINTER(i32), ctypes.POINTER(Info), vp]
        L.cbs_solve_batched.restype = i32
        L.cbs_solve_batched.argtypes = [i32, vp, i32, vp, ctypes.POINTER(Params), vp, i32, vp, vp,
                                        vp, vp]
        L.cbs_lambda_to_k.restype = i32
        L.cbs_lambda_to_k.argtypes = [i32, vp, dbl, vp]
        L.cbs_connect_branches.restype = i32
        L.cbs_connect_branches.argtypes = [i32, vp, vp, vp, dbl, dbl, vp, ctypes.POINTER(i32)]
        L.cbs_bands.restype = i32
        L.cbs_bands.argtypes = [vp, i32, vp, i32, dbl, i32, vp, vp, vp, vp, vp]
        L.cbs_grad_vloc.restype = i32
        L.cbs_grad_vloc.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        _LIB = L
    return _LIB


def _check(rc: int, what: str, ok=(CBS_OK,)):
    if rc not in ok:
        L = lib()
        raise CbsError(rc, f"{what}: {L.cbs_strerror(rc).decode()}: {L.cbs_last_error().decode()}")
    return rc


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def default_params(**kw) -> Params:
    p = Params()
    lib().cbs_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _host_c128(z) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(z, dtype=np.complex128))


class System:
    """One periodic cell on one device (wraps cbs_system)."""

    def __init__(self, nx, ny, nz, h, fd_order, v_loc, proj=None, device: int = 0):
        L = lib()
        self._keep = []
        g = Grid(nx, ny, nz, fd_order, h)
        v = np.ascontiguousarray(np.asarray(v_loc, dtype=np.float64))
        if v.size != nx * ny * nz:
            raise ValueError("v_loc has the wrong length")
        pr = None
        if proj is not None and proj.n_atoms > 0:
            arrs = [np.ascontiguousarray(proj.ball_off, dtype=np.int64),
                    np.ascontiguousarray(proj.ball_idx, dtype=np.int32),
                    np.ascontiguousarray(proj.ball_w, dtype=np.int8),
                    np.ascontiguousarray(proj.ball_val, dtype=np.float64),
                    np.ascontiguousarray(proj.coeff, dtype=np.float64)]
            self._keep = arrs
            pr = Proj(proj.n_atoms, proj.n_proj, *[a.ctypes.data for a in arrs])
        h_ = ctypes.c_void_p()
        _check(L.cbs_system_create(ctypes.byref(h_), device, ctypes.byref(g), v.ctypes.data,
                                   ctypes.byref(pr) if pr is not None else None),
               "cbs_system_create")
        self.handle = h_
        self.n = nx * ny * nz
        self.shape = (nx, ny, nz)
        self.cell_length = nz * h   # a in lambda = exp(i k a)
        self.device = device
        self._keep = []

    @classmethod
    def from_workload(cls, sys, device: int = 0):
        return cls(sys.nx, sys.ny, sys.nz, sys.h, sys.fd_order, sys.v_loc, sys.proj, device)

    def close(self):
        if getattr(self, "handle", None):
            lib().cbs_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve_id(self) -> int:
        """Counter of the solves whose eigenpairs the system stored (cbs_system_solve_id)."""
        return int(lib().cbs_system_solve_id(self.handle))

    def tiling(self):
        """(tile_y complex128, tile_y complex64, autotuner log)."""
        ty = np.zeros(2, dtype=np.int32)
        log = lib().cbs_system_tiling(self.handle, ty.ctypes.data).decode()
        return int(ty[0]), int(ty[1]), log

    def set_vloc(self, v_loc):
        v = np.ascontiguousarray(np.asarray(v_loc, dtype=np.float64)).reshape(-1)
        if v.size != self.n:
            raise ValueError(f"v_loc has {v.size} values, the cell has {self.n} points")
        _check(lib().cbs_system_set_vloc(self.handle, v.ctypes.data), "cbs_system_set_vloc")

    # ---- operator -----------------------------------------------------------
    def apply(self, E: float, z, x, y=None, stream=None):
        """y_v = P(z_v) x_v; x a [n_vec, N] complex128/complex64 CUDA tensor."""
        import torch
        x = x.contiguous()
        if y is None:
            y = torch.empty_like(x)
        zz = _host_c128(z)
        nv = x.shape[0]
        if zz.size != nv:
            raise ValueError("one z per vector")
        dt = {torch.complex128: CBS_C128, torch.complex64: CBS_C64}[x.dtype]
        _check(lib().cbs_apply(self.handle, float(E), nv, zz.ctypes.data, dt, _ptr(x), _ptr(y),
                               _stream(stream)), "cbs_apply")
        return y

    def apply_noalloc(self, E: float, z, x, y, stream=None):
        """y_v = P(z_v) x_v into the caller's y without any device allocation
        (cbs_apply_noalloc: staging in the library's fixed scratch array)."""
        import torch
        if not (x.is_contiguous() and y.is_contiguous()) or x.shape != y.shape or x.dtype != y.dtype:
            raise ValueError("x and y: contiguous tensors of one shape and dtype")
        zz = _host_c128(z)
        nv = x.shape[0]
        if zz.size != nv:
            raise ValueError("one z per vector")
        dt = {torch.complex128: CBS_C128, torch.complex64: CBS_C64}[x.dtype]
        _check(lib().cbs_apply_noalloc(self.handle, float(E), nv, zz.ctypes.data, dt, _ptr(x), _ptr(y),
                                       _stream(stream)), "cbs_apply_noalloc")
        return y

    def apply_parts(self, E: float, c0, cp, cm, x, y=None, stream=None):
        import torch
        x = x.contiguous()
        if y is None:
            y = torch.empty_like(x)
        a, b, c = _host_c128(c0), _host_c128(cp), _host_c128(cm)
        _check(lib().cbs_apply_parts(self.handle, float(E), x.shape[0], a.ctypes.data,
                                     b.ctypes.data, c.ctypes.data, _ptr(x), _ptr(y),
                                     _stream(stream)), "cbs_apply_parts")
        return y

    # ---- step 1 ------------------------------------------------------------
    def bicg(self, E: float, z, V, params: Optional[Params] = None, stream=None, history=None):
        """Solve P(z_j) Y = V and P(z_j)^H Yt = V for every node; returns (Y, Yt, iters, relres, info, rc).
        history=(stride, max_rows): also returns the residual histories (cbs_bicg_history) as a
        seventh item, shape [max_rows][n_z][L][2] (NaN past a run's end)."""
        import torch
        params = params or default_params()
        V = V.contiguous()
        L_, N = V.shape
        zz = _host_c128(z)
        nz = zz.size
        Y = torch.empty((nz, L_, N), dtype=torch.complex128, device=V.device)
        Yt = torch.empty_like(Y)
        iters = np.zeros(nz * L_, dtype=np.int32)
        relres = np.zeros(2 * nz * L_, dtype=np.float64)
        info = Info()
        if history is None:
            rc = lib().cbs_bicg(self.handle, float(E), nz, zz.ctypes.data, L_, _ptr(V),
                                ctypes.byref(params), _ptr(Y), _ptr(Yt), iters.ctypes.data,
                                relres.ctypes.data, ctypes.byref(info), _stream(stream))
            _check(rc, "cbs_bicg", ok=(CBS_OK, CBS_ENOCONV))
            return Y, Yt, iters.reshape(nz, L_), relres.reshape(nz, L_, 2), info, rc
        stride, rows = int(history[0]), int(history[1])
        hist = np.zeros((rows, nz, L_, 2), dtype=np.float64)
        rc = lib().cbs_bicg_history(self.handle, float(E), nz, zz.ctypes.data, L_, _ptr(V),
                                    ctypes.byref(params), stride, rows, hist.ctypes.data, _ptr(Y), _ptr(Yt),
                                    iters.ctypes.data, relres.ctypes.data, ctypes.byref(info), _stream(stream))
        _check(rc, "cbs_bicg_history", ok=(CBS_OK, CBS_ENOCONV))
        return Y, Yt, iters.reshape(nz, L_), relres.reshape(nz, L_, 2), info, rc, hist

    # ---- the whole method ----------------------------------------------------
    def solve(self, E: float, V, params: Optional[Params] = None, max_eigs: int = 512,
              want_vectors: bool = True, stream=None):
        """Eigenpairs inside the annulus; returns (lam [m] complex128 numpy, vecs [m, N] tensor|None,
        resid [m], info, rc)."""
        import torch
        params = params or default_params()
        V = V.contiguous()
        lam = np.zeros(2 * max_eigs, dtype=np.float64)
        res = np.zeros(max_eigs, dtype=np.float64)
        vecs = torch.empty((max_eigs, self.n), dtype=torch.complex128, device=V.device) \
            if want_vectors else None
        n = ctypes.c_int32(0)
        info = Info()
        rc = lib().cbs_solve(self.handle, float(E), ctypes.byref(params), _ptr(V), max_eigs,
                             lam.ctypes.data, res.ctypes.data,
                             _ptr(vecs) if vecs is not None else None, ctypes.byref(n),
                             ctypes.byref(info), _stream(stream))
        _check(rc, "cbs_solve", ok=(CBS_OK, CBS_ENOCONV, CBS_ERANK))
        m = n.value
        lamc = lam[:2 * m].view(np.complex128).copy()
        return lamc, (vecs[:m] if vecs is not None else None), res[:m].copy(), info, rc

    def bands(self, k, n_bands: int, tol: float = 1e-10, max_iter: int = 400, want_vectors: bool = False,
              stream=None):
        """Lowest n_bands eigenvalues of the Hermitian H(k) at real wave numbers k (cbs_bands);
        returns (eps [n_k, n_bands], resid [n_k, n_bands], vecs [n_k, n_bands, N] | None,
        iters [n_k], rc)."""
        import torch
        kk = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1))
        nk = kk.size
        eps = np.zeros((nk, n_bands), dtype=np.float64)
        res = np.zeros((nk, n_bands), dtype=np.float64)
        it = np.zeros(nk, dtype=np.int32)
        vecs = torch.empty((nk, n_bands, self.n), dtype=torch.complex128, device=f"cuda:{self.device}") \
            if want_vectors else None
        rc = lib().cbs_bands(self.handle, nk, kk.ctypes.data, int(n_bands), float(tol), int(max_iter),
                             eps.ctypes.data, res.ctypes.data, _ptr(vecs) if vecs is not None else None,
                             it.ctypes.data, _stream(stream))
        _check(rc, "cbs_bands", ok=(CBS_OK, CBS_ENOCONV))
        return eps, res, vecs, it, rc

    def grad_vloc(self, sel: Sequence[int], stream=None):
        """d lambda_k / d V_loc for the eigenpairs sel of the last solve: [len(sel), N] complex128."""
        import torch
        s = np.ascontiguousarray(np.asarray(sel, dtype=np.int32))
        out = torch.empty((len(s), self.n), dtype=torch.complex128, device=f"cuda:{self.device}")
        _check(lib().cbs_grad_vloc(self.handle, len(s), s.ctypes.data, _ptr(out), None, None,
                                   _stream(stream)), "cbs_grad_vloc")
        return out

    def vjp_vloc(self, sel: Sequence[int], weights, stream=None):
        """sum_k Re(g_k conj(d lambda_k / d V_loc)) for host weights g: [N] float64 tensor."""
        import torch
        s = np.ascontiguousarray(np.asarray(sel, dtype=np.int32))
        w = _host_c128(weights)
        out = torch.empty(self.n, dtype=torch.float64, device=f"cuda:{self.device}")
        _check(lib().cbs_grad_vloc(self.handle, len(s), s.ctypes.data, None, w.ctypes.data, _ptr(out),
                                   _stream(stream)), "cbs_grad_vloc")
        return out


def _autograd():
    import torch

    class CbsEig(torch.autograd.Function):
        """lambda_sel(V_loc): eigenvalues of the annulus as a differentiable function of V_loc.

        forward solves (cbs_solve) with the given potential; backward calls the adjoint
        kernel (cbs_grad_vloc) with the incoming gradient as weights.  ``select`` maps the
        sorted eigenvalues (numpy) to the indices to return.  The adjoint reads the
        eigenpairs the system stored with its last solve; when another solve on the same
        system came between this forward and its backward (two forwards before one
        backward, gradcheck), backward solves again with this forward's potential and
        checks that it reproduces the same eigenvalues (the solve is deterministic).
        """

        @staticmethod
        def forward(ctx, v_loc, system, E, V, params, select):
            v = v_loc.detach().cpu().numpy().astype(np.float64).copy()
            system.set_vloc(v)
            lam, _, _, _, _ = system.solve(E, V, params, want_vectors=False)
            sel = np.asarray(select(lam), dtype=np.int32)
            ctx.system, ctx.sel, ctx.vdev = system, sel, v_loc.device
            ctx.v, ctx.E, ctx.V, ctx.params, ctx.lam = v, E, V, params, lam.copy()
            ctx.solve_id = system.solve_id()
            return torch.from_numpy(lam[sel].copy())

        @staticmethod
        def backward(ctx, grad):
            s = ctx.system
            if s.solve_id() != ctx.solve_id:
                s.set_vloc(ctx.v)
                lam, _, _, _, _ = s.solve(ctx.E, ctx.V, ctx.params, want_vectors=False)
                if lam.shape != ctx.lam.shape or not np.array_equal(lam, ctx.lam):
                    raise RuntimeError("CbsEig.backward: the repeated solve did not reproduce the "
                                       "forward's eigenvalues")
            g = grad.detach().cpu().numpy().astype(np.complex128)
            v = s.vjp_vloc(ctx.sel, g)
            return v.to(ctx.vdev), None, None, None, None, None

    return CbsEig


def cbs_eig(v_loc, system: "System", E: float, V, params: Optional[Params] = None, select=None):
    """Differentiable eigenvalues lambda(V_loc) (see CbsEig); default: all of them."""
    params = params or default_params()
    select = select or (lambda lam: np.arange(len(lam)))
    return _autograd().apply(v_loc, system, E, V, params, select)


def solve_batched(systems: List[System], energies, Vs, params: Optional[Params] = None,
                  max_eigs: int = 512, stream=None):
    """Every (system, energy) pair in one batched pass; returns (lam list-of-lists, infos, rc).
    infos[s * len(energies) + e].status is the code of pair (s, e)."""
    params = params or default_params()
    ns, ne = len(systems), len(energies)
    handles = (ctypes.c_void_p * ns)(*[s.handle for s in systems])
    vps = (ctypes.c_void_p * ns)(*[v.data_ptr() for v in Vs])
    E = np.ascontiguousarray(np.asarray(energies, dtype=np.float64))
    lam = np.zeros((ns, ne, 2 * max_eigs), dtype=np.float64)
    cnt = np.zeros(ns * ne, dtype=np.int32)
    infos = (Info * (ns * ne))()
    rc = lib().cbs_solve_batched(ns, handles, ne, E.ctypes.data, ctypes.byref(params), vps,
                                 max_eigs, lam.ctypes.data, cnt.ctypes.data, infos, _stream(stream))
    # pair-level codes come back in infos[i].status (a failed pair has no eigenvalues); the
    # call itself fails only on bad arguments, allocation or HIP errors
    _check(rc, "cbs_solve_batched", ok=(CBS_OK, CBS_ENOCONV, CBS_ERANK, CBS_EBREAKDOWN, CBS_ENONFINITE,
                                        CBS_EEIG, CBS_ETOOMANY))
    out = [[(lam[s, e, :2 * cnt[s * ne + e]].view(np.complex128).copy()
             if infos[s * ne + e].status != CBS_ETOOMANY else np.zeros(0, dtype=np.complex128))
            for e in range(ne)] for s in range(ns)]
    return out, [infos[i] for i in range(ns * ne)], rc


def lambda_to_k(lam, cell_length: float) -> np.ndarray:
    """Complex wave numbers k of Bloch factors lambda = exp(i k a) (cbs_lambda_to_k)."""
    lam = _host_c128(lam).reshape(-1)
    k = np.empty_like(lam)
    _check(lib().cbs_lambda_to_k(lam.size, lam.ctypes.data, float(cell_length), k.ctypes.data),
           "cbs_lambda_to_k")
    return k


def connect_branches(energies, ks, cell_length: float, max_jump: float):
    """Branch ids of the k of each energy (cbs_connect_branches): ks is a list of complex
    arrays, one per energy (increasing).  Returns (list of int arrays, n_branches)."""
    E = np.ascontiguousarray(np.asarray(energies, dtype=np.float64))
    counts = np.ascontiguousarray(np.array([len(k) for k in ks], dtype=np.int32))
    flat = np.ascontiguousarray(np.concatenate([_host_c128(k).reshape(-1) for k in ks])
                                if len(ks) else np.zeros(0, np.complex128))
    br = np.zeros(max(1, flat.size), dtype=np.int32)
    nb = ctypes.c_int32(0)
    _check(lib().cbs_connect_branches(E.size, E.ctypes.data, counts.ctypes.data, flat.ctypes.data,
                                      float(cell_length), float(max_jump), br.ctypes.data, ctypes.byref(nb)),
           "cbs_connect_branches")
    out, off = [], 0
    for c in counts:
        out.append(br[off:off + c].copy())
        off += c
    return out, nb.value


def cbs_sweep(system: "System", energies, V, params: Optional[Params] = None, max_eigs: int = 512,
              stream=None, max_jump: Optional[float] = None):
    """Complex band structure of one cell over increasing energies: one batched pass
    (cbs_solve_batched), k for every eigenvalue and its branch (cbs_connect_branches; max_jump
    defaults to a tenth of the zone width 2 pi / a).  Returns ([(E, lambda, k, branch)], infos, rc)."""
    lam, infos, rc = solve_batched([system], energies, [V], params, max_eigs, stream)
    ks = [lambda_to_k(l, system.cell_length) for l in lam[0]]
    jump = max_jump if max_jump is not None else 0.2 * np.pi / system.cell_length
    br, _ = connect_branches(energies, ks, system.cell_length, jump)
    out = [(float(E), l, k, b) for E, l, k, b in zip(energies, lam[0], ks, br)]
    return out, infos, rc
