"""Python binding of libkv_hip.so (the C ABI in include/kv.h).

Argument marshalling only: every computation runs in the library's HIP
kernels on the GPU.  Vectors are torch float64 CUDA (ROCm) tensors in the
packed [u | v | w | T] layout; the library enqueues its work on the torch
stream that is current when the Context is created.  There is no CPU
fallback: without the built library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkv_hip.so")

KV_OK, KV_EINVAL, KV_ENOMEM, KV_EDEVICE, KV_ENOCONV, KV_ENONFINITE, KV_ESTATE = range(7)
KV_PROJECT, KV_MIXED = 1, 2
KV_PC_NONE, KV_PC_STOKES = 0, 1
KV_WS_PROJECT_MIXED, KV_WS_APPLY_PRECONDITIONER, KV_WS_NEWTON, KV_WS_ARNOLDI, KV_WS_TIME_STEPS = 1, 2, 3, 4, 5
KV_SYM_REF_EVEN, KV_SYM_REF_ODD, KV_SYM_ROT_EVEN, KV_SYM_ROT_ODD = 1 << 4, 1 << 5, 1 << 6, 1 << 7
KV_ST_NONE, KV_ST_CAYLEY = 0, 1


def sym_flags(cls):
    """KV_SYM_* bits of a symmetry class (e_ref, e_rot), each +1 (kept),
    -1 (broken) or 0 (free); None is the unrestricted space."""
    if cls is None:
        return 0
    e_ref, e_rot = cls
    bits = {1: KV_SYM_REF_EVEN, -1: KV_SYM_REF_ODD, 0: 0}[e_ref]
    return bits | {1: KV_SYM_ROT_EVEN, -1: KV_SYM_ROT_ODD, 0: 0}[e_rot]
STATUS_NAMES = {0: "KV_OK", 1: "KV_EINVAL", 2: "KV_ENOMEM", 3: "KV_EDEVICE", 4: "KV_ENOCONV",
                5: "KV_ENONFINITE", 6: "KV_ESTATE"}

# every extern "C" symbol declared in include/kv.h
ABI_SYMBOLS = ("kv_create", "kv_destroy", "kv_layout", "kv_workspace_size", "kv_set_workspace",
               "kv_set_base_flow", "kv_residual",
               "kv_apply_jacobian", "kv_project", "kv_project_mixed_static", "kv_dot", "kv_axpby", "kv_symmetry_measures",
               "kv_symmetry_project", "kv_hessenberg_eigenvalues", "kv_set_gmres_restart", "kv_set_bicgstab_stall",
               "kv_set_gmres_deflation", "kv_set_spectral_transform", "kv_set_solver_projection",
               "kv_newton_correction", "kv_set_preconditioner", "kv_apply_preconditioner",
               "kv_arnoldi_leading_eigs", "kv_time_steps", "kv_cells_from_state",
               "kv_state_from_cells", "kv_state_add_cell_increment", "kv_timing", "kv_last_error")


class KVError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("xf", ctypes.POINTER(ctypes.c_double)), ("yf", ctypes.POINTER(ctypes.c_double)),
                ("zf", ctypes.POINTER(ctypes.c_double)), ("Gr", ctypes.c_double), ("Pr", ctypes.c_double)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("matvecs", ctypes.c_int), ("cycles", ctypes.c_int), ("used_gmres", ctypes.c_int),
                ("relres", ctypes.c_double), ("precond", ctypes.c_int)]


class _ArnoldiParams(ctypes.Structure):
    _fields_ = [("krylov_dim", ctypes.c_int), ("n_eigs", ctypes.c_int), ("max_matvec", ctypes.c_int),
                ("max_restarts", ctypes.c_int), ("cheb_degree_max", ctypes.c_int),
                ("tol", ctypes.c_double), ("v0", ctypes.c_void_p), ("flags", ctypes.c_uint),
                ("keep", ctypes.c_int)]


class _EigInfo(ctypes.Structure):
    _fields_ = [("n_out", ctypes.c_int), ("matvecs", ctypes.c_int), ("restarts", ctypes.c_int),
                ("converged", ctypes.c_int), ("relaxed_qr", ctypes.c_int), ("inner_matvecs", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2210_08816_amd.build")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.c_double
    PD = ctypes.POINTER(ctypes.c_double)
    lib.kv_create.argtypes = [ctypes.POINTER(_Params), P, ctypes.POINTER(P)]
    lib.kv_destroy.argtypes = [P]
    lib.kv_layout.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.kv_workspace_size.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    lib.kv_set_workspace.argtypes = [P, P, ctypes.c_size_t]
    lib.kv_set_base_flow.argtypes = [P, P]
    lib.kv_residual.argtypes = [P, P, PD]
    lib.kv_apply_jacobian.argtypes = [P, P, P, ctypes.c_uint]
    lib.kv_project.argtypes = [P, P, ctypes.c_uint, PD, ctypes.POINTER(ctypes.c_int)]
    lib.kv_project_mixed_static.argtypes = [P, P, PD, ctypes.POINTER(ctypes.c_int)]
    lib.kv_dot.argtypes = [P, P, P, PD]
    lib.kv_axpby.argtypes = [P, D, P, D, P]
    lib.kv_symmetry_measures.argtypes = [P, P, PD]
    lib.kv_symmetry_project.argtypes = [P, P, P, ctypes.c_uint]
    lib.kv_hessenberg_eigenvalues.argtypes = [P, PD, ctypes.c_int, PD, PD]
    lib.kv_newton_correction.argtypes = [P, P, D, ctypes.c_int, ctypes.c_uint, P, P, ctypes.POINTER(_SolveInfo)]
    lib.kv_set_preconditioner.argtypes = [P, ctypes.c_int, D]
    lib.kv_set_gmres_restart.argtypes = [P, ctypes.c_int]
    lib.kv_set_bicgstab_stall.argtypes = [P, ctypes.c_int]
    lib.kv_set_gmres_deflation.argtypes = [P, ctypes.c_int]
    lib.kv_apply_preconditioner.argtypes = [P, P, P]
    lib.kv_arnoldi_leading_eigs.argtypes = [P, ctypes.POINTER(_ArnoldiParams), PD, PD, PD, P,
                                            ctypes.POINTER(_EigInfo)]
    lib.kv_time_steps.argtypes = [P, D, ctypes.c_int, ctypes.c_int, P, P]
    lib.kv_cells_from_state.argtypes = [P, P, ctypes.c_int, PD, PD, P]
    lib.kv_state_from_cells.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, PD, PD, PD, PD, PD, P]
    lib.kv_state_add_cell_increment.argtypes = [P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, PD, PD, PD,
                                                PD, P]
    lib.kv_timing.argtypes = [P, ctypes.c_int, PD, ctypes.POINTER(ctypes.c_int)]
    lib.kv_last_error.argtypes = [P]
    lib.kv_last_error.restype = ctypes.c_char_p
    for name in ABI_SYMBOLS:
        if name != "kv_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _fptr(t, n=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (ROCm) torch tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("expected a contiguous float32 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _host4(v):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(4))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dptr(t, n=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (ROCm) torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One grid, one base flow, one HIP stream (the current torch stream)."""

    def __init__(self, xf, yf, zf, Gr: float, Pr: float, stream=None):
        import torch
        self._lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the Krylov-vector library runs on gfx950 only")
        self._faces = [np.ascontiguousarray(np.asarray(f, dtype=np.float64)) for f in (xf, yf, zf)]
        self.nx, self.ny, self.nz = (len(f) - 1 for f in self._faces)
        p = _Params(self.nx, self.ny, self.nz,
                    *(f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for f in self._faces),
                    float(Gr), float(Pr))
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._ws = None           # torch-owned workspace (kv_set_workspace)
        self._ws_bytes = 0
        h = ctypes.c_void_p()
        rc = self._lib.kv_create(ctypes.byref(p), ctypes.c_void_p(s.cuda_stream), ctypes.byref(h))
        if rc != KV_OK:
            raise KVError(rc, "kv_create failed")
        self._h = h
        n = ctypes.c_int64()
        off = (ctypes.c_int64 * 5)()
        self._check(self._lib.kv_layout(self._h, ctypes.byref(n), off))
        self.n = int(n.value)
        self.offsets = [int(o) for o in off]

    def _check(self, rc):
        if rc != KV_OK:
            raise KVError(rc, self._lib.kv_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            self._lib.kv_destroy(self._h)
            self._h = None
        self._ws = None

    # ---- workspace: torch allocates, the library carves its scratch from it ------------
    def workspace_size(self, op, krylov_dim=0, n_eigs=0):
        """Bytes of workspace op (KV_WS_*) needs."""
        b = ctypes.c_size_t()
        rc = self._lib.kv_workspace_size(self._h, int(op), int(krylov_dim), int(n_eigs), ctypes.byref(b))
        if rc != KV_OK:
            raise KVError(rc, f"kv_workspace_size(op={op}, krylov_dim={krylov_dim}, n_eigs={n_eigs})")
        return int(b.value)

    def set_workspace(self, buf):
        """Hand the library a caller-owned float64 CUDA tensor as its
        workspace (kept referenced here while it is set)."""
        import torch
        if not isinstance(buf, torch.Tensor) or not buf.is_cuda or not buf.is_contiguous():
            raise TypeError("expected a contiguous CUDA tensor")
        nbytes = buf.numel() * buf.element_size()
        self._check(self._lib.kv_set_workspace(self._h, ctypes.c_void_p(buf.data_ptr()), nbytes))
        self._ws, self._ws_bytes = buf, nbytes

    def _ensure_workspace(self, op, krylov_dim=0, n_eigs=0):
        import torch
        need = self.workspace_size(op, krylov_dim, n_eigs)
        if self._ws is not None and self._ws_bytes >= need:
            return
        # work queued on the context's stream may still use the old buffer
        self.stream.synchronize()
        self._check(self._lib.kv_set_workspace(self._h, None, 0))
        self._ws = None
        self.set_workspace(torch.empty((need + 7) // 8, dtype=torch.float64, device=self.device))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- the C-ABI calls -----------------------------------------------------------
    def set_base_flow(self, X):
        self._check(self._lib.kv_set_base_flow(self._h, _dptr(X, self.n)))

    def residual(self, F):
        norm = ctypes.c_double()
        self._check(self._lib.kv_residual(self._h, _dptr(F, self.n), ctypes.byref(norm)))
        return norm.value

    def apply_jacobian(self, x, y, project=True, mixed=False):
        flags = (KV_PROJECT if project else 0) | (KV_MIXED if mixed else 0)
        if mixed and project:
            self._ensure_workspace(KV_WS_PROJECT_MIXED)
        self._check(self._lib.kv_apply_jacobian(self._h, _dptr(x, self.n), _dptr(y, self.n), flags))

    def project(self, y, mixed=False):
        dm = ctypes.c_double()
        sw = ctypes.c_int()
        flags = KV_PROJECT | (KV_MIXED if mixed else 0)
        if mixed:
            self._ensure_workspace(KV_WS_PROJECT_MIXED)
        self._check(self._lib.kv_project(self._h, _dptr(y, self.n), flags, ctypes.byref(dm),
                                         ctypes.byref(sw)))
        return dm.value, sw.value

    def dot(self, a, b):
        out = ctypes.c_double()
        self._check(self._lib.kv_dot(self._h, _dptr(a, self.n), _dptr(b, self.n), ctypes.byref(out)))
        return out.value

    def axpby(self, a, x, b, y):
        """y <- a x + b y."""
        self._check(self._lib.kv_axpby(self._h, float(a), _dptr(x, self.n), float(b), _dptr(y, self.n)))

    def timing(self, enable: bool):
        """Start (True) or stop (False) phase timing; returns the sums since the
        last start: ms per phase (stencil, divergence, FD transforms,
        correction) and (stencil calls, projections)."""
        ms = (ctypes.c_double * 4)()
        calls = (ctypes.c_int * 2)()
        self._check(self._lib.kv_timing(self._h, 1 if enable else 0, ms, calls))
        return list(ms), (calls[0], calls[1])

    def symmetry_measures(self, X):
        out = (ctypes.c_double * 3)()
        self._check(self._lib.kv_symmetry_measures(self._h, _dptr(X, self.n), out))
        return tuple(out)

    def symmetry_project(self, x, y=None, cls=(1, 1)):
        """y = projection of x onto the symmetry class cls = (e_ref, e_rot)
        (see sym_flags); in place when y is None."""
        y = x if y is None else y
        self._check(self._lib.kv_symmetry_project(self._h, _dptr(x, self.n), _dptr(y, self.n), sym_flags(cls)))
        return y

    def hessenberg_eigenvalues(self, H, check=True):
        """Eigenvalues of the upper Hessenberg part of the host matrix H
        (m x m) by the library's GPU QR, in deflation order."""
        H = np.ascontiguousarray(H, dtype=np.float64)
        m = H.shape[0]
        wr = (ctypes.c_double * m)()
        wi = (ctypes.c_double * m)()
        rc = self._lib.kv_hessenberg_eigenvalues(self._h, H.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), m,
                                                 wr, wi)
        if check:
            self._check(rc)
        return np.array([complex(wr[i], wi[i]) for i in range(m)]), rc

    def newton_correction(self, F, delta, tol=1e-8, max_matvec=10000, delta0=None, check=True, sym=None):
        """sym: None, or a symmetry class (e_ref, e_rot) to solve in (see sym_flags)."""
        info = _SolveInfo()
        self._ensure_workspace(KV_WS_NEWTON)
        d0 = _dptr(delta0, self.n) if delta0 is not None else None
        rc = self._lib.kv_newton_correction(self._h, _dptr(F, self.n), float(tol), int(max_matvec), sym_flags(sym), d0,
                                            _dptr(delta, self.n), ctypes.byref(info))
        if check and rc != KV_ENOCONV:
            self._check(rc)
        return dict(status=rc, matvecs=info.matvecs, cycles=info.cycles, used_gmres=info.used_gmres,
                    relres=info.relres, precond=info.precond)

    def set_preconditioner(self, stokes=True, sigma=0.0):
        """Stokes/heat right preconditioner for newton_correction (or none)."""
        self._check(self._lib.kv_set_preconditioner(self._h, KV_PC_STOKES if stokes else KV_PC_NONE,
                                                    float(sigma)))

    def set_gmres_restart(self, m):
        """Restart length of the GMRES continuation of newton_correction."""
        self._check(self._lib.kv_set_gmres_restart(self._h, int(m)))

    def set_gmres_deflation(self, k):
        """Harmonic Ritz vectors kept across GMRES restarts (GMRES-DR; 0: plain)."""
        self._check(self._lib.kv_set_gmres_deflation(self._h, int(k)))

    def set_spectral_transform(self, kind, pole=0.0, zero=-1.0, inner_tol=1e-10, inner_max_matvec=20000):
        """Cayley transform (A - pole)^-1 (A - zero) for the thick-restarted
        Arnoldi (kind KV_ST_CAYLEY; KV_ST_NONE switches it off).  The inner
        solves are preconditioned GMRES with the context's restart length and
        preconditioner."""
        self._check(self._lib.kv_set_spectral_transform(self._h, int(kind), ctypes.c_double(pole),
                                                        ctypes.c_double(zero), ctypes.c_double(inner_tol),
                                                        int(inner_max_matvec)))

    def set_solver_projection(self, mixed):
        """The projection inside newton_correction and arnoldi_leading_eigs:
        the mixed form (True) or FP64 (False, the default)."""
        self._check(self._lib.kv_set_solver_projection(self._h, KV_MIXED if mixed else 0))

    def set_bicgstab_stall(self, cycles):
        """Cycles without a 10% residual drop after which the BiCGstab(2) part
        of newton_correction hands over to GMRES (0: GMRES from the start)."""
        self._check(self._lib.kv_set_bicgstab_stall(self._h, int(cycles)))

    def apply_preconditioner(self, x, y):
        self._ensure_workspace(KV_WS_APPLY_PRECONDITIONER)
        self._check(self._lib.kv_apply_preconditioner(self._h, _dptr(x, self.n), _dptr(y, self.n)))

    def time_steps(self, X, Xprev, dt, nsteps, start=True):
        """nsteps semi-implicit time steps of Eqs. 1-6 (SBDF2; the first at
        order 1 when start), X and Xprev updated in place (kv_time_steps)."""
        self._ensure_workspace(KV_WS_TIME_STEPS)
        self._check(self._lib.kv_time_steps(self._h, float(dt), int(nsteps), 1 if start else 0,
                                            _dptr(X, self.n), _dptr(Xprev, self.n)))

    def cells_from_state(self, X, factor, shift, scale, out):
        """Normalized cell-centred (u, v, w, theta) of X on the grid coarsened
        by factor, into out (float32 CUDA, 4 * ncells)."""
        f = int(factor)
        fits = f > 0 and self.nx % f == 0 and self.ny % f == 0 and self.nz % f == 0
        nc = (self.nx // f) * (self.ny // f) * (self.nz // f) if fits else None
        sh, psh = _host4(shift)
        sc, psc = _host4(scale)
        # a factor that does not divide the grid is left to the library to reject
        optr = _fptr(out, 4 * nc if fits else None)
        self._check(self._lib.kv_cells_from_state(self._h, _dptr(X, self.n), f, psh, psc, optr))

    def state_from_cells(self, cells, centres, shift, scale, X):
        """Packed state X from network fields cells (float32 CUDA,
        4 * rz * ry * rx) at the cell centres (xc, yc, zc) (host arrays)."""
        cen = [np.ascontiguousarray(np.asarray(c, dtype=np.float64)) for c in centres]
        rx, ry, rz = (len(c) for c in cen)
        sh, psh = _host4(shift)
        sc, psc = _host4(scale)
        pc = [c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for c in cen]
        self._check(self._lib.kv_state_from_cells(self._h, _fptr(cells, 4 * rx * ry * rz), rx, ry, rz, *pc,
                                                  psh, psc, _dptr(X, self.n)))

    def state_add_cell_increment(self, cells, cells_ref, centres, scale, X):
        """X += S(cells) - S(cells_ref) (S: the interpolation of state_from_cells)."""
        cen = [np.ascontiguousarray(np.asarray(c, dtype=np.float64)) for c in centres]
        rx, ry, rz = (len(c) for c in cen)
        sc, psc = _host4(scale)
        pc = [c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for c in cen]
        nc = 4 * rx * ry * rz
        self._check(self._lib.kv_state_add_cell_increment(self._h, _fptr(cells, nc), _fptr(cells_ref, nc), rx, ry,
                                                          rz, *pc, psc, _dptr(X, self.n)))

    def arnoldi_leading_eigs(self, v0, krylov_dim, n_eigs, tol=1e-8, max_matvec=100000,
                             max_restarts=1000, cheb_degree_max=200, sym=None, evecs=None, check=True, keep=0):
        """sym: a symmetry class (e_ref, e_rot) to restrict the Krylov space
        to (see sym_flags), or None.  evecs: None, or a float64 CUDA tensor of
        (n_eigs + 1) * n values that receives the eigenvectors, one per row
        (a conjugate pair as the real and imaginary part of the +Im member's)."""
        self._ensure_workspace(KV_WS_ARNOLDI, krylov_dim, n_eigs)
        p = _ArnoldiParams(int(krylov_dim), int(n_eigs), int(max_matvec), int(max_restarts),
                           int(cheb_degree_max), float(tol), _dptr(v0, self.n).value, sym_flags(sym),
                           int(keep))
        re = (ctypes.c_double * (n_eigs + 1))()
        im = (ctypes.c_double * (n_eigs + 1))()
        res = (ctypes.c_double * (n_eigs + 1))()
        info = _EigInfo()
        ev = _dptr(evecs, (n_eigs + 1) * self.n) if evecs is not None else None
        rc = self._lib.kv_arnoldi_leading_eigs(self._h, ctypes.byref(p), re, im, res, ev, ctypes.byref(info))
        if check and rc != KV_ENOCONV:
            self._check(rc)
        k = info.n_out
        vals = np.array([complex(re[i], im[i]) for i in range(k)])
        return vals, np.array(res[:k]), dict(status=rc, n_out=k, matvecs=info.matvecs,
                                              restarts=info.restarts, converged=bool(info.converged),
                                              relaxed_qr=info.relaxed_qr, inner_matvecs=info.inner_matvecs)
