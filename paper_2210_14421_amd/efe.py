"""Thin ctypes binding of libefe.so (C ABI in include/efe.h).

Argument marshalling only: every step of the Magnus propagation runs in the
library's HIP kernels.  Device arrays are torch tensors (complex128 orbital
blocks, float64 quadrature/nodal arrays); the library works on the current
torch HIP stream.  If the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libefe.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2210_14421_amd.build`")

_lib = C.CDLL(LIB_PATH)

EFE_OK, EFE_ERR_ARG, EFE_ERR_ALLOC, EFE_ERR_HIP = 0, -1, -2, -3
EFE_ERR_NOCONV, EFE_ERR_SINGULAR, EFE_ERR_NONFINITE, EFE_ERR_STATE = -4, -5, -6, -7
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f64sf": 3, "bf16x3": 4}
XC = {"none": 0, "slater": 1, "slater_pw92": 2}
OPS = {"H": 0, "x": 1, "y": 2, "z": 3}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class EfeSystem(C.Structure):
    _fields_ = [("ncell", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("degree", C.c_int32), ("natom", C.c_int32), ("R", _dp), ("Z", _dp),
                ("nuc_sigma", C.c_double), ("nenr", C.c_int32), ("enr_atom", _ip), ("enr_l", _ip),
                ("enr_m", _ip), ("enr_zeta", _dp), ("r_cut", C.c_double), ("norb", C.c_int32),
                ("occ", _dp), ("xc", C.c_int32), ("trap_omega", C.c_double), ("quad_cell", C.c_int32),
                ("quad_enr", C.c_int32), ("enr_drop_tol", C.c_double), ("cell_bounds", _dp)]


class EfeOptions(C.Structure):
    _fields_ = [("prod_dtype", C.c_int32), ("kmax", C.c_int32), ("krylov_tol", C.c_double),
                ("cg_tol", C.c_double), ("cg_maxit", C.c_int32), ("hip_stream", C.c_void_p),
                ("reorth", C.c_int32)]


REORTH = {"partial": 0, "full": 1, "partial_dot": 2}


class EfeField(C.Structure):
    _fields_ = [("kind", C.c_int32), ("direction", C.c_int32), ("ncomp", C.c_int32),
                ("A", _dp), ("w", _dp), ("phi", _dp), ("t0", C.c_double), ("s", C.c_double)]


class EfePulse(C.Structure):
    _fields_ = [("kind", C.c_int32), ("kappa", C.c_double), ("t0", C.c_double), ("s", C.c_double)]


class EfeStepStats(C.Structure):
    _fields_ = [("k_pred", C.c_int32 * 128), ("k_corr", C.c_int32 * 128), ("err_pred_max", C.c_double),
                ("err_corr_max", C.c_double), ("cg_iters", C.c_int32 * 2), ("mu", C.c_double * 3)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_plan_create = _sig("efe_plan_create", C.c_int32, [C.POINTER(EfeSystem), C.POINTER(C.c_void_p)])
_plan_free = _sig("efe_plan_free", C.c_int32, [C.c_void_p])
_plan_sizes = _sig("efe_plan_sizes", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)])
_plan_get = _sig("efe_plan_get", C.c_int32, [C.c_void_p, C.c_char_p, _dp, C.c_int64])
_plan_error = _sig("efe_plan_error", C.c_char_p, [C.c_void_p])
_setup = _sig("efe_setup", C.c_int32, [C.POINTER(EfeSystem), C.POINTER(EfeOptions), C.POINTER(C.c_void_p)])
_free = _sig("efe_free", C.c_int32, [C.c_void_p])
_dims = _sig("efe_dims", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)])
_set_options = _sig("efe_set_options", C.c_int32, [C.c_void_p, C.POINTER(EfeOptions)])
_initial_state = _sig("efe_initial_state", C.c_int32, [C.c_void_p, _ip, _dp, C.c_double, C.c_void_p])
_set_ham = _sig("efe_set_hamiltonian", C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.POINTER(EfeField)])
_apply_H = _sig("efe_apply_H", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int64])
_apply_H_noalloc = _sig("efe_apply_H_noalloc", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32])
_lanczos = _sig("lanczos_expm", C.c_int32, [C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_int32, C.c_int64,
                                            _ip, _ip, _dp])
_magnus = _sig("magnus_step", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                          C.POINTER(EfeField), _ip, C.POINTER(EfeStepStats)])
_magnus_extrap = _sig("magnus_step_extrap", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                                        C.POINTER(EfeField), _ip, C.c_int32, C.POINTER(EfeStepStats)])
EFE_STEP_KEEP_HAM = 1
_power = _sig("power_spectrum", C.c_int32, [C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_double, C.c_void_p,
                                            C.c_int64, C.c_void_p, C.c_void_p])
_spectrum = _sig("absorption_spectrum", C.c_int32, [C.c_void_p, _ip, C.c_int32, C.c_int64, C.c_double,
                                                     C.POINTER(EfePulse), C.c_double, C.c_void_p, C.c_int64,
                                                     C.c_void_p, C.c_void_p, C.c_void_p])
_magnus_graph = _sig("magnus_step_graph", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                                      C.POINTER(EfeField), C.POINTER(EfeStepStats)])
_batch_create = _sig("efe_batch_create", C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)])
_batch_free = _sig("efe_batch_free", C.c_int32, [C.c_void_p])
_batch_error = _sig("efe_batch_error", C.c_char_p, [C.c_void_p])
_batch_step = _sig("efe_batch_step", C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_double,
                                                 C.c_double, C.POINTER(C.POINTER(EfeField)),
                                                 C.POINTER(EfeStepStats)])
_adjoint = _sig("magnus_adjoint", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                               C.POINTER(EfeField), _dp, C.c_void_p, C.c_int64, _dp])
_dip_adjoint = _sig("dipole_adjoint", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, _dp, C.c_void_p, C.c_int64])
_density = _sig("density", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p])
_hartree = _sig("efe_hartree", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, _ip])
_dipole = _sig("dipole", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, _dp])
_timing_on = _sig("efe_enable_timing", C.c_int32, [C.c_void_p, C.c_int32])
_timing_get = _sig("efe_get_timing", C.c_int32, [C.c_void_p, _dp, C.POINTER(C.c_int64)])
_last_error = _sig("efe_last_error", C.c_char_p, [C.c_void_p])
_field_vjp = _sig("efe_field_vjp", C.c_int32, [C.POINTER(EfeField), C.c_int64, _dp, _dp, _dp])
_autotune = _sig("efe_autotune", C.c_int32, [C.c_void_p, C.c_char_p, C.c_int32, C.c_char_p, C.c_int32])
EFE_TUNE_FORCE = 1

EXPORTED = ["efe_plan_create", "efe_plan_free", "efe_plan_sizes", "efe_plan_get", "efe_plan_error",
            "efe_setup", "efe_free", "efe_dims", "efe_set_options", "efe_initial_state",
            "efe_set_hamiltonian", "efe_apply_H", "lanczos_expm", "magnus_step", "density",
            "efe_hartree", "dipole", "efe_enable_timing", "efe_get_timing", "efe_last_error",
            "magnus_step_graph", "efe_batch_create", "efe_batch_free", "efe_batch_error", "efe_batch_step",
            "magnus_adjoint", "dipole_adjoint", "magnus_step_extrap", "absorption_spectrum", "power_spectrum",
            "efe_field_vjp", "efe_apply_H_noalloc", "efe_autotune"]


class EfeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"efe status {status}: {msg}")
        self.status = status


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class _SystemHolder:
    """Keeps the numpy arrays referenced by an EfeSystem alive."""

    def __init__(self, spec):
        self.R = _arr(spec.R, np.float64).reshape(-1)
        self.Z = _arr(spec.Z, np.float64)
        self.ea = _arr(spec.enr_atom, np.int32)
        self.el = _arr(spec.enr_l, np.int32)
        self.em = _arr(spec.enr_m, np.int32)
        self.ez = _arr(spec.enr_zeta, np.float64)
        self.occ = _arr(spec.occ, np.float64)
        s = EfeSystem()
        for d in range(3):
            s.ncell[d] = int(spec.ncell[d])
            s.lo[d] = float(spec.lo[d])
            s.hi[d] = float(spec.hi[d])
        s.degree = int(spec.degree)
        s.natom = int(len(self.Z))
        s.R = self.R.ctypes.data_as(_dp)
        s.Z = self.Z.ctypes.data_as(_dp)
        s.nuc_sigma = float(spec.nuc_sigma)
        s.nenr = int(len(self.ez))
        s.enr_atom = self.ea.ctypes.data_as(_ip)
        s.enr_l = self.el.ctypes.data_as(_ip)
        s.enr_m = self.em.ctypes.data_as(_ip)
        s.enr_zeta = self.ez.ctypes.data_as(_dp)
        s.r_cut = float(spec.r_cut)
        s.norb = int(len(self.occ))
        s.occ = self.occ.ctypes.data_as(_dp)
        s.xc = XC[spec.xc]
        s.trap_omega = float(spec.trap_omega)
        s.quad_cell = int(spec.quad_cell)
        s.quad_enr = int(spec.quad_enr)
        s.enr_drop_tol = float(spec.enr_drop_tol)
        bounds = getattr(spec, "bounds", None)
        if bounds is not None:
            self.bounds = np.ascontiguousarray(np.concatenate([np.asarray(b, dtype=np.float64) for b in bounds]))
            s.cell_bounds = self.bounds.ctypes.data_as(_dp)
        self.sys = s


class Plan:
    """Host-only static data of the discretisation (no GPU needed)."""

    def __init__(self, spec):
        self._h = _SystemHolder(spec)
        self._p = C.c_void_p()
        st = _plan_create(C.byref(self._h.sys), C.byref(self._p))
        if st != EFE_OK:
            msg = _plan_error(self._p).decode() if self._p else ""
            _plan_free(self._p)
            self._p = None
            raise EfeError(st, msg)
        sz = (C.c_int64 * 6)()
        _plan_sizes(self._p, sz)
        (self.n_nodes, self.n_cells, self.n_quad, self.n_kept, self.n_union_rows, self.n_tcells) = list(sz)
        self.nenr = int(len(spec.enr_zeta))

    def get(self, name, count):
        out = np.empty(int(count), dtype=np.float64)
        st = _plan_get(self._p, name.encode(), out.ctypes.data_as(_dp), int(count))
        if st != EFE_OK:
            raise EfeError(st, f"plan array {name!r} of {count}")
        return out

    def __del__(self):
        if getattr(self, "_p", None):
            _plan_free(self._p)
            self._p = None


def absorption_spectrum(mu, dirs, dt, omega, tau, pulse, with_alpha=False):
    """S(omega) of Sec. 3.2 on the GPU from dipole traces.

    mu: cuda float64 tensor [ndir][nt + 1][3] (run r perturbed along dirs[r]);
    omega: cuda float64 tensor [nw]; pulse: dict(kind="kick"|"gauss", kappa, t0, s).
    Returns S (cuda [nw]) and, with with_alpha, alpha (cuda complex128 [ndir][nw])."""
    import torch
    if mu.dtype != torch.float64 or not mu.is_cuda or mu.dim() != 3 or mu.shape[2] != 3:
        raise ValueError("mu must be a cuda float64 tensor [ndir][nt + 1][3]")
    if omega.dtype != torch.float64 or not omega.is_cuda or omega.dim() != 1:
        raise ValueError("omega must be a cuda float64 tensor [nw]")
    mu, omega = mu.contiguous(), omega.contiguous()
    d = _arr(dirs, np.int32)
    if len(d) != mu.shape[0]:
        raise ValueError("one direction per trace")
    p = EfePulse()
    p.kind = {"kick": 0, "gauss": 1}[pulse["kind"]]
    p.kappa, p.t0, p.s = float(pulse["kappa"]), float(pulse.get("t0", 0.0)), float(pulse.get("s", 1.0))
    S = torch.empty(omega.shape[0], dtype=torch.float64, device=omega.device)
    alpha = torch.empty((mu.shape[0], omega.shape[0], 2), dtype=torch.float64, device=omega.device) if with_alpha else None
    st = _spectrum(C.c_void_p(mu.data_ptr()), d.ctypes.data_as(_ip), len(d), mu.shape[1] - 1, float(dt), C.byref(p),
                   float(tau), C.c_void_p(omega.data_ptr()), omega.shape[0], C.c_void_p(S.data_ptr()),
                   C.c_void_p(alpha.data_ptr()) if with_alpha else None,
                   C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != EFE_OK:
        raise EfeError(st, "absorption_spectrum")
    if with_alpha:
        return S, torch.view_as_complex(alpha)
    return S


def power_spectrum(mu, direction, dt, omega, tau):
    """Dipole power spectrum of a driven run (Sec. 3.5): mu (device float64 [nt + 1, 3]),
    omega (device float64 [nw]); returns P (device, nw)."""
    import torch
    for name, t in (("mu", mu), ("omega", omega)):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError(f"{name}: contiguous float64 device tensor expected")
    if mu.dim() != 2 or mu.shape[1] != 3:
        raise ValueError("mu: [nt + 1, 3] expected")
    P = torch.empty(omega.shape[0], dtype=torch.float64, device=omega.device)
    st = _power(C.c_void_p(mu.data_ptr()), int(direction), mu.shape[0] - 1, float(dt), float(tau),
                C.c_void_p(omega.data_ptr()), omega.shape[0], C.c_void_p(P.data_ptr()),
                C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != EFE_OK:
        raise EfeError(st, "power_spectrum")
    return P


def make_field(direction=2, A=(), w=(), phi=(), t0=0.0, s=1.0):
    """E(t) = dir * sum A_k sin(w_k t + phi_k) exp(-(t-t0)^2/s^2); returns (EfeField, keepalive)."""
    A, w, phi = _arr(A, np.float64), _arr(w, np.float64), _arr(phi, np.float64)
    f = EfeField()
    f.kind = 1 if len(A) else 0
    f.direction = int(direction)
    f.ncomp = int(len(A))
    f.A, f.w, f.phi = A.ctypes.data_as(_dp), w.ctypes.data_as(_dp), phi.ctypes.data_as(_dp)
    f.t0, f.s = float(t0), float(s)
    return f, (A, w, phi)


def field_vjp(field, t, dLdE):
    """sum_i dLdE[i] dE(t[i])/dtheta for a sum-of-sines field (efe_field_vjp);
    theta = (A, w, phi).  Returns 3 ncomp doubles."""
    tt, gg = _arr(t, np.float64), _arr(dLdE, np.float64)
    if tt.shape != gg.shape:
        raise ValueError("one sensitivity per time")
    out = np.zeros(3 * int(field.ncomp))
    st = _field_vjp(C.byref(field), len(tt), tt.ctypes.data_as(_dp), gg.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    if st != EFE_OK:
        raise EfeError(st, "efe_field_vjp")
    return out


def _stats_dict(st, n):
    return dict(k_pred=np.array(st.k_pred[:n]), k_corr=np.array(st.k_corr[:n]),
                err_pred_max=st.err_pred_max, err_corr_max=st.err_corr_max,
                cg_iters=tuple(st.cg_iters), mu=np.array(st.mu[:3]))


class Context:
    """A GPU context: static data uploaded, workspace allocated.

    reorth (efe_options.reorth): "partial" (default; with FP64 blocks the Lanczos
    coefficient alpha_j comes from the products), "partial_dot" (the same scheme with
    alpha_j from a dot pass) or "full"."""

    def __init__(self, spec, dtype="f64", kmax=None, tol=None, cg_tol=1e-12, cg_maxit=50, stream=None,
                 reorth="partial"):
        import torch
        self.torch = torch
        self.spec = spec
        self._h = _SystemHolder(spec)
        o = EfeOptions()
        o.prod_dtype = DTYPES[dtype]
        o.kmax = int(kmax if kmax is not None else min(spec.kmax, 64))
        o.krylov_tol = float(tol if tol is not None else spec.krylov_tol)
        o.cg_tol = float(cg_tol)
        o.cg_maxit = int(cg_maxit)
        o.reorth = REORTH[reorth]
        s = stream if stream is not None else torch.cuda.current_stream()
        o.hip_stream = C.c_void_p(s.cuda_stream)
        self._opt = o
        self._c = C.c_void_p()
        st = _setup(C.byref(self._h.sys), C.byref(o), C.byref(self._c))
        if st != EFE_OK:
            msg = _last_error(self._c).decode() if self._c else ""
            _free(self._c)
            self._c = None
            raise EfeError(st, msg)
        d = (C.c_int64 * 5)()
        _dims(self._c, d)
        self.n_rows, self.n_nodes, self.n_kept, self.n_quad, self.n_union_rows = [int(x) for x in d]
        self.norb = spec.norb
        self.kmax = o.kmax

    def set_options(self, kmax=None, tol=None, reorth=None):
        """Change the Krylov settings of the live context (kmax only downwards); a
        captured step is recorded again at its next use."""
        o = self._opt
        if kmax is not None:
            o.kmax = int(kmax)
        if tol is not None:
            o.krylov_tol = float(tol)
        if reorth is not None:
            o.reorth = REORTH[reorth]
        self._check(_set_options(self._c, C.byref(o)))
        self.kmax = o.kmax

    # -- helpers ---------------------------------------------------------------
    def _check(self, st):
        if st != EFE_OK:
            raise EfeError(st, _last_error(self._c).decode())

    def _ptr(self, t, dtype=None, rows=None):
        torch = self.torch
        if not t.is_cuda:
            raise ValueError("device tensor expected")
        if not t.is_contiguous():
            raise ValueError("contiguous tensor expected")
        if dtype is not None and t.dtype != dtype:
            raise ValueError(f"{dtype} expected, got {t.dtype}")
        if rows is not None and t.shape[0] != rows:
            raise ValueError(f"{rows} rows expected, got {t.shape[0]}")
        return C.c_void_p(t.data_ptr())

    def empty_block(self, ncol=None):
        torch = self.torch
        return torch.zeros((self.n_rows, ncol or self.norb), dtype=torch.complex128, device="cuda")

    # -- API ---------------------------------------------------------------------
    def initial_state(self, Psi=None):
        """Enrichment directions plus seeded FE noise, Loewdin-orthonormalised."""
        spec = self.spec
        Psi = self.empty_block() if Psi is None else Psi
        idx = _arr(spec.init_enr, np.int32)
        g = _arr(spec.noise(), np.float64).reshape(-1)
        self._check(_initial_state(self._c, idx.ctypes.data_as(_ip), g.ctypes.data_as(_dp),
                                   float(spec.noise_amp), self._ptr(Psi, self.torch.complex128, self.n_rows)))
        return Psi

    def set_hamiltonian(self, Psi, t=0.0, field=None):
        f = C.byref(field) if field is not None else None
        self._check(_set_ham(self._c, self._ptr(Psi, self.torch.complex128, self.n_rows), float(t), f))

    def apply_H(self, X, Y=None):
        ncol = X.shape[1]
        Y = self.torch.empty_like(X) if Y is None else Y
        self._check(_apply_H(self._c, self._ptr(X, self.torch.complex128, self.n_rows),
                             self._ptr(Y, self.torch.complex128, self.n_rows), ncol, ncol))
        return Y

    def apply_H_noalloc(self, X, Y):
        """Y = Hbar X enqueued with no allocation (efe_apply_H_noalloc): X, Y packed
        (n_rows x ncol contiguous), distinct; synchronise before reading Y."""
        torch = self.torch
        if X.shape != Y.shape or X.data_ptr() == Y.data_ptr():
            raise ValueError("X and Y: distinct blocks of the same shape")
        self._check(_apply_H_noalloc(self._c, self._ptr(X, torch.complex128, self.n_rows),
                                     self._ptr(Y, torch.complex128, self.n_rows), X.shape[1]))
        return Y

    def lanczos_expm(self, X, tau, op="H", k_force: Optional[Sequence[int]] = None):
        ncol = X.shape[1]
        ku = np.zeros(ncol, dtype=np.int32)
        er = np.zeros(ncol, dtype=np.float64)
        kf = None if k_force is None else _arr(k_force, np.int32)
        self._check(_lanczos(self._c, OPS[op], float(tau), self._ptr(X, self.torch.complex128, self.n_rows), ncol, ncol,
                             None if kf is None else kf.ctypes.data_as(_ip), ku.ctypes.data_as(_ip),
                             er.ctypes.data_as(_dp)))
        return ku, er

    def magnus_step(self, Psi, t, dt, field=None, k_force=None, graph=False, scheme="pc", keep_ham=True):
        """One Magnus-2 step in place.  graph=True replays a captured hipGraph of
        the device-driven step (no k_force).  scheme="extrap" takes the midpoint
        Hamiltonian at the density extrapolated from the last three steps
        (magnus_step_extrap); keep_ham=False leaves the midpoint Hamiltonian."""
        st = EfeStepStats()
        f = C.byref(field) if field is not None else None
        ptr = self._ptr(Psi, self.torch.complex128, self.n_rows)
        if scheme not in ("pc", "extrap"):
            raise ValueError(f"unknown scheme {scheme!r}")
        if scheme == "extrap":
            if graph:
                raise ValueError("the extrapolated step is host-driven (graph=False)")
            kf = None if k_force is None else _arr(k_force, np.int32).reshape(-1)
            self._check(_magnus_extrap(self._c, ptr, Psi.shape[1], float(t), float(dt), f,
                                       None if kf is None else kf.ctypes.data_as(_ip),
                                       EFE_STEP_KEEP_HAM if keep_ham else 0, C.byref(st)))
        elif graph:
            if k_force is not None:
                raise ValueError("k_force is not available with graph=True")
            self._check(_magnus_graph(self._c, ptr, Psi.shape[1], float(t), float(dt), f, C.byref(st)))
        else:
            kf = None if k_force is None else _arr(k_force, np.int32).reshape(-1)
            self._check(_magnus(self._c, ptr, Psi.shape[1], float(t), float(dt), f,
                                None if kf is None else kf.ctypes.data_as(_ip), C.byref(st)))
        return _stats_dict(st, self.norb)

    def magnus_adjoint(self, Psi, Psibar, t, dt, field=None, mubar=(0.0, 0.0, 0.0)):
        """Reverse of one step from Psi at t: Psibar (in: Xbar_{n+1}, out: Xbar_n).
        Returns (dL/dE(t), dL/dE(t + dt/2))."""
        mb = _arr(mubar, np.float64)
        out = np.zeros(2)
        f = C.byref(field) if field is not None else None
        self._check(_adjoint(self._c, self._ptr(Psi, self.torch.complex128, self.n_rows), Psi.shape[1], float(t),
                             float(dt), f, mb.ctypes.data_as(_dp),
                             self._ptr(Psibar, self.torch.complex128, self.n_rows), Psibar.shape[1],
                             out.ctypes.data_as(_dp)))
        return float(out[0]), float(out[1])

    def dipole_adjoint(self, Psi, mubar, Psibar=None):
        Psibar = self.torch.empty_like(Psi) if Psibar is None else Psibar
        mb = _arr(mubar, np.float64)
        self._check(_dip_adjoint(self._c, self._ptr(Psi, self.torch.complex128, self.n_rows), Psi.shape[1],
                                 mb.ctypes.data_as(_dp), self._ptr(Psibar, self.torch.complex128, self.n_rows),
                                 Psibar.shape[1]))
        return Psibar

    def density(self, Psi, rho=None):
        torch = self.torch
        rho = torch.empty(self.n_quad, dtype=torch.float64, device="cuda") if rho is None else rho
        self._check(_density(self._c, self._ptr(Psi, torch.complex128, self.n_rows), Psi.shape[1],
                             self._ptr(rho, torch.float64)))
        return rho

    def hartree(self, rho, phi=None):
        torch = self.torch
        phi = torch.empty(self.n_nodes, dtype=torch.float64, device="cuda") if phi is None else phi
        it = C.c_int32(0)
        self._check(_hartree(self._c, self._ptr(rho, torch.float64), self._ptr(phi, torch.float64), C.byref(it)))
        return phi, int(it.value)

    def dipole(self, Psi):
        mu = (C.c_double * 3)()
        self._check(_dipole(self._c, self._ptr(Psi, self.torch.complex128, self.n_rows), Psi.shape[1], mu))
        return np.array(mu[:3])

    def autotune(self, cache=None, force=False):
        """Pick the fastest cell-product kernel shape for this context (efe_autotune).
        Returns dict(choice, cached, times_us)."""
        buf = C.create_string_buffer(4096)
        self._check(_autotune(self._c, None if cache is None else os.fspath(cache).encode(),
                              EFE_TUNE_FORCE if force else 0, buf, len(buf)))
        out = {"times_us": {}, "rejected": {}}
        for tok in buf.value.decode().split():
            name, _, val = tok.partition("=")
            if name == "choice":
                out["choice"] = val
            elif name == "cached":
                out["cached"] = val == "1"
            elif val.startswith("rejected"):
                out["rejected"][name] = val
            else:
                out["times_us"][name] = float(val)
        return out

    def enable_timing(self, on=True):
        self._check(_timing_on(self._c, 1 if on else 0))

    def timing(self):
        ms = (C.c_double * 8)()
        n = C.c_int64(0)
        self._check(_timing_get(self._c, ms, C.byref(n)))
        keys = ["cell_hx", "coupling", "lanczos_vec", "tridiag_exp", "density", "poisson", "rebuild", "total"]
        out = dict(zip(keys, list(ms)))
        out["n_hx"] = int(n.value)
        return out

    def close(self):
        if getattr(self, "_c", None):
            _free(self._c)
            self._c = None

    def __del__(self):
        self.close()


class Batch:
    """Independent propagations stepped together: one captured hipGraph per
    step with the members' device-driven steps as concurrent branches.  Holds
    references to the contexts; close() before closing them."""

    def __init__(self, contexts):
        self.members = list(contexts)
        arr = (C.c_void_p * len(self.members))(*[c._c for c in self.members])
        self._b = C.c_void_p()
        st = _batch_create(arr, len(self.members), C.byref(self._b))
        if st != EFE_OK:
            msg = _batch_error(self._b).decode() if self._b else ""
            _batch_free(self._b)
            self._b = None
            raise EfeError(st, msg)

    def step(self, Psis, t, dt, fields=None):
        """One Magnus-2 step of every member in place; returns the per-member stats."""
        n = len(self.members)
        if len(Psis) != n:
            raise ValueError(f"{n} orbital blocks expected")
        ptrs = (C.c_void_p * n)(*[m._ptr(P, m.torch.complex128, m.n_rows).value for m, P in zip(self.members, Psis)])
        lds = (C.c_int64 * n)(*[P.shape[1] for P in Psis])
        fptr = None
        if fields is not None:
            fp = (C.POINTER(EfeField) * n)(*[C.pointer(f) if f is not None else None for f in fields])
            fptr = fp
        stats = (EfeStepStats * n)()
        st = _batch_step(self._b, ptrs, lds, float(t), float(dt), fptr, stats)
        if st != EFE_OK:
            raise EfeError(st, _batch_error(self._b).decode())
        return [_stats_dict(stats[i], m.norb) for i, m in enumerate(self.members)]

    def close(self):
        if getattr(self, "_b", None):
            _batch_free(self._b)
            self._b = None

    def __del__(self):
        self.close()
