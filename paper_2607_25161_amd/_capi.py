"""ctypes binding of include/fsd.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libfsd.so")

if not os.path.exists(library_path):
    raise ImportError(f"{library_path} is missing: build it with `python paper_2607_25161_amd/build.py`")

# One HIP runtime per process: PyTorch ships its own libamdhip64.so.7, and the
# library's dependency of that name must resolve to the copy torch uses (loading
# the system copy first leaves two runtimes competing for the device).
import torch  # noqa: E402,F401

lib = C.CDLL(library_path)

FSD_FP64, FSD_MIXED = 0, 1
_STATUS = {0: "FSD_OK", -1: "FSD_EINVAL", -2: "FSD_ENOMEM", -3: "FSD_ENOCONV", -4: "FSD_EDEVICE",
           -5: "FSD_ESTATE", -6: "FSD_EOVERLAP", -7: "FSD_EBUSY"}


class Params(C.Structure):
    _fields_ = [
        ("eta", C.c_double), ("radius", C.c_double), ("kT", C.c_double), ("xi", C.c_double),
        ("ewald_tol", C.c_double), ("grid", C.c_int), ("support", C.c_int), ("r_lub", C.c_double),
        ("r_precond", C.c_double), ("lub_eps_min", C.c_double), ("gmres_tol", C.c_double),
        ("gmres_restart", C.c_int), ("gmres_maxit", C.c_int), ("precision", C.c_int),
        ("lanczos_tol", C.c_double), ("seed", C.c_uint64), ("lanczos_maxit", C.c_int),
    ]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("restarts", C.c_int),
                ("refinements", C.c_int), ("rel_residual_fp64", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("L", C.c_double), ("xi", C.c_double), ("r_cut", C.c_double), ("h", C.c_double),
                ("eta_tilde", C.c_double), ("self_t", C.c_double), ("self_r", C.c_double),
                ("grid", C.c_int), ("support", C.c_int), ("n_bead", C.c_int), ("n_agg", C.c_int),
                ("nnz_real", C.c_longlong), ("n_lub_pairs", C.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_SYS = C.c_void_p


def _sig(name, res, *args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("fsd_default_params", None, C.POINTER(Params))
_sig("fsd_create", C.c_int, C.POINTER(Params), C.c_void_p, C.POINTER(C.c_void_p))
_sig("fsd_init_box", C.c_int, _SYS, C.c_double, C.c_double, C.c_double)
_sig("fsd_init_aggregates", C.c_int, _SYS, C.c_int32, _I32, _D, _D, _D)
_sig("fsd_set_forces", C.c_int, _SYS, _D)
_sig("fsd_set_bead_forces", C.c_int, _SYS, _D)
_sig("fsd_set_shear", C.c_int, _SYS, _D)
_sig("fsd_solve", C.c_int, _SYS, _D, _D, C.POINTER(SolveInfo))
_sig("fsd_solve_dev", C.c_int, _SYS, C.c_void_p, C.c_void_p, C.POINTER(SolveInfo))
_sig("fsd_step", C.c_int, _SYS, C.c_double, C.c_int, C.POINTER(SolveInfo))
_sig("fsd_get_state", C.c_int, _SYS, _D, _D, _D)
_sig("fsd_get_velocities", C.c_int, _SYS, _D)
_sig("fsd_get_info", C.c_int, _SYS, C.POINTER(Info))
_sig("fsd_get_stresslets", C.c_int, _SYS, _D, _D)
_sig("fsd_estimate_bytes", C.c_size_t, C.POINTER(Params), C.c_int32, C.c_int32, C.c_double)
_sig("fsd_last_error", C.c_char_p, _SYS)
_sig("fsd_destroy", None, _SYS)
_sig("fsd_apply_mobility", C.c_int, _SYS, _D, _D, C.c_int, C.c_int)
_sig("fsd_apply_saddle", C.c_int, _SYS, _D, _D, C.c_int)
_sig("fsd_apply_precond", C.c_int, _SYS, _D, _D)
_sig("fsd_get_rhs", C.c_int, _SYS, _D)
_sig("fsd_real_functions", C.c_int, _SYS, C.c_int, _D, _D)
_sig("fsd_fft3d", C.c_int, C.c_int, C.c_int, _D)
_sig("fsd_fft3d_noalloc", C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p)
_U64P = C.POINTER(C.c_uint64)
_sig("fsd_set_brownian", C.c_int, _SYS, C.c_double, C.c_uint64, C.c_uint64)
_sig("fsd_set_noise", C.c_int, _SYS, _D, _D, _D)
_sig("fsd_brownian_terms", C.c_int, _SYS, _D, _D, C.POINTER(C.c_int))
_sig("fsd_philox4x64", C.c_int, C.c_uint64, C.c_uint64, _U64P, C.c_int, _U64P)
_sig("fsd_normals", C.c_int, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_size_t, _D)
_sig("fsd_set_timing", C.c_int, _SYS, C.c_int)
_sig("fsd_set_graphs", C.c_int, _SYS, C.c_int, C.c_int)
_sig("fsd_get_timers", C.c_int, _SYS, _D, C.POINTER(C.c_longlong), _D)
_sig("fsd_set_pair_forces", C.c_int, _SYS, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double)
_sig("fsd_get_pair_forces", C.c_int, _SYS, _D)
_sig("fsd_set_roughness", C.c_int, _SYS, C.c_double, C.c_double)
_sig("fsd_set_lees_edwards", C.c_int, _SYS, C.c_int, C.c_double)
_sig("fsd_get_strain", C.c_int, _SYS, _D)
_sig("fsd_set_warm_start", C.c_int, _SYS, C.c_int)
_sig("fsd_set_drift", C.c_int, _SYS, C.c_int, C.c_double)
_sig("fsd_rfd_drift", C.c_int, _SYS, _D, _D)
_sig("fsd_time_kernel", C.c_int, _SYS, C.c_int, C.c_int, _D)
_sig("fsd_autotune_xi", C.c_int, _SYS, C.c_double, C.c_double, C.c_int, _D, _D)
_sig("fsd_autotune_tiles", C.c_int, _SYS, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int))

_sig("fsd_batch_create", C.c_int, C.c_size_t, C.c_int, C.c_void_p, C.POINTER(C.c_void_p))
_sig("fsd_batch_admit", C.c_int, C.c_void_p, _SYS, C.POINTER(C.c_int))
_sig("fsd_batch_retire", C.c_int, C.c_void_p, C.c_int)
_sig("fsd_batch_solve", C.c_int, C.c_void_p)
_sig("fsd_batch_step", C.c_int, C.c_void_p, C.c_double)
_sig("fsd_batch_step_counts", C.c_int, C.c_void_p, C.c_double, C.POINTER(C.c_int))
_sig("fsd_batch_slot_info", C.c_int, C.c_void_p, C.c_int, C.POINTER(SolveInfo))
_sig("fsd_batch_used_bytes", C.c_size_t, C.c_void_p)
_sig("fsd_batch_destroy", None, C.c_void_p)
_sig("fsd_batch_set_fused", C.c_int, C.c_void_p, C.c_int)
_sig("fsd_batch_set_graphs", C.c_int, C.c_void_p, C.c_int)
_sig("fsd_batch_set_timing", C.c_int, C.c_void_p, C.c_int)
_sig("fsd_batch_get_timers", C.c_int, C.c_void_p, _D, C.POINTER(C.c_longlong), _D)
_sig("fsd_batch_time_kernel", C.c_int, C.c_void_p, C.c_int, C.c_int, _D, _D)
_sig("fsd_batch_autotune_tiles", C.c_int, C.c_void_p, C.c_int, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t))
_sig("fsd_batch_set_lds_caps", C.c_int, C.c_void_p, C.c_size_t, C.c_size_t)

TIMER_NAMES = ("real_sum", "spread", "fft_first", "fft_y", "fft_green", "fft_last", "interp", "rigid_lub",
               "precond", "cgs_dot", "cgs_update", "cgs_norm_arnoldi")


class FsdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


def _dptr(a):
    return a.ctypes.data_as(_D)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def default_params(**kw) -> Params:
    p = Params()
    lib.fsd_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def estimate_bytes(params: Params, n_bead: int, n_agg: int, L: float) -> int:
    return int(lib.fsd_estimate_bytes(C.byref(params), n_bead, n_agg, L))


def philox4x64(k0: int, k1: int, counter, n_blocks: int) -> np.ndarray:
    """Raw device Philox4x64-10 words: block b enciphers (counter[0] + b, counter[1:])."""
    ctr = np.ascontiguousarray(counter, dtype=np.uint64)
    out = np.zeros(4 * n_blocks, dtype=np.uint64)
    rc = lib.fsd_philox4x64(k0, k1, ctr.ctypes.data_as(_U64P), n_blocks, out.ctypes.data_as(_U64P))
    if rc:
        raise FsdError(rc, f"fsd_philox4x64: {lib.fsd_last_error(None).decode()}")
    return out


def normals(k0: int, k1: int, purpose: int, step: int, n: int) -> np.ndarray:
    out = np.zeros(n)
    rc = lib.fsd_normals(k0, k1, purpose, step, n, _dptr(out))
    if rc:
        raise FsdError(rc, f"fsd_normals: {lib.fsd_last_error(None).decode()}")
    return out


def fft3d(data: np.ndarray, sign: int) -> np.ndarray:
    """Library 3D FFT of a complex n^3 array (index order [z, y, x]); unnormalised."""
    a = np.ascontiguousarray(data, dtype=np.complex128)
    n = a.shape[0]
    buf = a.view(np.float64).copy()
    rc = lib.fsd_fft3d(n, sign, _dptr(buf))
    if rc:
        raise FsdError(rc, f"fsd_fft3d: {lib.fsd_last_error(None).decode()}")
    return buf.view(np.complex128).reshape(a.shape)


def fft3d_noalloc(n: int, sign: int, data_ptr: int, stream=None):
    """fsd_fft3d_noalloc: in place on a device buffer of n^3 complex doubles (e.g. a torch
    complex128 tensor's data_ptr()), stream-ordered on `stream` (a hipStream_t handle)."""
    rc = lib.fsd_fft3d_noalloc(int(n), int(sign), C.c_void_p(int(data_ptr)), C.c_void_p(stream) if stream else None)
    if rc:
        raise FsdError(rc, f"fsd_fft3d_noalloc: {lib.fsd_last_error(None).decode()}")


class System:
    """One periodic suspension resident on the GPU (wraps fsd_system)."""

    def __init__(self, params: Params | None = None, stream=None, **kw):
        self.params = params if params is not None else default_params(**kw)
        h = C.c_void_p()
        st = C.c_void_p(int(stream)) if stream else None
        self._check(lib.fsd_create(C.byref(self.params), st, C.byref(h)), "fsd_create", raw=True)
        self._h = h
        self.n_agg = self.n_bead = 0

    # -- plumbing ---------------------------------------------------------------------
    def _check(self, rc, what, raw=False):
        if rc:
            msg = what if raw else f"{what}: {lib.fsd_last_error(self._h).decode()}"
            raise FsdError(rc, msg)
        return rc

    def close(self):
        if getattr(self, "_h", None):
            lib.fsd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- setup ------------------------------------------------------------------------
    def init_box(self, L, Ly=None, Lz=None):
        Ly = L if Ly is None else Ly
        Lz = L if Lz is None else Lz
        self._check(lib.fsd_init_box(self._h, float(L), float(Ly), float(Lz)), "fsd_init_box")

    def init_aggregates(self, offsets, x_body, com, quat):
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        na = len(off) - 1
        nb = int(off[-1])
        xb, X, q = _f64(x_body, 3 * nb), _f64(com, 3 * na), _f64(quat, 4 * na)
        self._check(lib.fsd_init_aggregates(self._h, na, off.ctypes.data_as(_I32), _dptr(xb), _dptr(X), _dptr(q)),
                    "fsd_init_aggregates")
        self.n_agg, self.n_bead = na, nb

    def set_forces(self, ft):
        a = _f64(ft, 6 * self.n_agg)
        self._check(lib.fsd_set_forces(self._h, _dptr(a)), "fsd_set_forces")

    def set_bead_forces(self, f):
        a = _f64(f, 3 * self.n_bead)
        self._check(lib.fsd_set_bead_forces(self._h, _dptr(a)), "fsd_set_bead_forces")

    def set_shear(self, grad_u):
        a = _f64(grad_u, 9)
        self._check(lib.fsd_set_shear(self._h, _dptr(a)), "fsd_set_shear")

    # -- solve ------------------------------------------------------------------------
    def solve(self, want_lambda=False, check=True):
        U = np.zeros((self.n_agg, 6))
        lam = np.zeros((self.n_bead, 6)) if want_lambda else None
        info = SolveInfo()
        rc = lib.fsd_solve(self._h, _dptr(U), _dptr(lam) if lam is not None else None, C.byref(info))
        if check:
            self._check(rc, "fsd_solve")
        return U, lam, info

    def solve_dev(self, U_ptr: int, lam_ptr: int | None = None, check=True):
        info = SolveInfo()
        rc = lib.fsd_solve_dev(self._h, C.c_void_p(U_ptr), C.c_void_p(lam_ptr) if lam_ptr else None, C.byref(info))
        if check:
            self._check(rc, "fsd_solve_dev")
        return info

    def step(self, dt, n_steps=1):
        info = SolveInfo()
        self._check(lib.fsd_step(self._h, float(dt), int(n_steps), C.byref(info)), "fsd_step")
        return info

    def state(self, beads=False):
        X = np.zeros((self.n_agg, 3))
        q = np.zeros((self.n_agg, 4))
        xb = np.zeros((self.n_bead, 3)) if beads else None
        self._check(lib.fsd_get_state(self._h, _dptr(X), _dptr(q), _dptr(xb) if beads else None), "fsd_get_state")
        return (X, q, xb) if beads else (X, q)

    def stresslets(self):
        """(per-aggregate constraint stresslets (n_agg, 3, 3), suspension particle stress (3, 3))
        of the last solve."""
        S = np.zeros((self.n_agg, 3, 3))
        m = np.zeros((3, 3))
        self._check(lib.fsd_get_stresslets(self._h, _dptr(S), _dptr(m)), "fsd_get_stresslets")
        return S, m

    def velocities(self):
        """Aggregate velocities (n_agg, 6) of the last completed solve, by any call."""
        U = np.zeros((self.n_agg, 6))
        self._check(lib.fsd_get_velocities(self._h, _dptr(U)), "fsd_get_velocities")
        return U

    def info(self) -> Info:
        inf = Info()
        self._check(lib.fsd_get_info(self._h, C.byref(inf)), "fsd_get_info")
        return inf

    # -- operators --------------------------------------------------------------------
    def apply_mobility(self, lam, parts=3, precision=FSD_FP64):
        a = _f64(lam, 6 * self.n_bead)
        out = np.zeros(6 * self.n_bead)
        self._check(lib.fsd_apply_mobility(self._h, _dptr(a), _dptr(out), parts, precision), "fsd_apply_mobility")
        return out

    def apply_saddle(self, x, precision=FSD_FP64):
        n = 6 * (self.n_bead + self.n_agg)
        a = _f64(x, n)
        out = np.zeros(n)
        self._check(lib.fsd_apply_saddle(self._h, _dptr(a), _dptr(out), precision), "fsd_apply_saddle")
        return out

    def apply_precond(self, r):
        n = 6 * (self.n_bead + self.n_agg)
        a = _f64(r, n)
        out = np.zeros(n)
        self._check(lib.fsd_apply_precond(self._h, _dptr(a), _dptr(out)), "fsd_apply_precond")
        return out

    def rhs(self):
        out = np.zeros(6 * (self.n_bead + self.n_agg))
        self._check(lib.fsd_get_rhs(self._h, _dptr(out)), "fsd_get_rhs")
        return out

    def real_functions(self, r):
        r = _f64(r)
        out = np.zeros((len(r), 5))
        self._check(lib.fsd_real_functions(self._h, len(r), _dptr(r), _dptr(out)), "fsd_real_functions")
        return out

    # -- launch mode and timing ---------------------------------------------------------
    def set_pair_forces(self, k_n=0.0, hamaker=0.0, Z=0.0, kappa=0.0, h_c=0.0, r_cut=None):
        """Hertz contact, van der Waals and double-layer forces between beads of different
        bodies (all zero: off).  r_cut defaults to 3a."""
        rc = 3.0 * self.params.radius if r_cut is None else float(r_cut)
        self._check(lib.fsd_set_pair_forces(self._h, float(k_n), float(hamaker), float(Z), float(kappa),
                                            float(h_c), rc), "fsd_set_pair_forces")

    def pair_forces(self):
        """(n_bead, 3) conservative bead forces at the current positions."""
        out = np.zeros(3 * self.n_bead)
        self._check(lib.fsd_get_pair_forces(self._h, _dptr(out)), "fsd_get_pair_forces")
        return out.reshape(-1, 3)

    def set_lees_edwards(self, enable=True, strain=0.0):
        """Sheared periodic lattice of the given strain (before init_aggregates to switch
        on; the strain may be reset later)."""
        self._check(lib.fsd_set_lees_edwards(self._h, int(bool(enable)), float(strain)), "fsd_set_lees_edwards")

    def set_warm_start(self, mode=1):
        """GMRES initial guess: 0 (or False) zero, 1 (or True) the previous converged solution,
        2 and 3 the linear and quadratic extrapolations of the last two and three (same
        stopping test)."""
        self._check(lib.fsd_set_warm_start(self._h, int(mode)), "fsd_set_warm_start")

    def strain(self):
        out = C.c_double(0.0)
        self._check(lib.fsd_get_strain(self._h, C.byref(out)), "fsd_get_strain")
        return out.value

    def set_roughness(self, alpha=0.0, h0=0.0):
        """Tangential roughness of lubrication: strength alpha below the asperity height h0
        (alpha 0: off)."""
        self._check(lib.fsd_set_roughness(self._h, float(alpha), float(h0)), "fsd_set_roughness")

    def set_drift(self, mode=1, eps=0.0):
        """Brownian drift in every step: 1 random finite differences (eps; <= 0: default),
        2 Fixman's midpoint scheme (eps is m; <= 0: 100), 0 off."""
        self._check(lib.fsd_set_drift(self._h, int(mode), float(eps)), "fsd_set_drift")

    def rfd_drift(self, dq=None):
        """(n_agg, 6) drift kT (U+ - U-) / eps for dq (n_agg, 6), or the next step's dq."""
        out = np.zeros(6 * self.n_agg)
        a = _f64(dq, 6 * self.n_agg) if dq is not None else None
        self._check(lib.fsd_rfd_drift(self._h, _dptr(a) if a is not None else None, _dptr(out)), "fsd_rfd_drift")
        return out.reshape(-1, 6)

    def set_brownian(self, dt, step=0, stream=0):
        self._check(lib.fsd_set_brownian(self._h, float(dt), int(step), int(stream)), "fsd_set_brownian")

    def set_noise(self, psi_w=None, psi_r=None, psi_nf=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (psi_w, psi_r, psi_nf)]
        ptrs = [None if a is None else _dptr(a) for a in arrs]
        self._check(lib.fsd_set_noise(self._h, *ptrs), "fsd_set_noise")

    def brownian_terms(self):
        """(u_B (n_bead, 6), F_B (n_bead, 3), lanczos steps (real, near))."""
        u = np.zeros((self.n_bead, 6))
        f = np.zeros((self.n_bead, 3))
        its = (C.c_int * 2)()
        self._check(lib.fsd_brownian_terms(self._h, _dptr(u), _dptr(f), its), "fsd_brownian_terms")
        return u, f, (its[0], its[1])

    def set_graphs(self, enable=True, batch=0):
        self._check(lib.fsd_set_graphs(self._h, 1 if enable else 0, int(batch)), "fsd_set_graphs")

    def set_timing(self, enable=True):
        self._check(lib.fsd_set_timing(self._h, 1 if enable else 0), "fsd_set_timing")

    def timers(self):
        """{class: (total_ms, launches, algorithmic_bytes)} since the last set_timing."""
        ms = np.zeros(len(TIMER_NAMES))
        by = np.zeros(len(TIMER_NAMES))
        cnt = (C.c_longlong * len(TIMER_NAMES))()
        self._check(lib.fsd_get_timers(self._h, _dptr(ms), cnt, _dptr(by)), "fsd_get_timers")
        return {n: (float(ms[k]), int(cnt[k]), float(by[k])) for k, n in enumerate(TIMER_NAMES)}

    def time_kernel(self, timer, reps=200):
        """Average ms of one launch of the kernel behind `timer` (a TIMER_NAMES entry),
        replayed `reps` times back to back between one pair of events."""
        out = C.c_double(0.0)
        self._check(lib.fsd_time_kernel(self._h, TIMER_NAMES.index(timer), int(reps), C.byref(out)),
                    "fsd_time_kernel")
        return out.value

    def autotune_xi(self, xi_lo, xi_hi, reps=10):
        """(xi, ms per saddle apply) of the fastest splitting parameter in [xi_lo, xi_hi]."""
        xi, ms = C.c_double(0.0), C.c_double(0.0)
        self._check(lib.fsd_autotune_xi(self._h, float(xi_lo), float(xi_hi), int(reps), C.byref(xi), C.byref(ms)),
                    "fsd_autotune_xi")
        return xi.value, ms.value

    def autotune_tiles(self, reps=20):
        """(lines per workgroup of the z/y passes, row pairs per workgroup of the x+Green pass),
        measured and kept for this system."""
        b, g = C.c_int(0), C.c_int(0)
        self._check(lib.fsd_autotune_tiles(self._h, int(reps), C.byref(b), C.byref(g)), "fsd_autotune_tiles")
        return b.value, g.value

    # -- convenience ------------------------------------------------------------------
    @classmethod
    def from_suspension(cls, s, stream=None, lees_edwards=False, **overrides):
        """Build from any object with the workload attributes (L, a, eta, offsets, ...);
        lees_edwards=True puts it on the sheared lattice (strain 0) before the aggregates."""
        kw = dict(eta=s.eta, radius=s.a, xi=s.xi, ewald_tol=s.ewald_tol, grid=s.grid, r_lub=s.r_lub,
                  r_precond=s.r_precond, gmres_tol=s.gmres_tol, kT=getattr(s, "kT", 0.0))
        kw.update({k: v for k, v in (getattr(s, "extra", None) or {}).items() if k in ("gmres_maxit", "seed")})
        kw.update(overrides)
        sysm = cls(default_params(**kw), stream=stream)
        sysm.init_box(s.L)
        if lees_edwards:
            sysm.set_lees_edwards(True, 0.0)
        sysm.init_aggregates(s.offsets, s.x_body, s.com, s.quat)
        sysm.set_forces(s.force)
        sysm.set_shear(s.grad_u)
        return sysm


class Batch:
    """Independent systems sharing the GPU (wraps fsd_batch)."""

    def __init__(self, mem_budget_bytes: int, max_slots: int, stream=None):
        h = C.c_void_p()
        rc = lib.fsd_batch_create(int(mem_budget_bytes), int(max_slots), C.c_void_p(stream) if stream else None,
                                  C.byref(h))
        if rc:
            raise FsdError(rc, "fsd_batch_create")
        self._h = h
        self.max_slots = int(max_slots)
        self.systems = {}

    def admit(self, system: "System") -> int:
        slot = C.c_int()
        rc = lib.fsd_batch_admit(self._h, system._h, C.byref(slot))
        if rc:
            raise FsdError(rc, "fsd_batch_admit")
        self.systems[slot.value] = system
        return slot.value

    def try_admit(self, system: "System"):
        """Slot index, or None when the batch is full or over its memory budget."""
        slot = C.c_int()
        rc = lib.fsd_batch_admit(self._h, system._h, C.byref(slot))
        if rc == -7:
            return None
        if rc:
            raise FsdError(rc, "fsd_batch_admit")
        self.systems[slot.value] = system
        return slot.value

    def retire(self, slot: int):
        rc = lib.fsd_batch_retire(self._h, int(slot))
        if rc:
            raise FsdError(rc, "fsd_batch_retire")
        return self.systems.pop(slot)

    def solve(self):
        return lib.fsd_batch_solve(self._h)

    def step(self, dt: float):
        return lib.fsd_batch_step(self._h, float(dt))

    def step_counts(self, dt: float, counts: dict):
        """Time steps per slot in one call ({slot: n}; slots left out take none)."""
        n = (C.c_int * self.max_slots)()
        for sl, k in counts.items():
            n[int(sl)] = int(k)
        return lib.fsd_batch_step_counts(self._h, float(dt), n)

    def info(self, slot: int) -> SolveInfo:
        inf = SolveInfo()
        rc = lib.fsd_batch_slot_info(self._h, int(slot), C.byref(inf))
        if rc:
            raise FsdError(rc, "fsd_batch_slot_info")
        return inf

    def used_bytes(self) -> int:
        return int(lib.fsd_batch_used_bytes(self._h))

    def set_fused(self, enable=True):
        """Multi-system launches (True) or one stream per system (False)."""
        rc = lib.fsd_batch_set_fused(self._h, 1 if enable else 0)
        if rc:
            raise FsdError(rc, "fsd_batch_set_fused")

    def set_timing(self, enable=True):
        rc = lib.fsd_batch_set_timing(self._h, 1 if enable else 0)
        if rc:
            raise FsdError(rc, "fsd_batch_set_timing")

    def timers(self):
        """{timer: (total ms, launches, algorithmic bytes)} of the multi-system launches."""
        n = len(TIMER_NAMES)
        ms, by = np.zeros(n), np.zeros(n)
        cnt = (C.c_longlong * n)()
        rc = lib.fsd_batch_get_timers(self._h, _dptr(ms), cnt, _dptr(by))
        if rc:
            raise FsdError(rc, "fsd_batch_get_timers")
        return {name: (float(ms[k]), int(cnt[k]), float(by[k])) for k, name in enumerate(TIMER_NAMES)}

    def time_kernel(self, timer, reps=50):
        """(average ms, algorithmic bytes) of one multi-system launch of `timer` over every
        admitted system, replayed back to back."""
        ms, by = C.c_double(0.0), C.c_double(0.0)
        rc = lib.fsd_batch_time_kernel(self._h, TIMER_NAMES.index(timer), int(reps), C.byref(ms), C.byref(by))
        if rc:
            raise FsdError(rc, "fsd_batch_time_kernel")
        return ms.value, by.value

    def autotune_tiles(self, reps=20):
        """Measured LDS caps (bytes, 0: none) of the multi-system line passes and x+Green
        pass; later launches of the batch use them."""
        a, g = C.c_size_t(0), C.c_size_t(0)
        rc = lib.fsd_batch_autotune_tiles(self._h, int(reps), C.byref(a), C.byref(g))
        if rc:
            raise FsdError(rc, "fsd_batch_autotune_tiles")
        return a.value, g.value

    def set_graphs(self, enable=True):
        """Captured graphs for the lock-step segments (default on)."""
        rc = lib.fsd_batch_set_graphs(self._h, 1 if enable else 0)
        if rc:
            raise FsdError(rc, "fsd_batch_set_graphs")

    def set_lds_caps(self, lines, green):
        """LDS caps (bytes, 0: none) of the multi-system line passes and x+Green pass."""
        rc = lib.fsd_batch_set_lds_caps(self._h, int(lines), int(green))
        if rc:
            raise FsdError(rc, "fsd_batch_set_lds_caps")

    def close(self):
        if getattr(self, "_h", None):
            lib.fsd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
