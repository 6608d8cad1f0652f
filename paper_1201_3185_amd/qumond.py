"""Thin ctypes binding of libqumond.so (include/qumond.h, qumond_kernels.h,
qumond_tune.h, qumond_unet.h, qumond_batch.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream (``torch.cuda.current_stream()``); every step of the solve runs in the
library's gfx950 kernels.  ``torch`` is imported before the library is loaded
so both use the one HIP runtime in the process.  There is no fallback: if the
library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional

import torch  # noqa: F401  (must precede loading libqumond.so: shared HIP runtime)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqumond.so")
MAX_BOX = 16

QUMOND_OK, QUMOND_ERR_INVALID, QUMOND_ERR_STATE, QUMOND_ERR_OOM, QUMOND_ERR_HIP, QUMOND_ERR_NOT_CONVERGED, \
    QUMOND_ERR_RANGE = range(7)
QUMOND_FP64, QUMOND_MIXED = 0, 1
QUMOND_BC_ZERO, QUMOND_BC_MONOPOLE = 0, 1
FIELD_RHO_FIXED, FIELD_RHS, FIELD_PHI_N, FIELD_SOURCE, FIELD_PHI = range(5)
GUESS_NONE, GUESS_F64, GUESS_F32, GUESS_BF16 = range(4)
GUESS_NO_FALLBACK = 16
WHICH_NEWTON, WHICH_QUMOND, WHICH_ALGEBRAIC = range(3)


class qumond_config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("nbox", ctypes.c_int32), ("box_side", ctypes.c_double * MAX_BOX),
        ("G", ctypes.c_double), ("a0", ctypes.c_double), ("npre", ctypes.c_int32), ("npost", ctypes.c_int32),
        ("ncycle_fmg", ctypes.c_int32), ("max_vcycles", ctypes.c_int32), ("tol_rel", ctypes.c_double),
        ("precision", ctypes.c_int32), ("outer_bc", ctypes.c_int32), ("gather_frac", ctypes.c_double),
        ("fixed_shift", ctypes.c_int32), ("use_graphs", ctypes.c_int32), ("nu_n", ctypes.c_double),
    ]


class qumond_solve_info(ctypes.Structure):
    _fields_ = [
        ("nbox", ctypes.c_int32), ("vcycles", ctypes.c_int32 * MAX_BOX), ("converged", ctypes.c_int32 * MAX_BOX),
        ("refine_iters", ctypes.c_int32 * MAX_BOX), ("relres0", ctypes.c_double * MAX_BOX),
        ("relres", ctypes.c_double * MAX_BOX), ("used_fallback", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        nb = self.nbox
        return {"vcycles": list(self.vcycles[:nb]), "converged": list(self.converged[:nb]),
                "refine_iters": list(self.refine_iters[:nb]), "relres0": list(self.relres0[:nb]),
                "relres": list(self.relres[:nb]), "used_fallback": int(self.used_fallback)}


class qumond_batch_config(ctypes.Structure):
    _fields_ = [
        ("nprob", ctypes.c_int32), ("box_side", ctypes.c_double), ("G", ctypes.c_double), ("a0", ctypes.c_double),
        ("npre", ctypes.c_int32), ("npost", ctypes.c_int32), ("ncycle_fmg", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32), ("max_extra", ctypes.c_int32), ("tol_rel", ctypes.c_double),
        ("gather_frac", ctypes.c_double), ("naz", ctypes.c_int32), ("autotune", ctypes.c_int32),
        ("nu_n", ctypes.c_double),
    ]


class qumond_batch_problem_info(ctypes.Structure):
    _fields_ = [
        ("relres_newton", ctypes.c_double), ("relres_mond", ctypes.c_double), ("steps_newton", ctypes.c_int32),
        ("steps_mond", ctypes.c_int32), ("converged", ctypes.c_int32), ("redone", ctypes.c_int32),
        ("n_inside", ctypes.c_int64),
    ]


class qumond_kernel_stats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double),
                ("sweeps_per_launch", ctypes.c_int32)]


_P, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIGNATURES = {
    "qumond_default_config": (None, [ctypes.POINTER(qumond_config)]),
    "qumond_validate_config": (_I32, [ctypes.POINTER(qumond_config)]),
    "qumond_create": (_I32, [ctypes.POINTER(qumond_config), _P, ctypes.POINTER(_P)]),
    "qumond_destroy": (_I32, [_P]),
    "qumond_deposit": (_I32, [_P, _P, _P, _P, _P, _I64, _D, ctypes.POINTER(_I64)]),
    "qumond_solve_newton": (_I32, [_P, ctypes.POINTER(qumond_solve_info)]),
    "qumond_mond_source": (_I32, [_P]),
    "qumond_solve": (_I32, [_P, ctypes.POINTER(qumond_solve_info), ctypes.POINTER(qumond_solve_info)]),
    "qumond_solve_mond": (_I32, [_P, _P, _I32, ctypes.POINTER(qumond_solve_info)]),
    "qumond_gather_forces": (_I32, [_P, _P, _P, _P, _I64, _I32, _P, _P, _P, _P]),
    "qumond_rotation_curve": (_I32, [_P, _P, _I32, _I32, _I32, _P]),
    "qumond_sigma_z": (_I32, [_P, _P, _I32, _I32, _D, _D, _I32, _P]),
    "qumond_get_field": (_I32, [_P, _I32, _I32, _P]),
    "qumond_set_field": (_I32, [_P, _I32, _I32, _P]),
    "qumond_device_bytes": (_I64, [_P]),
    "qumond_profile_enable": (_I32, [_P, _I32]),
    "qumond_profile_read": (_I32, [_P, ctypes.POINTER(qumond_kernel_stats)]),
    "qumond_status_string": (ctypes.c_char_p, [_I32]),
    "qumond_last_error": (ctypes.c_char_p, []),
    "qumond_k_rbgs_sweep": (_I32, [_I32, _D, _P, _P, _P, _P]),
    "qumond_k_rbgs_sweep_from_zero": (_I32, [_I32, _D, _P, _P, _P]),
    "qumond_k_rbgs_double_sweep": (_I32, [_I32, _D, _P, _P, _P, _P, _P]),
    "qumond_k_residual_restrict": (_I32, [_I32, _D, _P, _P, _P, _P, _P, _P]),
    "qumond_k_rbgs_sweep_restrict": (_I32, [_I32, _D, _P, _P, _P, _P, _P, _P, _P]),
    "qumond_k_restrict": (_I32, [_I32, _P, _P, _P]),
    "qumond_k_prolong_add": (_I32, [_I32, _P, _P, _P]),
    "qumond_k_interp": (_I32, [_I32, _P, _P, _P]),
    "qumond_k_mond_source": (_I32, [_I32, _D, _D, _P, _P, _P]),
    "qumond_k_bc_from_coarse": (_I32, [_I32, _P, _P, _P]),
    "qumond_k_resid_norms": (_I32, [_I32, _D, _P, _P, _P, _P]),
    "qumond_k_resid_norms_noalloc": (_I32, [_I32, _D, _P, _P, _P, _P]),
    "qumond_k_fmg": (_I32, [_I32, _D, _P, _P, _I32, _I32, _I32, _I32, _D, ctypes.POINTER(_D),
                            ctypes.POINTER(_I32), _P]),
    "qumond_k_vcycles": (_I32, [_I32, _D, _P, _P, _I32, _I32, _I32, ctypes.POINTER(_D), _P]),
    "qumond_unet_create": (_I32, [_I32, ctypes.c_uint64, _P, ctypes.POINTER(_P)]),
    "qumond_unet_destroy": (_I32, [_P]),
    "qumond_unet_param_count": (_I64, [_P]),
    "qumond_unet_get_params": (_I32, [_P, _P]),
    "qumond_unet_set_params": (_I32, [_P, _P]),
    "qumond_unet_get_grads": (_I32, [_P, _P]),
    "qumond_unet_prepare_sample": (_I32, [_P, _P, _P, _P, _D, _D, _D, _D, _D, _D, _P, _P]),
    "qumond_unet_train_step": (_I32, [_P, _P, _P, ctypes.c_float, ctypes.POINTER(_D)]),
    "qumond_unet_infer": (_I32, [_P, _P, _P, _D, _D, _D, _D, _D, _D, _P]),
    "qumond_k_conv3d_fwd": (_I32, [_I32, _I32, _P, _I32, _P, _P, _I32, _I32, _P, _P]),
    "qumond_k_conv3d_dgrad": (_I32, [_I32, _I32, _I32, _P, _I32, _P, _P, _P]),
    "qumond_k_conv3d_wgrad": (_I32, [_I32, _I32, _P, _I32, _P, _I32, _P, _P]),
    "qumond_tune_set": (_I32, [_I32, _I32, _I32, _I32]),
    "qumond_tune_get": (_I32, [_I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "qumond_tune_set_corr": (_I32, [_I32, _I32, _I32, _I32]),
    "qumond_tune_set_sweep_restrict": (_I32, [_I32, _I32, _I32]),
    "qumond_tune_get_sweep_restrict": (_I32, [_I32, _I32, ctypes.POINTER(_I32)]),
    "qumond_tune_get_corr": (_I32, [_I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "qumond_tune_set_fused": (_I32, [_I32, _I32, _I32, _I32]),
    "qumond_tune_get_fused": (_I32, [_I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "qumond_k_rbgs_sweep_shape": (_I32, [_I32, _D, _P, _P, _P, _I32, _I32, _P, _P]),
    "qumond_k_rbgs_sweep_stacked": (_I32, [_I32, _I32, _D, _P, _P, _P, _I32, _I32, _P]),
    "qumond_autotune": (_I32, [_I32, _I32, _I32, ctypes.c_char_p, ctypes.POINTER(_D), _P]),
    "qumond_tune_load": (_I32, [ctypes.c_char_p]),
    "qumond_tune_set_rr": (_I32, [_I32, _I32, _I32]),
    "qumond_tune_get_rr": (_I32, [_I32, _I32, ctypes.POINTER(_I32)]),
    "qumond_tune_set_split": (_I32, [_I32, _I32, _I32]),
    "qumond_tune_get_split": (_I32, [_I32, _I32, ctypes.POINTER(_I32)]),
    "qumond_batch_default_config": (None, [ctypes.POINTER(qumond_batch_config)]),
    "qumond_batch_validate": (_I32, [ctypes.POINTER(qumond_batch_config), _P, _P, _I32]),
    "qumond_batch_create": (_I32, [ctypes.POINTER(qumond_batch_config), _P, _P, _I32, _P, ctypes.POINTER(_P)]),
    "qumond_batch_destroy": (_I32, [_P]),
    "qumond_batch_set_particles": (_I32, [_P, _I32, _P, _P, _P, _P, _I64, _D]),
    "qumond_batch_run": (_I32, [_P, _I32, _P]),
    "qumond_batch_rotation_curves": (_I32, [_P, _I32, _P]),
    "qumond_batch_get_field": (_I32, [_P, _I32, _I32, _P]),
    "qumond_batch_describe": (_I32, [_P, ctypes.c_char_p, _I64]),
    "qumond_batch_device_bytes": (_I64, [_P]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libqumond.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1201_3185_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> List[str]:
    return list(_SIGNATURES)


class QumondError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().qumond_last_error().decode()
        super().__init__(f"{where}: {lib().qumond_status_string(status).decode()} ({msg})")


def check(status: int, where: str, allow=()) -> int:
    if status != QUMOND_OK and status not in allow:
        raise QumondError(status, where)
    return status


@dataclass
class Config:
    n: int = 65
    box_side: List[float] = field(default_factory=lambda: [100.0])
    G: float = 4.300917270e-6
    a0: float = 3600.0
    npre: int = 2
    npost: int = 2
    ncycle_fmg: int = 6
    max_vcycles: int = 50
    tol_rel: float = 1e-10
    precision: int = QUMOND_FP64
    outer_bc: int = QUMOND_BC_MONOPOLE
    gather_frac: float = 0.2
    fixed_shift: int = 0
    use_graphs: int = 0
    nu_n: float = 1.0            # 1: Eq. 2's nu; else the n-family member (2: the standard nu)

    def to_c(self) -> qumond_config:
        c = qumond_config()
        c.n, c.nbox = self.n, len(self.box_side)
        for b, Lb in enumerate(self.box_side[:MAX_BOX]):
            c.box_side[b] = Lb
        c.G, c.a0, c.npre, c.npost = self.G, self.a0, self.npre, self.npost
        c.ncycle_fmg, c.max_vcycles, c.tol_rel = self.ncycle_fmg, self.max_vcycles, self.tol_rel
        c.precision, c.outer_bc, c.gather_frac = self.precision, self.outer_bc, self.gather_frac
        c.fixed_shift, c.use_graphs = self.fixed_shift, self.use_graphs
        c.nu_n = float(self.nu_n)
        return c


def validate_config(cfg: Config) -> int:
    c = cfg.to_c()
    return lib().qumond_validate_config(ctypes.byref(c))


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 device tensor")
    return t


def current_stream_handle() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _order_in(stream):
    """The library works on `stream`: order it after the caller's current
    stream, where the inputs (and the output tensors' memory) were last used."""
    cur = torch.cuda.current_stream()
    if cur != stream:
        stream.wait_stream(cur)


def _order_out(stream):
    """Order the caller's current stream after `stream`, where the library
    wrote its outputs."""
    cur = torch.cuda.current_stream()
    if cur != stream:
        cur.wait_stream(stream)


class Context:
    """One solver context: the nested-box grids on the current device, bound to a stream."""

    def __init__(self, cfg: Config, stream: Optional[torch.cuda.Stream] = None):
        self.cfg = cfg
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._c = cfg.to_c()
        h = ctypes.c_void_p()
        check(lib().qumond_create(ctypes.byref(self._c), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "qumond_create")
        self._h = h
        self.n = cfg.n
        self.nbox = len(cfg.box_side)

    def close(self):
        if getattr(self, "_h", None):
            lib().qumond_destroy(self._h)
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

    @property
    def device_bytes(self) -> int:
        return int(lib().qumond_device_bytes(self._h))

    def deposit(self, x, y, z, m, total_mass: float, count_outside: bool = True):
        """Step 1.  total_mass (Msun) is the mass of all particles, also those
        outside every box: the caller states it (it sets the monopole boundary
        value and the fixed-point scale)."""
        np_ = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (m, "m")):
            _f64(t, nm)
            if t.numel() != np_:
                raise ValueError("particle arrays differ in length")
        out = ctypes.c_int64(0)
        _order_in(self.stream)
        check(lib().qumond_deposit(self._h, _ptr(x), _ptr(y), _ptr(z), _ptr(m), np_, float(total_mass),
                                   ctypes.byref(out) if count_outside else None), "qumond_deposit")
        return int(out.value) if count_outside else None

    def solve_newton(self, allow_not_converged: bool = False) -> dict:
        info = qumond_solve_info()
        check(lib().qumond_solve_newton(self._h, ctypes.byref(info)), "qumond_solve_newton",
              allow=(QUMOND_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return info.as_dict()

    def mond_source(self):
        check(lib().qumond_mond_source(self._h), "qumond_mond_source")

    def solve_mond(self, guess: Optional[torch.Tensor] = None, allow_not_converged: bool = False,
                   no_fallback: bool = False) -> dict:
        info = qumond_solve_info()
        kind = GUESS_NONE
        if guess is not None:
            kind = {torch.float64: GUESS_F64, torch.float32: GUESS_F32, torch.bfloat16: GUESS_BF16}[guess.dtype]
            if guess.numel() != self.nbox * self.n ** 3:
                raise ValueError("guess must hold nbox * n^3 values")
            if no_fallback:
                kind |= GUESS_NO_FALLBACK
            _order_in(self.stream)
        check(lib().qumond_solve_mond(self._h, _ptr(guess), kind, ctypes.byref(info)), "qumond_solve_mond",
              allow=(QUMOND_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return info.as_dict()

    def solve(self, allow_not_converged: bool = False):
        """Steps 2-4 with the Newtonian and QUMOND chains overlapped on two streams."""
        a, b = qumond_solve_info(), qumond_solve_info()
        check(lib().qumond_solve(self._h, ctypes.byref(a), ctypes.byref(b)), "qumond_solve",
              allow=(QUMOND_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return a.as_dict(), b.as_dict()

    def gather_forces(self, x, y, z, which: int = 1, with_box: bool = True):
        np_ = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z")):
            _f64(t, nm)
        ax = torch.empty_like(x)
        ay = torch.empty_like(x)
        az = torch.empty_like(x)
        used = torch.empty(np_, dtype=torch.uint8, device=x.device) if with_box else None
        _order_in(self.stream)
        check(lib().qumond_gather_forces(self._h, _ptr(x), _ptr(y), _ptr(z), np_, int(which), _ptr(ax), _ptr(ay),
                                         _ptr(az), _ptr(used)), "qumond_gather_forces")
        _order_out(self.stream)
        return ax, ay, az, used

    def rotation_curve(self, R: torch.Tensor, naz: int = 16, which: int = 1) -> torch.Tensor:
        _f64(R, "R")
        vc2 = torch.empty_like(R)
        _order_in(self.stream)
        check(lib().qumond_rotation_curve(self._h, _ptr(R), R.numel(), int(naz), int(which), _ptr(vc2)),
              "qumond_rotation_curve")
        _order_out(self.stream)
        return vc2

    def sigma_z(self, R: torch.Tensor, z: float, z0: float, naz: int = 16, which: int = 1) -> torch.Tensor:
        """Eq. 5: sigma_z^2 (km/s)^2 at the radii R for a sech^2(z/z0) stellar
        disk, from the vertical acceleration at heights +-z."""
        _f64(R, "R")
        s2 = torch.empty_like(R)
        _order_in(self.stream)
        check(lib().qumond_sigma_z(self._h, _ptr(R), R.numel(), int(naz), float(z), float(z0), int(which),
                                   _ptr(s2)), "qumond_sigma_z")
        _order_out(self.stream)
        return s2

    def get_field(self, box: int, fld: int) -> torch.Tensor:
        dt = torch.int64 if fld == FIELD_RHO_FIXED else torch.float64
        out = torch.empty((self.n,) * 3, dtype=dt, device="cuda")
        _order_in(self.stream)
        check(lib().qumond_get_field(self._h, int(box), int(fld), _ptr(out)), "qumond_get_field")
        _order_out(self.stream)
        return out

    def profile_enable(self, on: bool = True, level_n: int = 0):
        """Time smoother launches with hipEvents: all levels, or with level_n
        only the levels of level_n points per side."""
        v = 0 if not on else (int(level_n) if level_n else 1)
        check(lib().qumond_profile_enable(self._h, v), "qumond_profile_enable")

    def profile_read(self) -> dict:
        st = qumond_kernel_stats()
        check(lib().qumond_profile_read(self._h, ctypes.byref(st)), "qumond_profile_read")
        return {"launches": int(st.launches), "total_ms": float(st.total_ms), "alg_bytes": float(st.alg_bytes),
                "sweeps_per_launch": int(st.sweeps_per_launch)}

    def set_field(self, box: int, fld: int, src: torch.Tensor):
        _f64(src, "src")
        if src.numel() != self.n ** 3:
            raise ValueError("field must hold n^3 values")
        _order_in(self.stream)
        check(lib().qumond_set_field(self._h, int(box), int(fld), _ptr(src)), "qumond_set_field")


# ----------------------------------------------------- single-grid entries

def _s(stream=None):
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def k_rbgs_sweep_from_zero(f, u_out, h):
    n = u_out.shape[0]
    check(lib().qumond_k_rbgs_sweep_from_zero(n, float(h), _ptr(f), _ptr(u_out), _s()),
          "qumond_k_rbgs_sweep_from_zero")


def k_rbgs_sweep(f, u_in, u_out, h):
    n = u_in.shape[0]
    check(lib().qumond_k_rbgs_sweep(n, float(h), _ptr(f), _ptr(u_in), _ptr(u_out), _s()), "qumond_k_rbgs_sweep")


def k_rbgs_double_sweep(f, u_in, u_out, h, uc=None):
    """Two sweeps u_in -> u_out in one launch; u_in None = a zero iterate."""
    check(lib().qumond_k_rbgs_double_sweep(u_out.shape[0], float(h), _ptr(f), _ptr(u_in), _ptr(u_out), _ptr(uc), _s()),
          "qumond_k_rbgs_double_sweep")


def k_residual_restrict(f, u, h, fc, uc0, uc1=None):
    check(lib().qumond_k_residual_restrict(u.shape[0], float(h), _ptr(f), _ptr(u), _ptr(fc), _ptr(uc0), _ptr(uc1),
                                           _s()), "qumond_k_residual_restrict")


def k_rbgs_sweep_restrict(f, u_in, u_out, h, fc, uc0, uc1=None):
    """One sweep u_in -> u_out fused with the residual restriction of u_out."""
    check(lib().qumond_k_rbgs_sweep_restrict(u_out.shape[0], float(h), _ptr(f), _ptr(u_in), _ptr(u_out), _ptr(fc),
                                             _ptr(uc0), _ptr(uc1), _s()), "qumond_k_rbgs_sweep_restrict")


def k_restrict(src, dst):
    check(lib().qumond_k_restrict(src.shape[0], _ptr(src), _ptr(dst), _s()), "qumond_k_restrict")


def k_prolong_add(uc, uf):
    check(lib().qumond_k_prolong_add(uc.shape[0], _ptr(uc), _ptr(uf), _s()), "qumond_k_prolong_add")


def k_interp(uc, uf):
    check(lib().qumond_k_interp(uc.shape[0], _ptr(uc), _ptr(uf), _s()), "qumond_k_interp")


def k_mond_source(phin, h, a0, S):
    check(lib().qumond_k_mond_source(phin.shape[0], float(h), float(a0), _ptr(phin), _ptr(S), _s()),
          "qumond_k_mond_source")


def k_bc_from_coarse(uc, uf):
    check(lib().qumond_k_bc_from_coarse(uc.shape[0], _ptr(uc), _ptr(uf), _s()), "qumond_k_bc_from_coarse")


def k_resid_norms(f, u, h, out2):
    check(lib().qumond_k_resid_norms(u.shape[0], float(h), _ptr(f), _ptr(u), _ptr(out2), _s()),
          "qumond_k_resid_norms")


def k_resid_norms_noalloc(f, u, h, out3):
    """k_resid_norms without allocating: partial sums in the library's fixed
    per-device workspace (calls overlapping on one device race)."""
    check(lib().qumond_k_resid_norms_noalloc(u.shape[0], float(h), _ptr(f), _ptr(u), _ptr(out3), _s()),
          "qumond_k_resid_norms_noalloc")


def k_fmg(f, u, L, npre=2, npost=2, ncycle=6, max_extra=50, tol=1e-10):
    rr = ctypes.c_double(0)
    ex = ctypes.c_int32(0)
    check(lib().qumond_k_fmg(u.shape[0], float(L), _ptr(f), _ptr(u), npre, npost, ncycle, max_extra, float(tol),
                             ctypes.byref(rr), ctypes.byref(ex), _s()), "qumond_k_fmg")
    return float(rr.value), int(ex.value)


def k_vcycles(f, u, L, ncyc, npre=2, npost=2):
    rr = ctypes.c_double(0)
    check(lib().qumond_k_vcycles(u.shape[0], float(L), _ptr(f), _ptr(u), npre, npost, ncyc, ctypes.byref(rr), _s()),
          "qumond_k_vcycles")
    return float(rr.value)


# ------------------------------------------------------------------ tuning

SMOOTHER_VARIANTS = {0: (32, 8), 1: (64, 4), 2: (64, 8), 3: (128, 4), 4: (32, 16), 5: "brick8",
                     6: "pairs64x8", 7: "pairs64x16", 8: "pairs128x8", 9: "brick4", 10: "brick6",
                     11: "pairs32x16", 12: "pairs32x8", 13: "pairs64x16_deep", 14: "pairs128x8_deep",
                     15: "pairs64x32_deep"}
FUSED_VARIANTS = {0: (32, 8), 1: (64, 4), 2: "brick8", 3: "brick4", 4: "brick6", 5: "pairs64x16_deep",
                  6: "pairs64x8_deep", 7: "pairs32x16_deep", 8: "skew64x16", 9: "skew32x8"}


def tune_set(n, variant, kchunk, fp32=False):
    check(lib().qumond_tune_set(int(n), int(bool(fp32)), int(variant), int(kchunk)), "qumond_tune_set")


def tune_get(n, fp32=False):
    v, k = ctypes.c_int32(0), ctypes.c_int32(0)
    check(lib().qumond_tune_get(int(n), int(bool(fp32)), ctypes.byref(v), ctypes.byref(k)), "qumond_tune_get")
    return int(v.value), int(k.value)


def tune_set_corr(n, variant, kchunk, fp32=False):
    """Shape of the single sweep that applies the coarse-grid correction
    (variant -1: the level's plain-sweep shape)."""
    check(lib().qumond_tune_set_corr(int(n), int(bool(fp32)), int(variant), int(kchunk)), "qumond_tune_set_corr")


def tune_get_corr(n, fp32=False):
    v, k = ctypes.c_int32(0), ctypes.c_int32(0)
    check(lib().qumond_tune_get_corr(int(n), int(bool(fp32)), ctypes.byref(v), ctypes.byref(k)), "qumond_tune_get_corr")
    return int(v.value), int(k.value)


def tune_set_sweep_restrict(n, fused, fp32=False):
    """1: the last pre-smoothing sweep of level n runs fused with its residual
    restriction; 0: two launches."""
    check(lib().qumond_tune_set_sweep_restrict(int(n), int(bool(fp32)), int(fused)), "qumond_tune_set_sweep_restrict")


def tune_get_sweep_restrict(n, fp32=False):
    v = ctypes.c_int32(0)
    check(lib().qumond_tune_get_sweep_restrict(int(n), int(bool(fp32)), ctypes.byref(v)),
          "qumond_tune_get_sweep_restrict")
    return int(v.value)


def tune_set_fused(n, variant, kchunk, fp32=False):
    check(lib().qumond_tune_set_fused(int(n), int(bool(fp32)), int(variant), int(kchunk)), "qumond_tune_set_fused")


def tune_get_fused(n, fp32=False):
    v, k = ctypes.c_int32(0), ctypes.c_int32(0)
    check(lib().qumond_tune_get_fused(int(n), int(bool(fp32)), ctypes.byref(v), ctypes.byref(k)),
          "qumond_tune_get_fused")
    return int(v.value), int(k.value)


def k_rbgs_sweep_shape(f, u_in, u_out, h, variant, kchunk, uc=None):
    check(lib().qumond_k_rbgs_sweep_shape(u_out.shape[0], float(h), _ptr(f), _ptr(u_in), _ptr(u_out), int(variant),
                                          int(kchunk), _ptr(uc), _s()), "qumond_k_rbgs_sweep_shape")


def k_rbgs_sweep_stacked(f, u_in, u_out, h, variant, kchunk):
    """One sweep of the nb problems of u_out ([nb, n, n, n]) in one launch;
    u_in None = zero iterates."""
    nb, n = u_out.shape[0], u_out.shape[1]
    check(lib().qumond_k_rbgs_sweep_stacked(n, nb, float(h), _ptr(f), _ptr(u_in), _ptr(u_out), int(variant),
                                            int(kchunk), _s()), "qumond_k_rbgs_sweep_stacked")


def autotune(n_max=513, both=True, reps=5, json_path=None):
    best = (ctypes.c_double * 11)()
    check(lib().qumond_autotune(int(n_max), int(bool(both)), int(reps), json_path.encode() if json_path else None,
                                best, _s()), "qumond_autotune")
    return {(1 << J) + 1: best[J] for J in range(5, 11) if best[J] > 0}


def tune_set_rr(n, variant, fp32=False):
    check(lib().qumond_tune_set_rr(int(n), int(bool(fp32)), int(variant)), "qumond_tune_set_rr")


def tune_get_rr(n, fp32=False):
    v = ctypes.c_int32()
    check(lib().qumond_tune_get_rr(int(n), int(bool(fp32)), ctypes.byref(v)), "qumond_tune_get_rr")
    return v.value


def tune_set_split(n, split, fp32=False):
    check(lib().qumond_tune_set_split(int(n), int(bool(fp32)), int(split)), "qumond_tune_set_split")


def tune_get_split(n, fp32=False):
    v = ctypes.c_int32()
    check(lib().qumond_tune_get_split(int(n), int(bool(fp32)), ctypes.byref(v)), "qumond_tune_get_split")
    return v.value


def tune_load(json_path):
    check(lib().qumond_tune_load(json_path.encode()), "qumond_tune_load")


# ------------------------------------------------------------------ U-Net

class UNet:
    """The learned initial guess (include/qumond_unet.h): BF16 MFMA 3D U-Net."""

    def __init__(self, n: int = 129, seed: int = 1201, stream: Optional[torch.cuda.Stream] = None):
        self.n = n
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check(lib().qumond_unet_create(int(n), ctypes.c_uint64(seed), ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(h)), "qumond_unet_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().qumond_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def param_count(self) -> int:
        return int(lib().qumond_unet_param_count(self._h))

    def get_params(self):
        import numpy as np
        out = np.zeros(self.param_count, dtype=np.float32)
        check(lib().qumond_unet_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p)), "qumond_unet_get_params")
        return out

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.param_count:
            raise ValueError("parameter count mismatch")
        check(lib().qumond_unet_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)), "qumond_unet_set_params")

    def get_grads(self):
        import numpy as np
        out = np.zeros(self.param_count, dtype=np.float32)
        check(lib().qumond_unet_get_grads(self._h, out.ctypes.data_as(ctypes.c_void_p)), "qumond_unet_get_grads")
        return out

    def prepare_sample(self, phin, S, phi, h, c_phin, c_out, x=None, t=None, GM=0.0, a0=3600.0, soft=1.0):
        N = self.n ** 3
        x = torch.empty(N * 2, dtype=torch.bfloat16, device="cuda") if x is None else x
        t = torch.empty(N, dtype=torch.float32, device="cuda") if t is None else t
        _order_in(self.stream)
        check(lib().qumond_unet_prepare_sample(self._h, _ptr(phin), _ptr(S), _ptr(phi), float(h), float(c_phin),
                                               float(c_out), float(GM), float(a0), float(soft), _ptr(x), _ptr(t)),
              "qumond_unet_prepare_sample")
        _order_out(self.stream)
        return x, t

    def train_step(self, x, target, lr: float = 1e-3, want_loss: bool = True):
        loss = ctypes.c_double(0.0)
        _order_in(self.stream)
        check(lib().qumond_unet_train_step(self._h, _ptr(x), _ptr(target), ctypes.c_float(lr),
                                           ctypes.byref(loss) if want_loss else None), "qumond_unet_train_step")
        return float(loss.value) if want_loss else None

    def infer(self, phin, S, h, c_phin, c_out, out: Optional[torch.Tensor] = None, GM=0.0, a0=3600.0, soft=1.0):
        if out is None:
            out = torch.empty(self.n ** 3, dtype=torch.float64, device="cuda")
        _order_in(self.stream)
        check(lib().qumond_unet_infer(self._h, _ptr(phin), _ptr(S), float(h), float(c_phin), float(c_out),
                                      float(GM), float(a0), float(soft), _ptr(out)), "qumond_unet_infer")
        _order_out(self.stream)
        return out


def k_conv3d_fwd(x, n_in, cin, w, cout, bias=None, stride=1, relu=False):
    n_out = (n_in + 1) // 2 if stride == 2 else n_in
    y = torch.empty(n_out ** 3 * cout, dtype=torch.bfloat16, device="cuda")
    check(lib().qumond_k_conv3d_fwd(n_in, cin, _ptr(x), cout, _ptr(w), _ptr(bias), stride, int(relu), _ptr(y), _s()),
          "qumond_k_conv3d_fwd")
    return y


def k_conv3d_dgrad(n_in, cin, cout, w, dy, stride=1):
    dx = torch.empty(n_in ** 3 * cin, dtype=torch.bfloat16, device="cuda")
    check(lib().qumond_k_conv3d_dgrad(n_in, cin, cout, _ptr(w), stride, _ptr(dy), _ptr(dx), _s()),
          "qumond_k_conv3d_dgrad")
    return dx


def k_conv3d_wgrad(n_in, cin, x, cout, dy, stride=1):
    kpad = (27 * cin + 31) // 32 * 32
    dw = torch.empty(cout * kpad, dtype=torch.float32, device="cuda")
    check(lib().qumond_k_conv3d_wgrad(n_in, cin, _ptr(x), cout, _ptr(dy), stride, _ptr(dw), _s()),
          "qumond_k_conv3d_wgrad")
    return dw


# ------------------------------------------------------------- batches

@dataclass
class BatchConfig:
    """Mirror of qumond_batch_config (defaults from qumond_batch_default_config)."""
    box_side: float = 120.0
    G: float = 4.300917270e-6
    a0: float = 3600.0
    npre: int = 2
    npost: int = 2
    ncycle_fmg: int = 2
    refine_iters: int = 4
    max_extra: int = 20
    tol_rel: float = 1e-6
    gather_frac: float = 0.2
    naz: int = 16
    autotune: bool = False
    nu_n: float = 1.0

    def to_c(self, nprob: int) -> qumond_batch_config:
        c = qumond_batch_config()
        lib().qumond_batch_default_config(ctypes.byref(c))
        c.nprob = int(nprob)
        for k in ("box_side", "G", "a0", "tol_rel", "gather_frac"):
            setattr(c, k, float(getattr(self, k)))
        for k in ("npre", "npost", "ncycle_fmg", "refine_iters", "max_extra", "naz"):
            setattr(c, k, int(getattr(self, k)))
        c.autotune = int(bool(self.autotune))
        c.nu_n = float(self.nu_n)
        return c


def batch_validate(cfg: BatchConfig, n_per_problem, R) -> int:
    ns = (ctypes.c_int32 * len(n_per_problem))(*[int(v) for v in n_per_problem])
    rr = (ctypes.c_double * max(1, len(R)))(*[float(v) for v in R])
    c = cfg.to_c(len(n_per_problem))
    return int(lib().qumond_batch_validate(ctypes.byref(c), ns, rr if len(R) else None, len(R)))


class Batch:
    """Many single-box disks solved together (include/qumond_batch.h)."""

    def __init__(self, cfg: BatchConfig, n_per_problem, R, stream: Optional[torch.cuda.Stream] = None):
        self.cfg = cfg
        self.n_of = [int(v) for v in n_per_problem]
        self.nprob = len(self.n_of)
        self.R = [float(v) for v in R]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ns = (ctypes.c_int32 * self.nprob)(*self.n_of)
        rr = (ctypes.c_double * len(self.R))(*self.R)
        self._c = cfg.to_c(self.nprob)
        h = ctypes.c_void_p()
        check(lib().qumond_batch_create(ctypes.byref(self._c), ns, rr, len(self.R),
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
              "qumond_batch_create")
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().qumond_batch_destroy(self._h)
            self._h = None
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def device_bytes(self) -> int:
        return int(lib().qumond_batch_device_bytes(self._h))

    def set_particles(self, p: int, x, y, z, m, total_mass: float):
        """Particles of problem p; total_mass (Msun, > 0) as for deposit."""
        np_ = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (m, "m")):
            _f64(t, nm)
            if t.numel() != np_:
                raise ValueError("particle arrays differ in length")
        check(lib().qumond_batch_set_particles(self._h, int(p), _ptr(x), _ptr(y), _ptr(z), _ptr(m), np_,
                                               float(total_mass)), "qumond_batch_set_particles")
        self._keep[int(p)] = (x, y, z, m)   # the batch reads them at every run

    def run(self, use_graph: bool = True, allow_not_converged: bool = False) -> List[dict]:
        info = (qumond_batch_problem_info * self.nprob)()
        _order_in(self.stream)          # particles written on the caller's stream
        check(lib().qumond_batch_run(self._h, int(bool(use_graph)), info), "qumond_batch_run",
              allow=(QUMOND_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return [{k: getattr(i, k) for k, _ in qumond_batch_problem_info._fields_} for i in info]

    def rotation_curves(self, mond: bool = True) -> torch.Tensor:
        out = torch.empty((self.nprob, len(self.R)), dtype=torch.float64, device="cuda")
        _order_in(self.stream)
        check(lib().qumond_batch_rotation_curves(self._h, int(bool(mond)), _ptr(out)), "qumond_batch_rotation_curves")
        _order_out(self.stream)
        return out

    def get_field(self, p: int, fld: int) -> torch.Tensor:
        n = self.n_of[p]
        out = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
        _order_in(self.stream)
        check(lib().qumond_batch_get_field(self._h, int(p), int(fld), _ptr(out)), "qumond_batch_get_field")
        _order_out(self.stream)
        return out

    def describe(self) -> dict:
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        check(lib().qumond_batch_describe(self._h, buf, len(buf)), "qumond_batch_describe")
        return json.loads(buf.value.decode())
