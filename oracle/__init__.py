"""CPU oracle for the particle-mesh QUMOND solve (Angus et al., arXiv:1201.3185, Sec. 2).

TEST INFRASTRUCTURE ONLY: the plain FP64 judge of the HIP library.  It shares no
code with the product package and may be imported only by the test suite, the
smoke check and the benchmark's CPU-baseline leg.

The arithmetic lives in ``qumond_oracle.c`` (``gcc -O2 -ffp-contract=off``,
one thread unless ``set_threads`` asks for more; the node-parallel loops give
the same bits at any thread count); this module builds it on demand, declares
its C signatures, and chains the steps in the order of Sec. 2:

    step 1  CIC density per box           (cic_deposit, rhs_from_q)
    step 2  Newtonian FMG, box by box     (fmg, outer BC, BC from coarser box)
    step 3  Eq. 2 source per box          (mond_source)
    step 4  QUMOND FMG, box by box        (fmg)
    then    finite-difference gravity + CIC interpolation (gather)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qumond_oracle.c")
_SRC_UNET = os.path.join(_HERE, "unet_oracle.c")
_SO = os.path.join(_HERE, "_qumond_oracle.so")

# Units: kpc, Msun, km/s.  G in kpc (km/s)^2 / Msun; a0 = 3.6 (km/s)^2/pc (Eq. 2).
G_KPC = 4.300917270e-6
A0_KPC = 3600.0


def build(force: bool = False) -> str:
    """Compile the oracle shared object with gcc (no FMA contraction)."""
    stale = not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(f) for f in (_SRC, _SRC_UNET))
    if force or stale:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
             "-D_DEFAULT_SOURCE", _SRC, _SRC_UNET, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        d, i, i64, vp = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        sig = {
            "orc_set_threads": (None, [i]),
            "orc_get_threads": (i, []),
            "orc_nu": (d, [d]),
            "orc_nu_n": (d, [d, d]),
            "orc_fixed_shift": (i, [d]),
            "orc_cic_deposit": (i64, [i, d, i64, vp, vp, vp, vp, i, vp]),
            "orc_rhs_from_q": (None, [i, d, d, i, vp, vp]),
            "orc_phi_point_newton": (d, [d, d, d]),
            "orc_phi_point_mond": (d, [d, d, d, d]),
            "orc_bc_outer": (None, [i, d, i, d, d, d, vp]),
            "orc_bc_from_coarse": (None, [i, d, vp, d, vp]),
            "orc_rbgs_colour": (None, [i, d, vp, vp, i]),
            "orc_rbgs_sweep": (None, [i, d, vp, vp]),
            "orc_residual": (None, [i, d, vp, vp, vp]),
            "orc_interior_sumsq": (d, [i, vp]),
            "orc_boundary_coupling_sumsq": (d, [i, d, vp]),
            "orc_restrict_fw": (None, [i, vp, vp]),
            "orc_prolong_add": (None, [i, vp, vp]),
            "orc_interp": (None, [i, vp, vp]),
            "orc_fmg": (i, [i, d, vp, vp, i, i, i, i, d, vp, vp]),
            "orc_vcycles": (d, [i, d, vp, vp, i, i, i]),
            "orc_mond_source": (None, [i, d, d, vp, vp]),
            "orc_mond_source_nu": (None, [i, d, d, d, vp, vp]),
            "orc_gather": (None, [i, i, vp, vp, i64, vp, vp, vp, d, d, d, d, i, vp, vp, vp, vp]),
            "orc_gather_nu": (None, [i, i, vp, vp, i64, vp, vp, vp, d, d, d, d, i, d, vp, vp, vp, vp]),
            "orc_conv3d_fwd": (None, [i, i, vp, i, vp, vp, i, i, vp]),
            "orc_conv3d_dgrad": (None, [i, i, i, vp, i, vp, vp]),
            "orc_conv3d_wgrad": (None, [i, i, vp, i, vp, i, vp]),
            "orc_upsample": (None, [i, i, vp, vp]),
            "orc_adam_step": (None, [i, vp, vp, vp, vp, d, d, d, d, i]),
            "orc_upsample_adj": (None, [i, i, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def set_threads(t: int) -> int:
    """Threads of the oracle's node-parallel loops (colour passes, residual,
    transfers, source, gather); the deposit and every sum stay serial, so the
    results do not depend on the count.  Returns the previous count."""
    prev = lib().orc_get_threads()
    lib().orc_set_threads(int(t))
    return prev


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- pointwise

def nu(y, nu_n=1.0):
    """Eq. 2 interpolating function, elementwise; nu_n != 1 selects the
    n-family member [(1 + sqrt(1 + 4 y^-n)) / 2]^(1/n) (Sec. 2 allows other
    forms of nu; n = 1 is Eq. 2's)."""
    if nu_n == 1.0:
        return np.vectorize(lib().orc_nu, otypes=[np.float64])(np.asarray(y, dtype=np.float64))
    return np.vectorize(lambda v: lib().orc_nu_n(v, float(nu_n)), otypes=[np.float64])(np.asarray(y, dtype=np.float64))


def _nu_minus_one_at(s, nu_n):
    """nu_n(1/s^2) - 1 without cancellation: with w = s^(2n),
    nu^n = 1 + q, q = 2 w / (1 + sqrt(1 + 4 w)), so nu - 1 = expm1(log1p(q) / n)."""
    w = s ** (2.0 * nu_n)
    q = 2.0 * w / (1.0 + math.sqrt(1.0 + 4.0 * w))
    return math.expm1(math.log1p(q) / nu_n)


def point_mond_integral(t, nu_n):
    """I(t) = int_0^t (nu_n(1/s^2) - 1) / s^2 ds (scipy quad on geometric
    pieces), the dimensionless part of the point-mass QUMOND potential."""
    from scipy import integrate
    f = lambda s: _nu_minus_one_at(s, nu_n) / (s * s) if s > 0.0 else (1.0 if nu_n == 1.0 else 0.0)
    edges = [0.0] + [e for e in (1e-3 * 4.0 ** k for k in range(40)) if e < t] + [t]
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        val, _ = integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-13, limit=200)
        total += val
    return total


def phi_point_mond_family(r, G=G_KPC, M=1.0, a0=A0_KPC, nu_n=1.0):
    """Point-mass QUMOND potential for the n-family: the radial integral of
    nu_n(g_N/a0) g_N fixed to tend to -GM/r at small r, i.e.
    -GM/r + sqrt(G M a0) I(r / r_M), r_M = sqrt(G M / a0)."""
    GM = G * M
    r = np.asarray(r, dtype=np.float64)
    if a0 <= 0.0 or GM <= 0.0:
        return -GM / r
    rm = math.sqrt(GM / a0)
    out = np.array([-GM / rr + math.sqrt(GM * a0) * point_mond_integral(rr / rm, nu_n) for rr in r.ravel()])
    return out.reshape(r.shape)


def fixed_shift(total_mass: float) -> int:
    return int(lib().orc_fixed_shift(float(total_mass)))


def phi_point_newton(r, G=G_KPC, M=1.0):
    return np.vectorize(lambda rr: lib().orc_phi_point_newton(rr, G, M), otypes=[np.float64])(r)


def phi_point_mond(r, G=G_KPC, M=1.0, a0=A0_KPC):
    return np.vectorize(lambda rr: lib().orc_phi_point_mond(rr, G, M, a0), otypes=[np.float64])(r)


# ----------------------------------------------------------------- per box

def cic_deposit(n, L, x, y, z, m, shift):
    """Step 1 in fixed point: int64 grid [n,n,n] (z,y,x order) and the count inside."""
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    q = np.zeros((n, n, n), dtype=np.int64)
    inside = lib().orc_cic_deposit(n, float(L), len(x), _p(x), _p(y), _p(z), _p(m), int(shift), _p(q))
    return q, int(inside)


def rhs_from_q(n, L, q, shift, G=G_KPC):
    f = np.zeros((n, n, n))
    q = np.ascontiguousarray(q, dtype=np.int64)
    lib().orc_rhs_from_q(n, float(L), float(G), int(shift), _p(q), _p(f))
    return f


def bc_outer(u, L, mode, G=G_KPC, a0=A0_KPC, M=0.0, nu_n=1.0):
    """mode 0 zero, 1 Newtonian monopole, 2 QUMOND monopole (boundary nodes only).
    For nu_n != 1 the QUMOND monopole is the quadrature of phi_point_mond_family,
    once per distinct radius."""
    n = u.shape[0]
    if mode != 2 or nu_n == 1.0:
        lib().orc_bc_outer(n, float(L), int(mode), float(G), float(a0), float(M), _p(u))
        return u
    h = L / (n - 1)
    c = -0.5 * L + h * np.arange(n)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    bnd = np.zeros((n, n, n), dtype=bool)
    bnd[0], bnd[-1], bnd[:, 0], bnd[:, -1], bnd[:, :, 0], bnd[:, :, -1] = (True,) * 6
    r = np.sqrt(X[bnd] ** 2 + Y[bnd] ** 2 + Z[bnd] ** 2)
    ru, inv = np.unique(r, return_inverse=True)
    u[bnd] = phi_point_mond_family(ru, G, M, a0, nu_n)[inv]
    return u


def bc_from_coarse(uc, Lc, uf, Lf):
    n = uc.shape[0]
    uc = _f64(uc)
    lib().orc_bc_from_coarse(n, float(Lc), _p(uc), float(Lf), _p(uf))
    return uf


def rbgs_colour(f, u, h, colour):
    lib().orc_rbgs_colour(u.shape[0], float(h), _p(_f64(f)), _p(u), int(colour))
    return u


def rbgs_sweep(f, u, h):
    lib().orc_rbgs_sweep(u.shape[0], float(h), _p(_f64(f)), _p(u))
    return u


def residual(f, u, h):
    r = np.zeros_like(u)
    lib().orc_residual(u.shape[0], float(h), _p(_f64(f)), _p(_f64(u)), _p(r))
    return r


def restrict_fw(rf):
    nc = (rf.shape[0] + 1) // 2
    fc = np.zeros((nc, nc, nc))
    lib().orc_restrict_fw(rf.shape[0], _p(_f64(rf)), _p(fc))
    return fc


def prolong_add(uc, uf):
    lib().orc_prolong_add(uc.shape[0], _p(_f64(uc)), _p(uf))
    return uf


def interp(uc, uf):
    lib().orc_interp(uc.shape[0], _p(_f64(uc)), _p(uf))
    return uf


def fmg(f, u, L, npre=2, npost=2, ncycle=6, max_extra=50, tol=1e-10):
    """FMG in place on u (boundary = Dirichlet values). Returns (status, relres, extra)."""
    f = _f64(f)
    rr = ctypes.c_double(0.0)
    ex = ctypes.c_int(0)
    st = lib().orc_fmg(u.shape[0], float(L), _p(f), _p(u), npre, npost, ncycle, max_extra,
                       float(tol), ctypes.byref(rr), ctypes.byref(ex))
    return int(st), float(rr.value), int(ex.value)


def vcycles(f, u, L, ncyc, npre=2, npost=2):
    return float(lib().orc_vcycles(u.shape[0], float(L), _p(_f64(f)), _p(u), npre, npost, ncyc))


def mond_source(phin, L, a0=A0_KPC, nu_n=1.0):
    phin = _f64(phin)
    S = np.zeros_like(phin)
    lib().orc_mond_source_nu(phin.shape[0], float(L), float(a0), float(nu_n), _p(phin), _p(S))
    return S


def gather(phis, Ls, x, y, z, frac=0.2, G=G_KPC, a0=A0_KPC, M=0.0, mond=True, nu_n=1.0):
    """Accelerations (ax, ay, az) and the box index used (255 = monopole)."""
    n = phis[0].shape[0]
    nbox = len(phis)
    phis = [_f64(p) for p in phis]
    ptrs = (ctypes.c_void_p * nbox)(*[p.ctypes.data for p in phis])
    Ls_a = _f64(Ls)
    x, y, z = _f64(x), _f64(y), _f64(z)
    np_ = len(x)
    ax, ay, az = np.zeros(np_), np.zeros(np_), np.zeros(np_)
    used = np.zeros(np_, dtype=np.uint8)
    lib().orc_gather_nu(nbox, n, _p(Ls_a), ctypes.cast(ptrs, ctypes.c_void_p), np_, _p(x), _p(y), _p(z),
                        float(frac), float(G), float(a0), float(M), int(bool(mond)), float(nu_n),
                        _p(ax), _p(ay), _p(az), _p(used))
    return ax, ay, az, used


def rotation_curve_points(R, naz=16):
    """Midplane sample points: naz azimuths per radius, phi_k = 2 pi k / naz."""
    R = np.asarray(R, dtype=np.float64)
    phi = 2.0 * np.pi * np.arange(naz) / naz
    x = (R[:, None] * np.cos(phi)[None, :]).ravel()
    y = (R[:, None] * np.sin(phi)[None, :]).ravel()
    return x, y, np.zeros_like(x)


def vc2_from_acc(x, y, ax, ay, nR, naz=16):
    """Eq. 4: v_c^2 = R dPhi/dR = -(x a_x + y a_y), averaged over the azimuths."""
    return (-(x * ax + y * ay)).reshape(nR, naz).mean(axis=1)


# ------------------------------------------------------------ diagnostics

def algebraic_field(ax, ay, az, a0=A0_KPC, nu_n=1.0):
    """Eq. 3, the algebraic MOND relation: g = nu(|g_N| / a0) g_N, point by
    point, from Newtonian accelerations (g_N = 0 stays 0)."""
    ax, ay, az = _f64(ax), _f64(ay), _f64(az)
    if a0 <= 0.0:                      # nu -> 1: the Newtonian field
        return ax.copy(), ay.copy(), az.copy()
    g = np.sqrt(ax * ax + ay * ay + az * az)
    k = np.zeros_like(g)
    pos = g > 0.0
    k[pos] = nu(g[pos] / a0, nu_n)
    return k * ax, k * ay, k * az


def sigma_z_points(R, z, naz=16):
    """Sample points of the Eq. 5 diagnostic: for each radius, naz azimuths
    phi_k = 2 pi k / naz at height +z, then the same azimuths at -z."""
    R = np.asarray(R, dtype=np.float64)
    phi = 2.0 * np.pi * np.arange(naz) / naz
    x = np.concatenate([R[:, None] * np.cos(phi)[None, :]] * 2, axis=1).ravel()
    y = np.concatenate([R[:, None] * np.sin(phi)[None, :]] * 2, axis=1).ravel()
    zz = np.concatenate([np.full((len(R), naz), z), np.full((len(R), naz), -z)], axis=1).ravel()
    return x, y, zz


def sigma_z2_from_az(zs, az, z0, nR, naz=16):
    """Eq. 5 for stars whose density falls off as sech^2(z / z0) at every
    radius: rho / d_z rho = -z0 / (2 tanh(z / z0)), so
    sigma_z^2 = -(d Phi / dz) rho / d_z rho = (d Phi / dz) z0 / (2 tanh(z / z0))
              = -a_z z0 / (2 tanh(z / z0)),
    averaged over the 2 naz sample points of each radius (sigma_z_points)."""
    zs, az = _f64(zs), _f64(az)
    s2 = -az * z0 / (2.0 * np.tanh(zs / z0))
    return s2.reshape(nR, 2 * naz).mean(axis=1)


# ------------------------------------------------------------ the pipeline

@dataclass
class OracleConfig:
    n: int
    box_side: list                # kpc, outermost first, each half the previous
    G: float = G_KPC
    a0: float = A0_KPC
    npre: int = 2
    npost: int = 2
    ncycle_fmg: int = 6
    max_vcycles: int = 50
    tol_rel: float = 1e-10
    outer_bc: int = 1             # 0 zero, 1 monopole
    gather_frac: float = 0.2
    fixed_shift: int = 0          # 0 = from the total mass
    nu_n: float = 1.0             # interpolating function: 1 = Eq. 2's nu, else the n-family


@dataclass
class OracleResult:
    q: list = field(default_factory=list)
    f: list = field(default_factory=list)
    phin: list = field(default_factory=list)
    S: list = field(default_factory=list)
    phi: list = field(default_factory=list)
    info_newton: list = field(default_factory=list)
    info_mond: list = field(default_factory=list)
    n_outside: int = 0
    shift: int = 0


def solve_chain(cfg: OracleConfig, rhs: list, mond: bool, M: float):
    """Steps 2 and 4: FMG box by box, the outer box from its Dirichlet value,
    every inner box from the converged solution of the next coarser one."""
    out, info = [], []
    for b, Lb in enumerate(cfg.box_side):
        u = np.zeros((cfg.n,) * 3)
        if b == 0:
            mode = 0 if cfg.outer_bc == 0 else (2 if mond else 1)
            bc_outer(u, Lb, mode, cfg.G, cfg.a0, M, cfg.nu_n)
        else:
            bc_from_coarse(out[b - 1], cfg.box_side[b - 1], u, Lb)
        st, rr, ex = fmg(rhs[b], u, Lb, cfg.npre, cfg.npost, cfg.ncycle_fmg, cfg.max_vcycles, cfg.tol_rel)
        out.append(u)
        info.append((st, rr, ex))
    return out, info


def run_pipeline(cfg: OracleConfig, x, y, z, m, total_mass: float) -> OracleResult:
    res = OracleResult()
    shift = cfg.fixed_shift if cfg.fixed_shift else fixed_shift(total_mass)
    res.shift = shift
    inside_outer = None
    for b, Lb in enumerate(cfg.box_side):
        q, inside = cic_deposit(cfg.n, Lb, x, y, z, m, shift)
        if b == 0:
            inside_outer = inside
        res.q.append(q)
        res.f.append(rhs_from_q(cfg.n, Lb, q, shift, cfg.G))
    res.n_outside = len(np.asarray(x)) - inside_outer
    res.phin, res.info_newton = solve_chain(cfg, res.f, False, total_mass)
    res.S = [mond_source(p, Lb, cfg.a0, cfg.nu_n) for p, Lb in zip(res.phin, cfg.box_side)]
    res.phi, res.info_mond = solve_chain(cfg, res.S, True, total_mass)
    return res


# ------------------------------------------------------- network layers (O2)

def conv3d_fwd(x, w, b=None, stride=1, relu=False):
    """x: [n^3, cin] channel-last, w: [cout, 27, cin]; returns [n_out^3, cout]."""
    x, w = _f64(x), _f64(w)
    cout, _, cin = w.shape
    nin = round(x.shape[0] ** (1 / 3))
    nout = (nin - 1) // stride + 1
    y = np.zeros((nout ** 3, cout))
    bb = _f64(b) if b is not None else None
    lib().orc_conv3d_fwd(nin, cin, _p(x), cout, _p(w), _p(bb) if bb is not None else None, stride, int(relu), _p(y))
    return y


def conv3d_dgrad(w, dy, nin, stride=1):
    w, dy = _f64(w), _f64(dy)
    cout, _, cin = w.shape
    dx = np.zeros((nin ** 3, cin))
    lib().orc_conv3d_dgrad(nin, cin, cout, _p(w), stride, _p(dy), _p(dx))
    return dx


def conv3d_wgrad(x, dy, cout, stride=1):
    x, dy = _f64(x), _f64(dy)
    nin = round(x.shape[0] ** (1 / 3))
    cin = x.shape[1]
    dw = np.zeros((cout, 27, cin))
    lib().orc_conv3d_wgrad(nin, cin, _p(x), cout, _p(dy), stride, _p(dw))
    return dw


def upsample(xc, nc):
    xc = _f64(xc)
    ch = xc.shape[1]
    nf = 2 * nc - 1
    xf = np.zeros((nf ** 3, ch))
    lib().orc_upsample(nc, ch, _p(xc), _p(xf))
    return xf


def upsample_adj(gf, nc):
    gf = _f64(gf)
    ch = gf.shape[1]
    gc = np.zeros((nc ** 3, ch))
    lib().orc_upsample_adj(nc, ch, _p(gf), _p(gc))
    return gc


class Adam:
    """Adam (Kingma and Ba 2015, Algorithm 1) in FP64 on a flat parameter
    vector: m and v start at zero, step t counts from 1."""

    def __init__(self, w, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.w = _f64(w).copy()
        self.m = np.zeros_like(self.w)
        self.v = np.zeros_like(self.w)
        self.lr, self.b1, self.b2, self.eps = float(lr), float(b1), float(b2), float(eps)
        self.t = 0

    def step(self, g, lr=None):
        g = _f64(g)
        assert g.shape == self.w.shape
        self.t += 1
        lib().orc_adam_step(self.w.size, _p(self.w), _p(self.m), _p(self.v), _p(g),
                            self.lr if lr is None else float(lr), self.b1, self.b2, self.eps, self.t)
        return self.w
