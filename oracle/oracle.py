"""ctypes front end of the FP64 CPU oracle (lbdem_oracle.c).

Test infrastructure: imported only by the tests, the smoke check and the CPU
baseline leg of the benchmark. It shares no code with the GPU library; it
only consumes the seeded inputs of paper_1711_00336_amd.inputs.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbdem_oracle.c")
_LIB = os.path.join(_HERE, "liblbdem_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("periodic", C.c_int32 * 3),
                ("tau", C.c_double), ("rho_f", C.c_double),
                ("g", C.c_double * 3), ("fb", C.c_double * 3),
                ("e_n", C.c_double), ("mu_c", C.c_double), ("T_c", C.c_double),
                ("h_c", C.c_double), ("h_min", C.c_double),
                ("lub_stab", C.c_int32), ("use_lub", C.c_int32), ("use_am", C.c_int32),
                ("n_int", C.c_int32), ("n_dem", C.c_int32),
                ("c_am", C.c_double), ("use_lift", C.c_int32),
                ("use_eilers", C.c_int32), ("use_les", C.c_int32), ("lub_contact", C.c_int32)]


class State(C.Structure):
    _fields_ = [("df", C.c_void_p), ("uprev", C.c_void_p), ("step", C.c_int64),
                ("np", C.c_int64), ("x", C.c_void_p), ("u", C.c_void_p),
                ("w", C.c_void_p), ("a", C.c_void_p), ("d", C.c_void_p),
                ("rho_p", C.c_void_p)]


class Aux(C.Structure):
    _fields_ = [("f_acc", C.c_void_p), ("eps_f", C.c_void_p), ("dudt", C.c_void_p),
                ("gradp", C.c_void_p), ("rho", C.c_void_p), ("j", C.c_void_p),
                ("F_am", C.c_void_p), ("F_d", C.c_void_p), ("F_pr", C.c_void_p),
                ("F_const", C.c_void_p),
                ("impulse_pr", C.c_double * 3), ("impulse_gb", C.c_double * 3),
                ("impulse_fb", C.c_double * 3), ("min_eps_f", C.c_double),
                ("status", C.c_int32), ("F_l", C.c_void_p), ("curl", C.c_void_p)]


class Diag(C.Structure):
    _fields_ = [("mass_dev", C.c_double), ("mom_fluid", C.c_double * 3),
                ("mom_part", C.c_double * 3), ("u_ps", C.c_double),
                ("mean_eps_f", C.c_double), ("min_eps_f", C.c_double),
                ("max_u", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _load(_LIB)
    return _lib


def build_variant(src_text: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source (the tests plant known
    mistakes in it to show that the pins catch them)."""
    src_path = out_path + ".c"
    with open(src_path, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(["gcc", "-std=gnu11", "-O1", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                           "-w", "-o", out_path, src_path, "-lm"])
    return out_path


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


@contextlib.contextmanager
def using_library(path: str):
    """Route every call of this module through another build of the oracle
    (a variant from build_variant) inside the block."""
    global _lib
    saved = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def _load(path):
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    L.orc_roma.restype = C.c_double
    L.orc_roma.argtypes = [C.c_double]
    L.orc_axis_stencil.restype = C.c_int
    L.orc_axis_stencil.argtypes = [C.c_double, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    L.orc_drag_factor.restype = C.c_double
    L.orc_drag_factor.argtypes = [C.c_double, C.c_double]
    L.orc_drag.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_void_p]
    L.orc_lift.argtypes = [C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_curl_field.argtypes = [C.POINTER(Params), C.c_void_p, C.c_void_p]
    L.orc_tau_e.restype = C.c_double
    L.orc_tau_e.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_void_p, C.c_void_p]
    L.orc_feq_dev.argtypes = [C.c_double, C.c_void_p, C.c_double, C.c_void_p]
    L.orc_guo.argtypes = [C.c_void_p, C.c_double, C.c_void_p, C.c_double, C.c_void_p]
    L.orc_moments.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_collision_params.argtypes = [C.c_double] * 3 + [C.c_void_p, C.c_void_p]
    L.orc_lub_coeffs.argtypes = [C.c_double] * 3 + [C.c_void_p, C.c_void_p]
    L.orc_lbm_collide_stream.argtypes = [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_eps_field.argtypes = [C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_interp_scalar.restype = C.c_double
    L.orc_interp_scalar.argtypes = [C.POINTER(Params), C.c_void_p, C.c_void_p]
    L.orc_spread_scalar.argtypes = [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_double]
    L.orc_pair_force.argtypes = ([C.POINTER(Params)] + [C.c_void_p] * 3 + [C.c_double, C.c_double]
                                 + [C.c_void_p] * 3 + [C.c_double, C.c_double] + [C.c_double, C.c_void_p, C.c_void_p])
    L.orc_wall_force.argtypes = ([C.POINTER(Params)] + [C.c_void_p] * 3 + [C.c_double, C.c_double]
                                 + [C.c_double, C.c_void_p, C.c_void_p])
    L.orc_dem_forces.argtypes = ([C.POINTER(Params), C.c_int64] + [C.c_void_p] * 5
                                 + [C.c_double, C.c_void_p, C.c_void_p])
    L.orc_step.restype = C.c_int
    L.orc_step.argtypes = [C.POINTER(Params), C.POINTER(State), C.POINTER(Aux)]
    L.orc_diagnostics.argtypes = [C.POINTER(Params), C.POINTER(State), C.POINTER(Diag)]
    L.orc_num_threads.restype = C.c_int
    L.orc_set_celllist_threshold.argtypes = [C.c_int64]
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_params(prm) -> Params:
    """orc_params from an inputs.Params. f_b is resolved here when the
    workload asks for the balancing body force (filled in by the caller
    through `fb`); T_c <= 0 is resolved inside the oracle."""
    P = Params()
    P.n[:] = [int(v) for v in prm.n]
    P.periodic[:] = [int(v) for v in prm.periodic]
    P.tau = prm.tau
    P.rho_f = prm.rho_f
    P.g[:] = list(prm.gravity)
    P.fb[:] = list(prm.body_force)
    P.e_n, P.mu_c, P.T_c, P.h_c, P.h_min = prm.e_n, prm.mu_c, prm.T_c, prm.h_c, prm.h_min
    P.lub_stab, P.use_lub, P.use_am = prm.lub_stab, prm.use_lub, prm.use_am
    P.n_int, P.n_dem = prm.n_int, prm.n_dem
    P.c_am = prm.c_am
    P.use_lift = int(getattr(prm, "use_lift", 0))
    P.use_eilers = int(getattr(prm, "use_eilers", 0))
    P.use_les = int(getattr(prm, "use_les", 0))
    P.lub_contact = int(getattr(prm, "lub_contact", 1))
    return P


def balancing_body_force(prm, particles) -> tuple:
    """Fluid body force that balances the particles' submerged weight in a
    fully periodic box (Sec. 4.1, Setup): f_b = -sum_p (rho_p - rho_f) V_p g / (Lx Ly Lz).
    Zero for walled domains, where the walls carry the load."""
    if not all(prm.periodic):
        return (0.0, 0.0, 0.0)
    nc = prm.n[0] * prm.n[1] * prm.n[2]
    V = np.pi * particles.d ** 3 / 6.0
    s = float(((particles.rho_p - prm.rho_f) * V).sum()) / nc
    return tuple(-s * g for g in prm.gravity)


@dataclass
class OState:
    df: np.ndarray      # (19, Nc)
    uprev: np.ndarray   # (3, Nc)
    step: int
    x: np.ndarray
    u: np.ndarray
    w: np.ndarray
    a: np.ndarray
    d: np.ndarray
    rho_p: np.ndarray

    @staticmethod
    def initial(prm, particles, df=None):
        nc = prm.n[0] * prm.n[1] * prm.n[2]
        return OState(np.zeros((19, nc)) if df is None else np.array(df, np.float64, copy=True),
                      np.zeros((3, nc)), 0,
                      particles.x.copy(), particles.u.copy(), particles.w.copy(), particles.a.copy(),
                      particles.d.copy(), particles.rho_p.copy())

    def copy(self):
        return OState(self.df.copy(), self.uprev.copy(), self.step, self.x.copy(), self.u.copy(),
                      self.w.copy(), self.a.copy(), self.d.copy(), self.rho_p.copy())

    def cstruct(self) -> State:
        for k in ("df", "uprev", "x", "u", "w", "a", "d", "rho_p"):
            v = getattr(self, k)
            assert v.dtype == np.float64 and v.flags.c_contiguous, k
        S = State()
        S.df, S.uprev, S.step = _p(self.df), _p(self.uprev), self.step
        S.np = len(self.d)
        S.x, S.u, S.w, S.a, S.d, S.rho_p = (_p(self.x), _p(self.u), _p(self.w), _p(self.a),
                                            _p(self.d), _p(self.rho_p))
        return S


class Oracle:
    """One domain advanced by the oracle."""

    def __init__(self, prm, particles, df=None):
        self.prm = prm
        fb = prm.body_force
        if prm.body_force_auto:
            fb = balancing_body_force(prm, particles)
        self.fb = fb
        self.P = make_params(prm)
        self.P.fb[:] = list(fb)
        self.state = OState.initial(prm, particles, df)
        self.nc = prm.n[0] * prm.n[1] * prm.n[2]

    def step(self, nsteps=1, aux=False):
        L = lib()
        out = None
        for _ in range(nsteps):
            S = self.state.cstruct()
            A = Aux()
            keep = {}
            if aux:
                nc, np_ = self.nc, len(self.state.d)
                for k, shp in (("f_acc", (3, nc)), ("eps_f", (nc,)), ("dudt", (3, nc)),
                               ("gradp", (3, nc)), ("rho", (nc,)), ("j", (3, nc)),
                               ("F_am", (np_, 3)), ("F_d", (np_, 3)), ("F_pr", (np_, 3)),
                               ("F_const", (np_, 3)), ("F_l", (np_, 3)), ("curl", (3, nc))):
                    keep[k] = np.zeros(shp)
                    setattr(A, k, _p(keep[k]))
            st = L.orc_step(C.byref(self.P), C.byref(S), C.byref(A))
            self.state.step = S.step
            out = dict(keep)
            out["status"] = st
            out["impulse_pr"] = np.array(A.impulse_pr[:])
            out["impulse_gb"] = np.array(A.impulse_gb[:])
            out["impulse_fb"] = np.array(A.impulse_fb[:])
            out["min_eps_f"] = A.min_eps_f
            if st != 0:
                break
        return out

    def diagnostics(self):
        D = Diag()
        S = self.state.cstruct()
        lib().orc_diagnostics(C.byref(self.P), C.byref(S), C.byref(D))
        return dict(mass_dev=D.mass_dev, mom_fluid=np.array(D.mom_fluid[:]), mom_part=np.array(D.mom_part[:]),
                    u_ps=D.u_ps, mean_eps_f=D.mean_eps_f, min_eps_f=D.min_eps_f, max_u=D.max_u)

    def eps_field(self):
        e = np.zeros(self.nc)
        lib().orc_eps_field(C.byref(self.P), len(self.state.d), _p(self.state.x), _p(self.state.d), _p(e))
        return e


# -- thin wrappers for the closed-form tests --------------------------------
def roma(r: float) -> float:
    return lib().orc_roma(float(r))


def axis_stencil(xp, n, periodic):
    idx = np.zeros(3, np.int32)
    wt = np.zeros(3)
    m = lib().orc_axis_stencil(float(xp), int(n), int(periodic), _p(idx), _p(wt))
    return idx[:m].copy(), wt[:m].copy()


def feq_dev(drho, u, eps):
    out = np.zeros(19)
    lib().orc_feq_dev(float(drho), _p(np.asarray(u, np.float64)), float(eps), _p(out))
    return out


def guo(u, eps, f, tau):
    out = np.zeros(19)
    lib().orc_guo(_p(np.asarray(u, np.float64)), float(eps), _p(np.asarray(f, np.float64)), float(tau), _p(out))
    return out


def moments(dfq):
    dr = np.zeros(1)
    j = np.zeros(3)
    lib().orc_moments(_p(np.ascontiguousarray(dfq, np.float64)), _p(dr), _p(j))
    return dr[0], j


def drag_factor(Re, eps):
    return lib().orc_drag_factor(float(Re), float(eps))


def drag(d, mu, rho_f, eps, w):
    F = np.zeros(3)
    lib().orc_drag(float(d), float(mu), float(rho_f), float(eps), _p(np.asarray(w, np.float64)), _p(F))
    return F


def lift(d, mu, rho_f, w, om):
    F = np.zeros(3)
    lib().orc_lift(float(d), float(mu), float(rho_f), _p(_v(w)), _p(_v(om)), _p(F))
    return F


def tau_e(P, eps_p, rho, df, feq):
    """Per-cell relaxation time of a cell state (Eilers and/or LES per P)."""
    return lib().orc_tau_e(C.byref(P), float(eps_p), float(rho), _p(_v(df)), _p(_v(feq)))


def curl_field(P, u):
    """Lattice curl of a [3][Nc] velocity field (Sec. 3.2.3), walls by the
    ghost rule of the velocity gradient."""
    out = np.zeros((3, P.n[0] * P.n[1] * P.n[2]))
    lib().orc_curl_field(C.byref(P), _p(_v(u)), _p(out))
    return out


def collision_params(mij, e_n, T_c):
    kn = np.zeros(1); xi = np.zeros(1)
    lib().orc_collision_params(float(mij), float(e_n), float(T_c), _p(kn), _p(xi))
    return kn[0], xi[0]


def lub_coeffs(h, dm, mu):
    a = np.zeros(1); b = np.zeros(1)
    lib().orc_lub_coeffs(float(h), float(dm), float(mu), _p(a), _p(b))
    return a[0], b[0]


def _v(a):
    return np.ascontiguousarray(a, np.float64)


def pair_force(P, xi, ui, wi, di, rhoi, xj, uj, wj, dj, rhoj, dt_dem):
    F = np.zeros(3); T = np.zeros(3)
    args = [_v(xi), _v(ui), _v(wi), _v(xj), _v(uj), _v(wj)]
    lib().orc_pair_force(C.byref(P), _p(args[0]), _p(args[1]), _p(args[2]), float(di), float(rhoi),
                         _p(args[3]), _p(args[4]), _p(args[5]), float(dj), float(rhoj), float(dt_dem),
                         _p(F), _p(T))
    return F, T


def wall_force(P, xi, ui, wi, di, rhoi, dt_dem):
    F = np.zeros(3); T = np.zeros(3)
    args = [_v(xi), _v(ui), _v(wi)]
    lib().orc_wall_force(C.byref(P), _p(args[0]), _p(args[1]), _p(args[2]), float(di), float(rhoi),
                         float(dt_dem), _p(F), _p(T))
    return F, T


def dem_forces(P, x, u, w, d, rho_p, dt_dem):
    n = len(d)
    F = np.zeros((n, 3)); T = np.zeros((n, 3))
    arrs = [_v(x), _v(u), _v(w), _v(d), _v(rho_p)]
    lib().orc_dem_forces(C.byref(P), n, *[_p(a) for a in arrs], float(dt_dem), _p(F), _p(T))
    return F, T


def lbm_collide_stream(P, df, eps_f=None, f_acc=None):
    out = np.zeros_like(df)
    lib().orc_lbm_collide_stream(C.byref(P), _p(_v(df)), _p(out),
                                 _p(_v(eps_f)) if eps_f is not None else None,
                                 _p(_v(f_acc)) if f_acc is not None else None)
    return out


def interp_scalar(P, field, xp) -> float:
    """phi_|p of a scalar cell field at position xp (Eq. interpolation)."""
    return lib().orc_interp_scalar(C.byref(P), _p(_v(field)), _p(_v(xp)))


def spread_scalar(P, field, xp, val) -> None:
    """field += D(x, xp) val in place (Eq. distribution_filter)."""
    assert field.dtype == np.float64 and field.flags.c_contiguous
    lib().orc_spread_scalar(C.byref(P), _p(field), _p(_v(xp)), float(val))


def set_celllist_threshold(n: int) -> None:
    lib().orc_set_celllist_threshold(int(n))


def num_threads() -> int:
    return lib().orc_num_threads()
