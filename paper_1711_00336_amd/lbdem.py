"""ctypes binding of the C ABI in include/lbdem.h (argument marshalling only).

Every step of the coupled LBM-DEM time step runs in the HIP library
(_lib/liblbdem.so). Importing this module loads that library and raises if it
is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblbdem.so")

OK, E_INVALID, E_OOM, E_UNSTABLE, E_DEVICE, E_BUSY, E_STATE = range(7)
FP64, FP32_DEV = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
(FIELD_DRHO, FIELD_J, FIELD_EPS_F, FIELD_F_ACC, FIELD_DUDT, FIELD_GRADP, FIELD_UPREV, FIELD_PDF,
 FIELD_CURL) = range(9)
FIELD_NCOMP = {FIELD_DRHO: 1, FIELD_J: 3, FIELD_EPS_F: 1, FIELD_F_ACC: 3, FIELD_DUDT: 3,
               FIELD_GRADP: 3, FIELD_UPREV: 3, FIELD_PDF: 19, FIELD_CURL: 3}
FLAG_NO_GRAPH = 1
KCLASS = {"stream_collide": 0, "moments": 1, "cellfields": 2, "part_am": 3, "part_drag": 4,
          "gather_am": 5, "gather_fd": 6, "gather_eps": 7, "nlist": 8, "dem_force": 9,
          "integrate": 10, "bins": 11, "curl": 12}


class LbdemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbdem status {status}: {msg}")
        self.status = status


class lbdem_params(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("periodic", C.c_int32 * 3),
                ("tau", C.c_double), ("rho_f", C.c_double),
                ("gravity", C.c_double * 3), ("body_force", C.c_double * 3),
                ("body_force_auto", C.c_int32),
                ("e_n", C.c_double), ("mu_c", C.c_double), ("T_c", C.c_double),
                ("h_c", C.c_double), ("h_min", C.c_double),
                ("lub_stab", C.c_int32), ("use_lub", C.c_int32), ("use_am", C.c_int32),
                ("n_int", C.c_int32), ("n_dem", C.c_int32),
                ("c_am", C.c_double), ("precision", C.c_int32), ("flags", C.c_uint32),
                ("use_lift", C.c_int32), ("use_eilers", C.c_int32), ("use_les", C.c_int32),
                ("lub_contact", C.c_int32)]


class lbdem_diag(C.Structure):
    _fields_ = [("mass_dev", C.c_double), ("mom_fluid", C.c_double * 3),
                ("mom_part", C.c_double * 3), ("u_ps", C.c_double),
                ("mean_eps_f", C.c_double), ("min_eps_f", C.c_double),
                ("max_u", C.c_double), ("step", C.c_int64), ("np", C.c_int64)]


class lbdem_state_view(C.Structure):
    _fields_ = [("df", C.c_void_p), ("uprev", C.c_void_p), ("step", C.c_int64),
                ("np", C.c_int64), ("x", C.c_void_p), ("u", C.c_void_p),
                ("omega", C.c_void_p), ("accel", C.c_void_p), ("d", C.c_void_p),
                ("rho_p", C.c_void_p)]


class lbdem_tuning(C.Structure):
    _fields_ = [("gather_variant", C.c_int32), ("dem_order", C.c_int32), ("dem_block", C.c_int32 * 3),
                ("cell_waves", C.c_int32), ("fuse_substep", C.c_int32)]


class lbdem_request(C.Structure):
    _fields_ = [("params", lbdem_params), ("np", C.c_int64), ("x", C.c_void_p), ("u", C.c_void_p),
                ("omega", C.c_void_p), ("d", C.c_void_p), ("rho_p", C.c_void_p),
                ("steps", C.c_int64), ("avg_from", C.c_int64)]


class lbdem_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps_done", C.c_int64), ("u_ps", C.c_double),
                ("mean_eps_f", C.c_double), ("mom", C.c_double * 3), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} (run python -m paper_1711_00336_amd.build)")
        # PyTorch wheels bring their own HIP runtime and a process can use only
        # one: loading torch first (when installed) binds this library to the
        # runtime torch uses, so device pointers, streams and the caching
        # allocator can be shared with it whatever the import order.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        H = C.c_void_p
        st = C.c_int
        sig = {
            "lbdem_last_error": (C.c_char_p, [H]),
            "lbdem_params_default": (st, [C.POINTER(lbdem_params)]),
            "lbdem_set_allocator": (st, [C.c_void_p, C.c_void_p, C.c_void_p]),
            "lbdem_create": (st, [C.POINTER(lbdem_params), C.c_void_p, C.POINTER(H)]),
            "lbdem_destroy": (st, [H]),
            "lbdem_add_particles": (st, [H, C.c_int64] + [C.c_void_p] * 5),
            "lbdem_step": (st, [H, C.c_int64]),
            "lbdem_sync": (st, [H]),
            "lbdem_read_field": (st, [H, C.c_int, C.c_int, C.c_void_p]),
            "lbdem_read_particles": (st, [H, C.c_int] + [C.c_void_p] * 4),
            "lbdem_read_particle_forces": (st, [H] + [C.c_void_p] * 4),
            "lbdem_read_particle_lift": (st, [H, C.c_void_p]),
            "lbdem_diagnostics": (st, [H, C.POINTER(lbdem_diag)]),
            "lbdem_diagnostics_noalloc": (st, [H, C.POINTER(lbdem_diag)]),
            "lbdem_num_cells": (C.c_int64, [H]),
            "lbdem_num_particles": (C.c_int64, [H]),
            "lbdem_get_state": (st, [H, C.POINTER(lbdem_state_view)]),
            "lbdem_set_state": (st, [H, C.POINTER(lbdem_state_view)]),
            "lbdem_save_state": (st, [H, C.c_void_p, C.POINTER(C.c_size_t)]),
            "lbdem_load_state": (st, [H, C.c_void_p, C.c_size_t]),
            "lbdem_set_timing": (st, [H, C.c_int]),
            "lbdem_autotune": (st, [H, C.POINTER(C.c_int32)]),
            "lbdem_set_gather_variant": (st, [H, C.c_int32]),
            "lbdem_get_tuning": (st, [H, C.POINTER(lbdem_tuning)]),
            "lbdem_set_tuning": (st, [H, C.POINTER(lbdem_tuning)]),
            "lbdem_batch_create": (st, [C.c_int32, C.POINTER(lbdem_params), C.c_void_p, C.POINTER(H)]),
            "lbdem_batch_domain": (st, [H, C.c_int32, C.POINTER(H)]),
            "lbdem_batch_size": (C.c_int32, [H]),
            "lbdem_batch_autotune": (st, [H]),
            "lbdem_batch_step": (st, [H, C.c_int64]),
            "lbdem_batch_sync": (st, [H]),
            "lbdem_batch_destroy": (st, [H]),
            "lbdem_server_last_error": (C.c_char_p, []),
            "lbdem_server_create": (st, [C.c_size_t, C.c_int32, C.c_int32, C.POINTER(H)]),
            "lbdem_server_submit": (st, [H, C.POINTER(lbdem_request), C.POINTER(C.c_uint64)]),
            "lbdem_server_poll": (st, [H, C.c_uint64, C.POINTER(lbdem_result)]),
            "lbdem_server_cancel": (st, [H, C.c_uint64]),
            "lbdem_server_stats": (st, [H, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
            "lbdem_server_destroy": (st, [H]),
            "lbdem_kernel_time": (st, [H, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
            "lbdem_stability_limit": (st, [C.POINTER(lbdem_params), C.c_int64, C.c_void_p, C.c_void_p,
                                           C.POINTER(C.c_double)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _check(h, status):
    if status != OK:
        msg = lib().lbdem_last_error(h)
        raise LbdemError(status, msg.decode() if msg else "")


def params_from(prm) -> lbdem_params:
    """lbdem_params from an inputs.Params (or any object with the same fields)."""
    P = lbdem_params()
    _check(None, lib().lbdem_params_default(C.byref(P)))
    P.n[:] = [int(v) for v in prm.n]
    P.periodic[:] = [int(v) for v in prm.periodic]
    P.tau, P.rho_f = prm.tau, prm.rho_f
    P.gravity[:] = list(prm.gravity)
    P.body_force[:] = list(prm.body_force)
    P.body_force_auto = int(prm.body_force_auto)
    P.e_n, P.mu_c, P.T_c, P.h_c, P.h_min = prm.e_n, prm.mu_c, prm.T_c, prm.h_c, prm.h_min
    P.lub_stab, P.use_lub, P.use_am = int(prm.lub_stab), int(prm.use_lub), int(prm.use_am)
    P.n_int, P.n_dem = int(prm.n_int), int(prm.n_dem)
    P.c_am = prm.c_am
    P.precision = FP32_DEV if prm.precision == "fp32dev" else FP64
    P.flags = int(getattr(prm, "flags", 0))
    P.use_lift = int(getattr(prm, "use_lift", 0))
    P.use_eilers = int(getattr(prm, "use_eilers", 0))
    P.use_les = int(getattr(prm, "use_les", 0))
    P.lub_contact = int(getattr(prm, "lub_contact", 1))
    return P


def lbdem_stability_limit(prm, d, rho_p):
    """(status, largest stable interaction subcycle length) of the explicit
    coupling estimate for these particles (host-only; no device needed)."""
    P = params_from(prm)
    d = np.ascontiguousarray(d, np.float64).reshape(-1)
    rho_p = np.ascontiguousarray(rho_p, np.float64).reshape(-1)
    out = C.c_double(0.0)
    st = lib().lbdem_stability_limit(C.byref(P), len(d), _ptr(d), _ptr(rho_p), C.byref(out))
    if st not in (OK, E_UNSTABLE):
        _check(None, st)
    return st, out.value


class Domain:
    """One domain of the C library (lbdem_create ... lbdem_destroy)."""

    def __init__(self, prm, stream=None, handle=None):
        self.prm = prm
        self.P = params_from(prm)
        self.owned = handle is None
        if handle is None:
            self.h = C.c_void_p()
            s = None if stream is None else C.c_void_p(int(stream))
            _check(None, lib().lbdem_create(C.byref(self.P), s, C.byref(self.h)))
        else:
            self.h = handle
        self.nc = int(lib().lbdem_num_cells(self.h))

    def close(self):
        if self.h and self.owned:
            lib().lbdem_destroy(self.h)
        self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- calls with the names of the C ABI ----------------------------------
    def lbdem_add_particles(self, x, u, omega, d, rho_p):
        x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
        n = len(x)
        u = np.ascontiguousarray(u, np.float64).reshape(n, 3)
        omega = np.ascontiguousarray(omega, np.float64).reshape(n, 3)
        d = np.ascontiguousarray(d, np.float64).reshape(n)
        rho_p = np.ascontiguousarray(rho_p, np.float64).reshape(n)
        _check(self.h, lib().lbdem_add_particles(self.h, n, _ptr(x), _ptr(u), _ptr(omega), _ptr(d), _ptr(rho_p)))

    def add(self, particles):
        self.lbdem_add_particles(particles.x, particles.u, particles.w, particles.d, particles.rho_p)

    def lbdem_step(self, nsteps=1):
        _check(self.h, lib().lbdem_step(self.h, int(nsteps)))

    def lbdem_sync(self):
        _check(self.h, lib().lbdem_sync(self.h))

    def step(self, nsteps=1, sync=True):
        self.lbdem_step(nsteps)
        if sync:
            self.lbdem_sync()

    def lbdem_read_field(self, field, out=None):
        ncomp = FIELD_NCOMP[field]
        if out is None:
            out = np.zeros((ncomp, self.nc) if ncomp > 1 else (self.nc,))
            _check(self.h, lib().lbdem_read_field(self.h, field, MEM_HOST, _ptr(out)))
        else:  # torch tensor on the device
            _check(self.h, lib().lbdem_read_field(self.h, field, MEM_DEVICE, C.c_void_p(out.data_ptr())))
        return out

    def num_particles(self):
        return int(lib().lbdem_num_particles(self.h))

    def lbdem_read_particles(self):
        n = self.num_particles()
        x, u, w, a = (np.zeros((n, 3)) for _ in range(4))
        _check(self.h, lib().lbdem_read_particles(self.h, MEM_HOST, _ptr(x), _ptr(u), _ptr(w), _ptr(a)))
        return x, u, w, a

    def lbdem_read_particle_forces(self):
        n = self.num_particles()
        F = [np.zeros((n, 3)) for _ in range(4)]
        _check(self.h, lib().lbdem_read_particle_forces(self.h, *[_ptr(f) for f in F]))
        return dict(F_am=F[0], F_d=F[1], F_pr=F[2], F_const=F[3])

    def lbdem_read_particle_lift(self):
        F = np.zeros((self.num_particles(), 3))
        _check(self.h, lib().lbdem_read_particle_lift(self.h, _ptr(F)))
        return F

    def lbdem_diagnostics(self):
        D = lbdem_diag()
        _check(self.h, lib().lbdem_diagnostics(self.h, C.byref(D)))
        return dict(mass_dev=D.mass_dev, mom_fluid=np.array(D.mom_fluid[:]), mom_part=np.array(D.mom_part[:]),
                    u_ps=D.u_ps, mean_eps_f=D.mean_eps_f, min_eps_f=D.min_eps_f, max_u=D.max_u,
                    step=D.step, np=D.np)

    def lbdem_diagnostics_noalloc(self):
        D = lbdem_diag()
        _check(self.h, lib().lbdem_diagnostics_noalloc(self.h, C.byref(D)))
        return dict(mass_dev=D.mass_dev, mom_fluid=np.array(D.mom_fluid[:]), mom_part=np.array(D.mom_part[:]),
                    u_ps=D.u_ps, mean_eps_f=D.mean_eps_f, min_eps_f=D.min_eps_f, max_u=D.max_u,
                    step=D.step, np=D.np)

    def lbdem_get_state(self):
        n = self.num_particles()
        df = np.zeros((19, self.nc)); up = np.zeros((3, self.nc))
        x, u, w, a = (np.zeros((n, 3)) for _ in range(4))
        d = np.zeros(n); r = np.zeros(n)
        V = lbdem_state_view(_ptr(df).value, _ptr(up).value, 0, n, _ptr(x).value, _ptr(u).value,
                             _ptr(w).value, _ptr(a).value, _ptr(d).value, _ptr(r).value)
        _check(self.h, lib().lbdem_get_state(self.h, C.byref(V)))
        return dict(df=df, uprev=up, step=int(V.step), x=x, u=u, w=w, a=a, d=d, rho_p=r)

    def lbdem_set_state(self, df, uprev, step, x, u, w, a, d, rho_p):
        arrs = [np.ascontiguousarray(v, np.float64) for v in (df, uprev, x, u, w, a, d, rho_p)]
        n = len(arrs[6])
        assert arrs[0].size == 19 * self.nc and arrs[1].size == 3 * self.nc
        V = lbdem_state_view(_ptr(arrs[0]).value, _ptr(arrs[1]).value, int(step), n,
                             *[_ptr(v).value for v in arrs[2:]])
        _check(self.h, lib().lbdem_set_state(self.h, C.byref(V)))

    def lbdem_save_state(self) -> bytes:
        sz = C.c_size_t(0)
        _check(self.h, lib().lbdem_save_state(self.h, None, C.byref(sz)))
        buf = (C.c_char * sz.value)()
        _check(self.h, lib().lbdem_save_state(self.h, C.cast(buf, C.c_void_p), C.byref(sz)))
        return bytes(buf)

    def lbdem_load_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(self.h, lib().lbdem_load_state(self.h, C.cast(buf, C.c_void_p), len(blob)))

    def lbdem_set_timing(self, on: bool):
        _check(self.h, lib().lbdem_set_timing(self.h, 1 if on else 0))

    def lbdem_get_tuning(self):
        T = lbdem_tuning()
        _check(self.h, lib().lbdem_get_tuning(self.h, C.byref(T)))
        return dict(gather_variant=T.gather_variant, dem_order=T.dem_order, dem_block=tuple(T.dem_block[:]),
                    cell_waves=T.cell_waves, fuse_substep=T.fuse_substep)

    def lbdem_set_tuning(self, gather_variant=-1, dem_order=-1, dem_block=(32, 32, 32), cell_waves=-1,
                         fuse_substep=-1):
        T = lbdem_tuning(int(gather_variant), int(dem_order), (C.c_int32 * 3)(*[int(v) for v in dem_block]),
                         int(cell_waves), int(fuse_substep))
        _check(self.h, lib().lbdem_set_tuning(self.h, C.byref(T)))

    def lbdem_autotune(self):
        v = C.c_int32(-1)
        _check(self.h, lib().lbdem_autotune(self.h, C.byref(v)))
        return v.value

    def lbdem_set_gather_variant(self, variant):
        _check(self.h, lib().lbdem_set_gather_variant(self.h, int(variant)))

    def lbdem_kernel_time(self, cls):
        ms = C.c_double(0.0); n = C.c_int64(0)
        c = KCLASS[cls] if isinstance(cls, str) else int(cls)
        _check(self.h, lib().lbdem_kernel_time(self.h, c, C.byref(ms), C.byref(n)))
        return ms.value, n.value


class Batch:
    """Many independent domains advanced by one graph (lbdem_batch_*)."""

    def __init__(self, prms, stream=None):
        arr = (lbdem_params * len(prms))(*[params_from(p) for p in prms])
        self.h = C.c_void_p()
        s = None if stream is None else C.c_void_p(int(stream))
        _check(None, lib().lbdem_batch_create(len(prms), arr, s, C.byref(self.h)))
        self.domains = []
        for i, p in enumerate(prms):
            dh = C.c_void_p()
            _check(None, lib().lbdem_batch_domain(self.h, i, C.byref(dh)))
            self.domains.append(Domain(p, handle=dh))

    def lbdem_batch_autotune(self):
        _check(None, lib().lbdem_batch_autotune(self.h))
        out = []
        for d in self.domains:
            v = C.c_int32(-1)
            _check(d.h, lib().lbdem_autotune(d.h, C.byref(v)))
            out.append(v.value)
        return out

    def lbdem_batch_step(self, nsteps=1):
        _check(None, lib().lbdem_batch_step(self.h, int(nsteps)))

    def lbdem_batch_sync(self):
        _check(None, lib().lbdem_batch_sync(self.h))

    def step(self, nsteps=1):
        self.lbdem_batch_step(nsteps)
        self.lbdem_batch_sync()

    def close(self):
        if self.h:
            for d in self.domains:
                d.h = C.c_void_p()
            lib().lbdem_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _scheck(status):
    if status != OK:
        msg = lib().lbdem_server_last_error()
        raise LbdemError(status, msg.decode() if msg else "")


class Server:
    """Request loop for settling solves (lbdem_server_*)."""

    def __init__(self, hbm_budget, max_slots=64, chunk_steps=20):
        self.h = C.c_void_p()
        _scheck(lib().lbdem_server_create(int(hbm_budget), int(max_slots), int(chunk_steps), C.byref(self.h)))

    def lbdem_server_submit(self, prm, particles, steps, avg_from=0):
        P = particles
        arrs = [np.ascontiguousarray(v, np.float64) for v in (P.x, P.u, P.w, P.d, P.rho_p)]
        R = lbdem_request(params_from(prm), len(arrs[3]), *[_ptr(a).value for a in arrs], int(steps), int(avg_from))
        t = C.c_uint64(0)
        _scheck(lib().lbdem_server_submit(self.h, C.byref(R), C.byref(t)))
        return t.value

    def lbdem_server_poll(self, ticket):
        R = lbdem_result()
        st = lib().lbdem_server_poll(self.h, int(ticket), C.byref(R))
        if st == E_BUSY:
            return None
        _scheck(st)
        return dict(status=R.status, steps_done=R.steps_done, u_ps=R.u_ps, mean_eps_f=R.mean_eps_f,
                    mom=np.array(R.mom[:]), t_submit=R.t_submit, t_admit=R.t_admit, t_done=R.t_done)

    def lbdem_server_cancel(self, ticket):
        return lib().lbdem_server_cancel(self.h, int(ticket))

    def lbdem_server_stats(self):
        q = C.c_int64(0); a = C.c_int64(0); b = C.c_size_t(0)
        _scheck(lib().lbdem_server_stats(self.h, C.byref(q), C.byref(a), C.byref(b)))
        return dict(queued=q.value, active=a.value, bytes=b.value)

    def wait(self, ticket, timeout=600.0, poll_s=0.002):
        import time
        t0 = time.time()
        while True:
            r = self.lbdem_server_poll(ticket)
            if r is not None:
                return r
            if time.time() - t0 > timeout:
                raise TimeoutError(f"request {ticket} not done after {timeout} s")
            time.sleep(poll_s)

    def close(self):
        if self.h:
            lib().lbdem_server_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_allocator_refs = []


def use_torch_allocator(enable=True):
    """Route the device allocations of domains created from now on through
    PyTorch's caching allocator (lbdem_set_allocator), or back to
    hipMalloc/hipFree with enable=False. Domains free their memory after
    synchronising their stream, so torch reuses a block only once the
    library is done with it."""
    if not enable:
        _check(None, lib().lbdem_set_allocator(None, None, None))
        _allocator_refs.clear()
        return
    import torch

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except RuntimeError:
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a, f = _ALLOC_FN(_alloc), _FREE_FN(_free)
    _check(None, lib().lbdem_set_allocator(C.cast(a, C.c_void_p), C.cast(f, C.c_void_p), None))
    _allocator_refs[:] = [a, f]


def exported_symbols():
    """Names declared in include/lbdem.h (for the export test)."""
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "lbdem.h")
    src = open(hdr).read()
    return sorted(set(re.findall(r"\b(lbdem_[a-z_]+)\s*\(", src)))
