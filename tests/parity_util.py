"""Helpers for GPU-vs-oracle parity tests (test infrastructure)."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def rel_err(a, b, scale=None):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.size == 0 and b.size == 0:
        return 0.0
    s = np.abs(b).max() if scale is None else scale
    d = np.abs(a - b).max()
    if s == 0.0:
        return 0.0 if d == 0.0 else np.inf
    return d / s


def pos_err(xg, xo, n, periodic):
    """max |x_gpu - x_oracle| with the minimum image on periodic axes, / max|x|"""
    d = np.asarray(xg) - np.asarray(xo)
    for a in range(3):
        if periodic[a]:
            d[:, a] -= n[a] * np.round(d[:, a] / n[a])
    if d.size == 0:
        return 0.0
    return np.abs(d).max() / max(np.abs(xo).max(), 1.0)


def load_oracle_state(dom, st: "O.OState"):
    dom.lbdem_set_state(st.df, st.uprev, st.step, st.x, st.u, st.w, st.a, st.d, st.rho_p)


def compare_states(g, o: "O.OState", prm, tol):
    """Per-array relative errors (max|gpu - oracle| / max|oracle|)."""
    # du_p/dt is a difference quotient of velocities over one subcycle; its
    # error is measured against the velocity scale it is formed from.
    a_scale = max(np.abs(o.a).max() if o.a.size else 0.0,
                  (np.abs(o.u).max() if o.u.size else 0.0) * prm.n_int)
    errs = dict(df=rel_err(g["df"], o.df), uprev=rel_err(g["uprev"], o.uprev),
                x=pos_err(g["x"], o.x, prm.n, prm.periodic), u=rel_err(g["u"], o.u),
                w=rel_err(g["w"], o.w), a=rel_err(g["a"], o.a, scale=a_scale))
    bad = {k: v for k, v in errs.items() if not (v <= tol[k] if isinstance(tol, dict) else v <= tol)}
    return errs, bad


def warm_oracle(case, nsteps, perturb=None):
    """Oracle advanced nsteps from the case's initial state (gives non-trivial
    u_prev, velocities, accelerations and contacts). perturb: optional initial
    PDF deviations."""
    o = O.Oracle(case.params, case.particles, df=perturb)
    if nsteps:
        r = o.step(nsteps)
        assert r["status"] == 0
    return o
