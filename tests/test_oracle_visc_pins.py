"""Pins of the oracle's per-cell relaxation time tau_e = tau_* + tau_t
(Eilers viscosity, Eq. visc_eilers; Smagorinsky LES, Eqs. visc_turb and
tau_t; Alg. 1, the steps before the GNS-LBM step).

  * Eilers: the viscosity ratio mu_*/mu_0 starts at 1 with Einstein's slope
    2.5 (the dilute-suspension limit the intrinsic viscosity [mu] = 2.5
    encodes) and diverges at random close packing eps_p -> 0.64 (not at
    eps_p -> 1, which the garbled printed denominator would give).
  * Smagorinsky: on a Chapman-Enskog non-equilibrium state of strain rate S,
    f_neq = -(w rho tau_e / c_s^2)(c c - c_s^2 I) : S, the model's relaxation
    time is the fixed point tau_e = tau_* + (C_s dx)^2 |S| / c_s^2 with
    |S| = sqrt(2 S:S), C_s = 0.1 (Smagorinsky's nu_t = (C_s dx)^2 |S|).
  * Poiseuille flow through a uniform suspension is the exact BGK profile at
    the Eilers relaxation time.
  * The momentum budget of one collide-stream stays exact with a per-cell
    tau_e (the collision and the forcing prefactor use the same tau_e).
"""
import math

import numpy as np
import pytest

from paper_1711_00336_amd import inputs as I

C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
              [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], float)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
CS2 = 1.0 / 3.0


def _P(orc, tau=0.8, eilers=1, les=0, n=(4, 4, 4), periodic=(1, 1, 1)):
    return orc.make_params(I.Params(n=n, periodic=periodic, tau=tau, use_eilers=eilers, use_les=les))


def _ratio(orc, P, tau, ep):
    z = np.zeros(19)
    return (orc.tau_e(P, ep, 1.0, z, z) - 0.5) / (tau - 0.5)


def test_eilers_einstein_limit_and_close_packing(orc):
    tau = 0.8
    P = _P(orc, tau)
    assert orc.tau_e(P, 0.0, 1.0, np.zeros(19), np.zeros(19)) == tau
    h = 1e-7
    assert (_ratio(orc, P, tau, h) - 1.0) / h == pytest.approx(2.5, abs=1e-5)
    r = [_ratio(orc, P, tau, e) for e in np.linspace(0.0, 0.63, 64)]
    assert np.all(np.diff(r) > 0)
    assert _ratio(orc, P, tau, 0.64 - 1e-9) > 1e15
    assert _ratio(orc, _P(orc, tau, eilers=0), tau, 0.5) == 1.0


def _ce_state(rho, u, eps, S, tau_e):
    """feq (deviation form) and f = feq + Chapman-Enskog non-equilibrium part."""
    cu = C @ u
    feq = W * (rho - 1) + W * rho * (cu / CS2 + cu * cu / (2 * eps * CS2 ** 2) - (u @ u) / (2 * eps * CS2))
    cc = np.einsum("qa,qb->qab", C, C) - CS2 * np.eye(3)[None]
    fneq = -(W * rho * tau_e / CS2) * np.einsum("qab,ab->q", cc, S)
    return feq + fneq, feq


@pytest.mark.parametrize("eilers", [0, 1])
def test_smagorinsky_fixed_point_on_chapman_enskog_states(orc, eilers):
    rng = np.random.default_rng(4)
    tau = 0.62
    P = _P(orc, tau, eilers=eilers, les=1)
    cs = 0.1
    for _ in range(20):
        A = rng.normal(size=(3, 3)) * 10 ** rng.uniform(-4, -1)
        S = 0.5 * (A + A.T)
        rho, ep = rng.uniform(0.97, 1.03), rng.uniform(0.0, 0.5)
        u = rng.normal(size=3) * 1e-2
        tau_s = 0.5 + (tau - 0.5) * ((1 + 1.25 * ep / (1 - ep / 0.64)) ** 2 if eilers else 1.0)
        target = tau_s + cs * cs * math.sqrt(2 * np.sum(S * S)) / CS2
        df, feq = _ce_state(rho, u, 1 - ep, S, target)
        got = orc.tau_e(P, ep, rho, df, feq)
        assert got == pytest.approx(target, rel=1e-12)
    # no strain, no subgrid viscosity
    df, feq = _ce_state(1.01, np.array([1e-2, 0, 0]), 0.9, np.zeros((3, 3)), tau)
    assert orc.tau_e(_P(orc, tau, eilers=0, les=1), 0.1, 1.01, df, feq) == tau


@pytest.mark.parametrize("tau", [0.6, 0.8])
def test_poiseuille_with_eilers_viscosity(orc, tau):
    """Body-force Poiseuille flow through a uniform suspension (eps_f = 0.8)
    between half-way bounce-back walls: the exact BGK profile
    u = eps g/(2 nu)[z(H - z) + (16 Lambda - 3)/12], Lambda = (tau - 1/2)^2,
    evaluated at the Eilers relaxation time."""
    H, g, eps = 8, 1e-6, 0.8
    P = _P(orc, tau, eilers=1, n=(1, 1, H), periodic=(1, 1, 0))
    ep = 1 - eps
    ts = 0.5 + (tau - 0.5) * (1 + 2.5 * 0.5 * ep / (1 - ep / 0.64)) ** 2
    df = np.zeros((19, H))
    facc = np.zeros((3, H)); facc[0] = eps * g
    epsf = np.full(H, eps)
    nu = (ts - 0.5) / 3
    for _ in range(int(60 * H * H / nu)):
        df = orc.lbm_collide_stream(P, df, epsf, facc)
    rho = 1 + df.sum(0)
    ub = (C[:, 0] @ df + 0.5 * facc[0]) / rho
    z = np.arange(H) + 0.5
    exact = eps * g / (2 * nu) * (z * (H - z) + (16 * (ts - 0.5) ** 2 - 3) / 12)
    assert np.abs(ub - exact).max() < 1e-11 * exact.max()


def test_momentum_budget_with_per_cell_tau(orc):
    n, nc = (6, 5, 4), 120
    rng = np.random.default_rng(3)
    df = 1e-3 * rng.standard_normal((19, nc))
    f = 1e-5 * rng.standard_normal((3, nc))
    e = rng.uniform(0.5, 1.0, nc)
    P = _P(orc, 0.73, eilers=1, les=1, n=n)
    out = orc.lbm_collide_stream(P, df, e, f)
    assert abs(out.sum() - df.sum()) < 1e-15
    np.testing.assert_allclose(C.T @ out.sum(1), C.T @ df.sum(1) + f.sum(1), rtol=1e-12, atol=1e-17)
    # and the per-cell tau changed the result
    P0 = _P(orc, 0.73, eilers=0, les=0, n=n)
    assert np.abs(orc.lbm_collide_stream(P0, df, e, f) - out).max() > 1e-6 * np.abs(df).max()


def test_coupled_momentum_budget_with_all_models(orc):
    """Full coupled steps with lift, the Eilers viscosity and the LES on
    together: total momentum still changes only by the external impulses
    (body force, pressure force, submerged weight)."""
    c = I.case_settling(9, 12, 0.2, 0.8, 2.5, precision="fp64")
    c.particles.u[:] = np.random.default_rng(6).normal(size=c.particles.u.shape) * 1e-3
    o = orc.Oracle(c.params.copy(use_lift=1, use_eilers=1, use_les=1), c.particles)
    m = c.particles.rho_p * np.pi * c.particles.d ** 3 / 6
    for _ in range(5):
        d0 = o.diagnostics()
        r = o.step(1, aux=True)
        assert r["status"] == 0
        d1 = o.diagnostics()
        dP = (d1["mom_fluid"] + d1["mom_part"]) - (d0["mom_fluid"] + d0["mom_part"])
        ext = r["impulse_fb"] + r["impulse_pr"] + r["impulse_gb"]
        scale = np.abs(m[:, None] * o.state.u).sum() + 1e-3 * np.abs(r["impulse_gb"]).sum()
        assert np.abs(dP - ext).max() < 1e-11 * scale, (dP, ext)
        assert abs(d1["mass_dev"] - d0["mass_dev"]) < 1e-13
