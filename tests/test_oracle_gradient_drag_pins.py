"""Pins of the oracle's lattice gradient and of its Tenneti drag away from
the limits, against closed forms the paper's definitions fix.

Lattice gradient (Sec. 3.2.3): grad phi ~ (1/c_s^2) sum_q w_q c_q phi(x+c_q).
On the D3Q19 stencil the links with c_a = +1 carry a total weight of 1/6, so
for a field that varies along axis a only, d phi/dx_a is read as
(phi(x+e_a) - phi(x-e_a))/2 and a sine of wave number k differentiates to
sin(k) cos(k x) instead of k cos(k x). Fields that vary along another axis
cancel out of component a exactly. The oracle uses the operator in two
places, both read out through its auxiliary outputs after one step:
  * grad P = (1/c_s^2) sum_q w_q c_q P(x+c_q) with P = c_s^2 rho (Eq. MacVel),
  * the convective part (u_f . grad) u_f of Du_f/Dt (Table 1, added mass),
    which is all of Du_f/Dt at the first step (no time derivative yet).
Walls use the ghost rule of the oracle's reading: a scalar keeps the value of
the mirrored cell, a velocity flips its sign (no slip on the half-way plane).

Tenneti drag (Table 1): F_d = 3 pi d mu f(Re, eps) w with the printed
f = (1-eps)^2 [C_d0/(1-eps)^3 + 5.81 eps/(1-eps)^3 + 0.48 eps^(1/3)/(1-eps)^4
+ eps^3 Re (0.95 + 0.61 eps^3/(1-eps)^2)] and Re = (1-eps) d |w| / mu.
Pinned by limits each term fixes on its own (dilute, close-packed, inertial)
and by values evaluated by hand.

Each pin is a function that raises AssertionError; test_oracle_mutants.py
plants mistakes in copies of the oracle and checks that a pin catches each.
"""
import math

import numpy as np
import pytest

from paper_1711_00336_amd import inputs as I

# D3Q19 (standard set; the paper does not print it), written out here
C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
              [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], float)


def _empty():
    z = np.zeros((0, 3))
    return I.Particles(z, z, z, np.zeros(0), np.zeros(0))


def _centres(n):
    """cell-centre coordinates x, y, z of every cell (flat index x fastest)"""
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    return (i.ravel() + 0.5, j.ravel() + 0.5, k.ravel() + 0.5)


def _state(n, drho, u):
    """PDF deviations whose moments are rho - 1 = drho and j = u (rest
    deviation carries drho, each axis pair carries +-u_a/2)."""
    nc = n[0] * n[1] * n[2]
    df = np.zeros((19, nc))
    df[0] = drho
    for a in range(3):
        df[1 + 2 * a] = 0.5 * u[a]
        df[2 + 2 * a] = -0.5 * u[a]
    return df


def _first_step_aux(O, prm, df):
    o = O.Oracle(prm, _empty(), df=df)
    r = o.step(1, aux=True)
    assert r["status"] == 0
    return r


# ------------------------------------------------------------ pins (functions)
def pin_gradp_sinusoid(O):
    """rho = 1 + sum_a A_a sin(k_a x_a): (grad P)_a = A_a sin(k_a) cos(k_a x_a)/3
    exactly (c_s^2 times the lattice derivative), each component seeing only
    its own axis; and the closed form of a product field, which depends on
    the face-diagonal weights."""
    n = (8, 6, 10)
    prm = I.Params(n=n, periodic=(1, 1, 1), n_int=1)
    x = _centres(n)
    A = (3e-3, -2e-3, 1.5e-3)
    k = [2 * math.pi / n[a] for a in range(3)]
    drho = sum(A[a] * np.sin(k[a] * x[a]) for a in range(3))
    r = _first_step_aux(O, prm, _state(n, drho, np.zeros((3, drho.size))))
    want = np.stack([A[a] * math.sin(k[a]) * np.cos(k[a] * x[a]) / 3.0 for a in range(3)])
    err = np.abs(r["gradp"] - want).max()
    assert err <= 1e-15, f"grad P off its closed form by {err:.3e}"
    # a product field rho - 1 = B sin(k_x x) sin(k_y y) also weighs the face
    # diagonals: the c_x = +1 links sum to sin(k_y y) (1/9 + cos(k_y)/18), so
    # (grad P)_x = B sin(k_x) cos(k_x x) sin(k_y y) (2 + cos k_y)/9 and
    # symmetrically for y; an axis-only stencil would give (2 + 1)/9
    B = 4e-3
    drho = B * np.sin(k[0] * x[0]) * np.sin(k[1] * x[1])
    r = _first_step_aux(O, prm, _state(n, drho, np.zeros((3, drho.size))))
    want = np.stack([B * math.sin(k[0]) * np.cos(k[0] * x[0]) * np.sin(k[1] * x[1]) * (2 + math.cos(k[1])) / 9,
                     B * math.sin(k[1]) * np.cos(k[1] * x[1]) * np.sin(k[0] * x[0]) * (2 + math.cos(k[0])) / 9,
                     np.zeros_like(drho)])
    err = np.abs(r["gradp"] - want).max()
    assert err <= 1e-15, f"grad P of a product field off its closed form by {err:.3e}"


def pin_convective_sinusoid(O):
    """u = (U0 + U1 sin(k_y y), U2 sin(k_z z), U3 sin(k_x x)), rho = 1, first
    step: Du_f/Dt = (u . grad_L) u =
        (u_y U1 sin(k_y) cos(k_y y), u_z U2 sin(k_z) cos(k_z z), u_x U3 sin(k_x) cos(k_x x)).
    Each component needs the derivative of a different component along a
    different axis, so a transposed gradient (u_a d_b u_a) gives other values."""
    n = (8, 6, 10)
    prm = I.Params(n=n, periodic=(1, 1, 1), n_int=1)
    x = _centres(n)
    kx, ky, kz = (2 * math.pi / n[a] for a in range(3))
    U0, U1, U2, U3 = 2e-3, 1e-3, -1.5e-3, 2.5e-3
    u = np.stack([U0 + U1 * np.sin(ky * x[1]), U2 * np.sin(kz * x[2]), U3 * np.sin(kx * x[0])])
    r = _first_step_aux(O, prm, _state(n, np.zeros(u.shape[1]), u))
    want = np.stack([u[1] * U1 * math.sin(ky) * np.cos(ky * x[1]),
                     u[2] * U2 * math.sin(kz) * np.cos(kz * x[2]),
                     u[0] * U3 * math.sin(kx) * np.cos(kx * x[0])])
    err = np.abs(r["dudt"] - want).max() / np.abs(want).max()
    assert err <= 1e-12, f"convective term off its closed form by {err:.3e} (relative)"


def pin_gradient_wall_ghosts(O):
    """Walls at z = 0 and H. A linear density rho - 1 = alpha (z - H/2): the
    mirrored scalar ghost halves the one-sided difference at the wall cells,
    (grad P)_z = alpha/6 there and alpha/3 inside. A shear u_x = gamma z,
    which vanishes on the bottom wall plane, plus a uniform u_z = W: below the
    bottom wall the negated ghost is the shear's linear continuation, so
    d u_x/dz = gamma in every cell but the top one, where the ghost
    -u_x(H - 1/2) gives (-(H - 1/2) - (H - 3/2)) gamma/2 = -(H - 1) gamma;
    (u . grad) u_x = W d u_x/dz. d u_z/dz is W at the bottom wall cell (ghost
    -W below W), -W at the top one and 0 inside, so (u . grad) u_z = W^2,
    -W^2, 0."""
    n = (4, 3, 6)
    H = n[2]
    prm = I.Params(n=n, periodic=(1, 1, 0), n_int=1)
    x = _centres(n)
    kcell = (x[2] - 0.5).astype(int)
    alpha = 1e-3
    drho = alpha * (x[2] - 0.5 * H)
    r = _first_step_aux(O, prm, _state(n, drho, np.zeros((3, drho.size))))
    gz = np.where((kcell == 0) | (kcell == H - 1), alpha / 6.0, alpha / 3.0)
    assert np.abs(r["gradp"][2] - gz).max() <= 1e-17, "scalar ghost rule at the walls"
    assert np.abs(r["gradp"][:2]).max() <= 1e-17
    gamma, W = 2e-4, 3e-4
    u = np.stack([gamma * x[2], np.zeros_like(x[2]), np.full_like(x[2], W)])
    r = _first_step_aux(O, prm, _state(n, np.zeros(u.shape[1]), u))
    want_z = np.where(kcell == 0, W * W, np.where(kcell == H - 1, -W * W, 0.0))
    dudz = np.where(kcell == H - 1, -(H - 1) * gamma, gamma)
    assert np.abs(r["dudt"][0] - W * dudz).max() <= 1e-18, "velocity ghost rule at the walls"
    assert np.abs(r["dudt"][1]).max() <= 1e-20
    assert np.abs(r["dudt"][2] - want_z).max() <= 1e-18


def pin_drag_dilute_limit(O):
    """Re = 0, eps -> 0: f - 1 = 6.81 eps/(1-eps) + 0.48 eps^(1/3)/(1-eps)^2,
    so (f - 1)/eps^(1/3) -> 0.48; fixes the coefficient and the cube root."""
    for e in (1e-9, 1e-12):
        v = (O.drag_factor(0.0, e) - 1.0) / e ** (1.0 / 3.0)
        assert abs(v - 0.48) <= 1e-5, f"dilute limit {v} at eps {e}"


def pin_drag_packed_limit(O):
    """Re = 0, eps -> 1: (1-eps)^2 f -> 0.48 (only the eps^(1/3)/(1-eps)^4
    term survives, against the outer (1-eps)^2)."""
    for e1 in (1e-6, 1e-8):
        v = e1 * e1 * O.drag_factor(0.0, 1.0 - e1)
        assert abs(v - 0.48) <= 1e-4, f"close-packed limit {v} at 1-eps {e1}"


def pin_drag_inertial_slope(O):
    """At fixed eps and Re -> infinity the slope df/dRe tends to
    (1-eps)^2 eps^3 (0.95 + 0.61 eps^3/(1-eps)^2) (the Re^0.687 term's slope
    decays like Re^-0.313)."""
    for e in (0.2, 0.4):
        R = 1e15
        slope = (O.drag_factor(2 * R, e) - O.drag_factor(R, e)) / R
        want = (1 - e) ** 2 * e ** 3 * (0.95 + 0.61 * e ** 3 / (1 - e) ** 2)
        assert abs(slope / want - 1.0) <= 1e-3, f"inertial slope {slope} vs {want} at eps {e}"


def pin_drag_hand_values(O):
    """f(Re = 0) evaluated by hand from the printed correlation."""
    for e, v in ((0.05, 1.5544), (0.3, 4.5743), (0.4, 6.5224), (0.5, 9.3339)):
        got = O.drag_factor(0.0, e)
        assert abs(got - v) <= 6e-5 * v, f"f(0, {e}) = {got}, by hand {v}"


def pin_drag_reynolds_number(O):
    """Re carries (1-eps): at large slip the drag is quadratic,
    |F| -> 3 pi d^2 rho_f (1-eps)^3 eps^3 (0.95 + 0.61 eps^3/(1-eps)^2) |w|^2,
    one power of (1-eps) from Re and two from the correlation's prefactor."""
    d, mu, rho_f, e = 0.9, 0.1, 1.0, 0.3
    w = np.array([0.0, 0.0, 1e13])
    F = O.drag(d, mu, rho_f, e, w)
    want = 3 * math.pi * d * d * rho_f * (1 - e) ** 3 * e ** 3 * (0.95 + 0.61 * e ** 3 / (1 - e) ** 2) * w[2] ** 2
    assert abs(F[2] / want - 1.0) <= 1e-3, f"quadratic drag {F[2]} vs {want}"


PINS = [pin_gradp_sinusoid, pin_convective_sinusoid, pin_gradient_wall_ghosts, pin_drag_dilute_limit,
        pin_drag_packed_limit, pin_drag_inertial_slope, pin_drag_hand_values, pin_drag_reynolds_number]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(orc, pin):
    pin(orc)
