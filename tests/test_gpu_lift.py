"""Shear-induced lift (Table 1) with the lattice curl (Sec. 3.2.3) on the GPU
against the FP64 oracle, through the C ABI.

  * one coupled step from an identical state, every state array within 1e-12
    (FP64) or 1e-5 (FP32 deviations) of its largest oracle value, on a walled
    domain, a periodic settling box and a dense box with random velocities;
  * the curl field and the lift of every particle against the oracle's own
    values of the same step (FP64, 1e-12);
  * the per-particle lift pass (gather variant 3) and the LDS-tiled one give
    the same bits;
  * reading the curl or the lift of a domain without lift is an E_STATE error.
"""
import numpy as np
import pytest

from paper_1711_00336_amd import inputs as I
from tests.parity_util import compare_states, load_oracle_state, rel_err, warm_oracle

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def L():
    from paper_1711_00336_amd import lbdem
    lbdem.lib()
    return lbdem


def _say(msg):
    print(msg, flush=True)


def _lift(case):
    return I.Case(case.name + "-lift", case.params.copy(use_lift=1), case.particles, case.seed)


def _stirred(case, seed, scale):
    rng = np.random.default_rng(seed)
    case.particles.u[:] = rng.normal(size=case.particles.u.shape) * scale
    case.particles.w[:] = rng.normal(size=case.particles.w.shape) * scale
    return case


def _cases():
    dense_prm = I.Params(n=(14, 12, 16), periodic=(1, 1, 0), tau=0.7, gravity=(0, 0, -1e-5), e_n=0.9,
                         mu_c=0.25, T_c=0.0, h_c=1.0, n_int=3, n_dem=4, precision="fp64", use_lift=1)
    return {
        "walled": lambda: _stirred(_lift(I.case_small_walled(2)), 1, 1e-3),
        "periodic": lambda: _stirred(_lift(I.case_settling(5, 21, 0.1, 0.8, 2.5, precision="fp64")), 3, 1e-3),
        "dense": lambda: _stirred(I.Case("dense-lift", dense_prm, I.make_particles(4, dense_prm, 0.35, 0.9, 1.1, 2.5),
                                         4), 11, 2e-3),
    }


@pytest.mark.parametrize("name", ["walled", "periodic", "dense"])
def test_lift_step_parity_fp64(L, name):
    case = _cases()[name]()
    _say(f"case {case.name} n {case.params.n} np {case.particles.n}")
    o = warm_oracle(case, 2)
    worst = {}
    with L.Domain(case.params) as dom:
        for s in range(2):
            load_oracle_state(dom, o.state)
            dom.step(1)
            r = o.step(1, aux=True)
            assert r["status"] == 0
            errs, bad = compare_states(dom.lbdem_get_state(), o.state, case.params, TOL64)
            for k, v in errs.items():
                worst[k] = max(worst.get(k, 0.0), v)
            assert not bad, (s, errs)
    # the lift is really active in the compared steps
    assert np.abs(r["F_l"]).max() > 1e-5 * np.abs(r["F_d"]).max()
    _say(f"  worst rel errors {worst}")


def test_lift_step_parity_fp32dev(L):
    case = _stirred(_lift(I.case_settling(5, 24, 0.12, 0.8, 2.5, precision="fp32dev")), 3, 1e-3)
    _say(f"case {case.name} fp32dev np {case.particles.n}")
    o = warm_oracle(case, 2)
    with L.Domain(case.params) as dom:
        load_oracle_state(dom, o.state)
        dom.step(1)
        o.step(1)
        errs, bad = compare_states(dom.lbdem_get_state(), o.state, case.params, 1e-5)
    _say(f"  rel errors {errs}")
    assert not bad, errs


@pytest.mark.parametrize("walled", [False, True])
def test_curl_field_and_lift_match_oracle(L, walled):
    """The curl of u_f at the last subcycle's start and the last subcycle's
    lift and F_const of every particle, against the oracle's values."""
    case = _stirred(_lift(I.case_small_walled(4)), 2, 1e-3) if walled else \
        _stirred(_lift(I.case_settling(13, 22, 0.12, 0.8, 2.5, precision="fp64")), 5, 1e-3)
    o = warm_oracle(case, 2)
    with L.Domain(case.params) as dom:
        load_oracle_state(dom, o.state)
        dom.step(1)
        aux = o.step(1, aux=True)
        assert aux["status"] == 0
        got = {"curl": dom.lbdem_read_field(L.FIELD_CURL), "F_l": dom.lbdem_read_particle_lift(),
               "F_const": dom.lbdem_read_particle_forces()["F_const"]}
    errs = {k: rel_err(got[k], aux[k]) for k in got}
    _say(f"  curl/lift rel errors {errs}")
    assert np.abs(aux["curl"]).max() > 0 and np.abs(aux["F_l"]).max() > 0
    assert all(v <= TOL64 for v in errs.values()), errs


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_lift_pass_variants_bitwise_equal(L, precision):
    """Gather variant 3 runs the lift pass one thread per particle from global
    memory; the others use LDS tiles. Same sums in the same order: same bits."""
    case = _stirred(_lift(I.case_settling(7, 26, 0.12, 0.8, 2.5, precision=precision)), 9, 1e-3)
    _say(f"case {case.name} {precision} np {case.particles.n}")
    o = warm_oracle(case, 1)
    states = []
    for v in (0, 3):
        with L.Domain(case.params) as dom:
            dom.lbdem_set_gather_variant(v)
            load_oracle_state(dom, o.state)
            dom.step(2)
            states.append((dom.lbdem_get_state(), dom.lbdem_read_particle_lift()))
    for k, a in states[0][0].items():
        assert np.array_equal(np.asarray(states[1][0][k]), np.asarray(a)), k
    assert np.array_equal(states[0][1], states[1][1])


def test_curl_and_lift_need_lift_on(L):
    case = I.case_small_walled(0)
    with L.Domain(case.params) as dom:
        dom.step(1)
        with pytest.raises(L.LbdemError) as e:
            dom.lbdem_read_field(L.FIELD_CURL)
        assert e.value.status == L.E_STATE
        with pytest.raises(L.LbdemError) as e:
            dom.lbdem_read_particle_lift()
        assert e.value.status == L.E_STATE


@pytest.mark.parametrize("n", [(2, 9, 10), (9, 2, 10)])
def test_lift_thin_periodic_axis(L, n):
    """A periodic axis of 2 cells (x or y) with lift and the per-cell
    relaxation time: the curl's stencil, the kernel stencils and the
    neighbour bins wrap onto themselves (the gathers take their per-cell
    form)."""
    prm = I.Params(n=n, periodic=(1, 1, 0), tau=0.9, gravity=(0, 0, -1e-5), h_c=0.5, n_int=10,
                   precision="fp64", use_lift=1, use_eilers=1, use_les=1)
    parts = I.make_particles(6, prm, 6, 0.5, 0.5, 2.0)
    case = _stirred(I.Case("thin-axis-lift", prm, parts, 6), 4, 1e-3)
    _say(f"case {case.name} n {n} np {case.particles.n}")
    o = warm_oracle(case, 2)
    with L.Domain(case.params) as dom:
        for s in range(2):
            load_oracle_state(dom, o.state)
            dom.step(1)
            r = o.step(1, aux=True)
            assert r["status"] == 0
            errs, bad = compare_states(dom.lbdem_get_state(), o.state, case.params, TOL64)
            assert not bad, (s, errs)
        got = dom.lbdem_read_particle_lift()
    assert np.abs(r["F_l"]).max() > 0
    assert rel_err(got, r["F_l"]) <= TOL64
    _say(f"  rel errors {errs}")
