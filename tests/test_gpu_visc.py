"""Per-cell relaxation time (Eilers suspension viscosity, Smagorinsky LES;
Sec. 3.2.2 and Alg. 1) on the GPU against the FP64 oracle, through the C ABI:
one coupled step from an identical state, every state array within 1e-12
(FP64) or 1e-5 (FP32 deviations) of its largest oracle value.

Cases: a settling box with stirred particles (the Eilers term varies with the
local solid fraction), and a walled pure-fluid box with strong random
non-equilibrium PDFs (a large subgrid term), each with Eilers, LES and both.
"""
import numpy as np
import pytest

from paper_1711_00336_amd import inputs as I
from tests.parity_util import compare_states, load_oracle_state, warm_oracle

pytestmark = pytest.mark.gpu

MODELS = {"eilers": dict(use_eilers=1), "les": dict(use_les=1), "both": dict(use_eilers=1, use_les=1)}


@pytest.fixture(scope="module")
def L():
    from paper_1711_00336_amd import lbdem
    lbdem.lib()
    return lbdem


def _say(msg):
    print(msg, flush=True)


def _settling(precision, model):
    c = I.case_settling(6, 22, 0.15, 0.8, 2.5, precision=precision)
    rng = np.random.default_rng(8)
    c.particles.u[:] = rng.normal(size=c.particles.u.shape) * 1e-3
    return I.Case(c.name + "-" + model, c.params.copy(**MODELS[model]), c.particles, c.seed)


def _fluid(precision, model):
    prm = I.Params(n=(27, 19, 21), periodic=(1, 0, 0), tau=0.62, body_force=(2e-6, -1e-6, 3e-6), n_int=2,
                   precision=precision, **MODELS[model])
    empty = I.Particles(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    return I.Case("fluid-" + model, prm, empty, 0)


def _parity(L, case, tol, perturb=None, nsteps=2):
    _say(f"case {case.name} {case.params.precision} n {case.params.n} np {case.particles.n}")
    o = warm_oracle(case, 1 if perturb is None else 0, perturb)
    worst = {}
    with L.Domain(case.params) as dom:
        for s in range(nsteps):
            load_oracle_state(dom, o.state)
            dom.step(1)
            assert o.step(1)["status"] == 0
            errs, bad = compare_states(dom.lbdem_get_state(), o.state, case.params, tol)
            for k, v in errs.items():
                worst[k] = max(worst.get(k, 0.0), v)
            assert not bad, (s, errs)
    _say(f"  worst rel errors {worst}")


@pytest.mark.parametrize("model", list(MODELS))
def test_settling_step_parity_fp64(L, model):
    _parity(L, _settling("fp64", model), 1e-12)


@pytest.mark.parametrize("model", list(MODELS))
def test_fluid_step_parity_fp64(L, model):
    nc = 27 * 19 * 21
    _parity(L, _fluid("fp64", model), 1e-12, perturb=I.perturbed_state(5, nc, 3e-3))


@pytest.mark.parametrize("kind", ["settling", "fluid"])
def test_step_parity_fp32dev_both(L, kind):
    if kind == "settling":
        _parity(L, _settling("fp32dev", "both"), 1e-5, nsteps=1)
    else:
        _parity(L, _fluid("fp32dev", "both"), 1e-5, perturb=I.perturbed_state(5, 27 * 19 * 21, 3e-3), nsteps=1)


def test_models_change_the_step(L):
    """The per-cell relaxation time is really applied: with both models the
    PDFs after one step differ from the constant-tau step well above the
    parity tolerance."""
    nc = 27 * 19 * 21
    pert = I.perturbed_state(5, nc, 3e-3)
    out = []
    for model in (None, "both"):
        case = _fluid("fp64", "both")
        if model is None:
            case.params = case.params.copy(use_eilers=0, use_les=0)
        o = warm_oracle(case, 0, pert)
        with L.Domain(case.params) as dom:
            load_oracle_state(dom, o.state)
            dom.step(1)
            out.append(dom.lbdem_get_state()["df"])
    assert np.abs(out[0] - out[1]).max() > 1e-6 * np.abs(out[0]).max()
