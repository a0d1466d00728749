"""Failure detection through the C ABI on the GPU, each condition forced
from the host with inputs every kernel handles normally (no particles where
the fluid state is made non-finite, so no index is ever derived from it):

  * lbdem_add_particles rejects particles the explicit-coupling estimate
    calls unstable (E_UNSTABLE) and adds none of them;
  * a cell velocity above 0.1 (outside the low-Mach range of the
    equilibrium) is flagged by the collision and surfaces at lbdem_sync;
  * a non-finite PDF is flagged the same way;
  * centres on a wall plane are rejected (E_INVALID), just inside accepted.
"""
import numpy as np
import pytest

from paper_1711_00336_amd import inputs as I
from tests.test_stability_checks import _uniform_flow

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1711_00336_amd import lbdem
    lbdem.lib()
    return lbdem


def _say(msg):
    print(msg, flush=True)


def test_add_particles_applies_the_stability_estimate(L):
    case = I.case_small_walled(0)
    _say("add_particles of the small walled workload at n_int = 1 and 10")
    with L.Domain(case.params.copy(n_int=1)) as dom:
        with pytest.raises(L.LbdemError) as e:
            dom.add(case.particles)
        assert e.value.status == L.E_UNSTABLE
        assert dom.num_particles() == 0
    with L.Domain(case.params) as dom:
        dom.add(case.particles)
        assert dom.num_particles() == case.particles.n


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_fast_flow_is_flagged(L, precision):
    n = (8, 6, 4)
    prm = I.Params(n=n, periodic=(1, 1, 1), precision=precision, n_int=2)
    nc = n[0] * n[1] * n[2]
    for speed, flagged in ((0.06, False), (0.12, True)):
        _say(f"{precision}: uniform flow |u| = {speed}, no particles")
        with L.Domain(prm) as dom:
            dom.lbdem_set_state(_uniform_flow(n, [speed, 0.0, 0.0]), np.zeros((3, nc)), 0, np.zeros((0, 3)),
                                np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0))
            dom.lbdem_step(2)
            if flagged:
                with pytest.raises(L.LbdemError) as e:
                    dom.lbdem_sync()
                assert e.value.status == L.E_UNSTABLE and "Mach" in str(e.value)
            else:
                dom.lbdem_sync()


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_nonfinite_pdf_is_flagged(L, precision):
    n = (8, 6, 4)
    prm = I.Params(n=n, periodic=(1, 1, 0), precision=precision, n_int=2)
    nc = n[0] * n[1] * n[2]
    df = _uniform_flow(n, [0.01, 0.0, 0.0])
    df[11, 37] = np.nan
    _say(f"{precision}: one NaN PDF, no particles")
    with L.Domain(prm) as dom:
        dom.lbdem_set_state(df, np.zeros((3, nc)), 0, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)),
                            np.zeros((0, 3)), np.zeros(0), np.zeros(0))
        dom.lbdem_step(1)
        with pytest.raises(L.LbdemError) as e:
            dom.lbdem_sync()
        assert e.value.status == L.E_UNSTABLE and "non-finite fluid" in str(e.value)


def test_wall_overlap_rule(L):
    prm = I.Params(n=(8, 8, 8), periodic=(1, 1, 0), precision="fp64")
    with L.Domain(prm) as dom:
        for z in (0.0, 8.0, -1e-9):
            with pytest.raises(L.LbdemError) as e:
                dom.lbdem_add_particles(np.array([[1.0, 1.0, z]]), np.zeros((1, 3)), np.zeros((1, 3)),
                                        np.array([0.5]), np.array([2.0]))
            assert e.value.status == L.E_INVALID
        dom.lbdem_add_particles(np.array([[1.0, 1.0, 1e-9], [2.0, 2.0, 8.0 - 1e-9]]), np.zeros((2, 3)),
                                np.zeros((2, 3)), np.array([0.5, 0.5]), np.array([2.0, 2.0]))
        assert dom.num_particles() == 2
