"""Hindered settling configuration (Sec. 4.1 Setup mapped to lattice
units at tau = 0.505 with the Smagorinsky model; spheres settling at
~0.05 cells per step, T_c = dt/2, n_DEM = 50) on the GPU against the FP64
oracle, one coupled step from an identical state, at 1e-12 (the boxes are
16 diameters wide so that the oracle finishes in seconds)."""
import pytest

from paper_1711_00336_amd import inputs as I
from tests.parity_util import compare_states, load_oracle_state, warm_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1711_00336_amd import lbdem
    lbdem.lib()
    return lbdem


@pytest.mark.parametrize("eps", [0.0, 0.1])
def test_hindered_settling_step_parity(L, eps):
    case = I.case_hindered_settling(0, eps, edge_d=16)
    print(f"case {case.name} np {case.particles.n}", flush=True)
    o = warm_oracle(case, 2)
    with L.Domain(case.params) as dom:
        for _ in range(2):
            load_oracle_state(dom, o.state)
            dom.step(1)
            assert o.step(1)["status"] == 0
            errs, bad = compare_states(dom.lbdem_get_state(), o.state, case.params, 1e-12)
            assert not bad, errs
    print(f"  rel errors {errs}", flush=True)
