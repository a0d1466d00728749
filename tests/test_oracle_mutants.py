"""Planted mistakes: copies of the oracle with one plausible error each must
fail at least one pin of test_oracle_gradient_drag_pins.py. This shows the
pins of the lattice gradient (Sec. 3.2.3) and of the Tenneti drag (Table 1)
are sharp enough to catch a transposed index, a dropped or flipped sign, a
wrong weight, power or coefficient. Each mutant is a textual edit of the
oracle source, compiled with gcc into the test's temporary directory.
"""
import pytest

from tests import test_oracle_gradient_drag_pins as G

MUTANTS = {
    "gradient transposed":
        ("G[a][b] += WQ(q) * CV[q][a] * (sg * un[b * nc + nb]);",
         "G[b][a] += WQ(q) * CV[q][a] * (sg * un[b * nc + nb]);"),
    "convective term contracted on the wrong index":
        ("conv += un[a * nc + c] * (3.0 * G[a][b]);", "conv += un[a * nc + c] * (3.0 * G[b][a]);"),
    "grad P sign":
        ("gp[a] += WQ(q) * CV[q][a] * drho[nb];", "gp[a] -= WQ(q) * CV[q][a] * drho[nb];"),
    "grad P missing the diagonal weights":
        ("gp[a] += WQ(q) * CV[q][a] * drho[nb];", "gp[a] += (q <= 6 ? 3.0 * WQ(q) : 0.0) * CV[q][a] * drho[nb];"),
    "scalar ghost negated like a velocity":
        ("gp[a] += WQ(q) * CV[q][a] * drho[nb];", "gp[a] += WQ(q) * CV[q][a] * (sg * drho[nb]);"),
    "velocity ghost not negated":
        ("*sign = -*sign;", "*sign = *sign;"),
    "(1-eps)^3 for (1-eps)^4":
        ("/ (e1 * e1 * e1 * e1);", "/ (e1 * e1 * e1);"),
    "eps^(1/2) for eps^(1/3)":
        ("cbrt(ep)", "sqrt(ep)"),
    "0.48 coefficient":
        ("0.48 * (ep > 0.0", "0.84 * (ep > 0.0"),
    "eps^2 for eps^3 in the inertial term":
        ("double B = ep * ep * ep * Re", "double B = ep * ep * Re"),
    "0.95 coefficient":
        ("Re * (0.95 + 0.61", "Re * (0.59 + 0.61"),
    "Reynolds number without (1-eps)":
        ("double Re = (1.0 - ep) * rho_f * d * wn / mu;", "double Re = rho_f * d * wn / mu;"),
    "Reynolds number with the diameter squared":
        ("double Re = (1.0 - ep) * rho_f * d * wn / mu;", "double Re = (1.0 - ep) * rho_f * d * d * wn / mu;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(orc, tmp_path, name):
    old, new = MUTANTS[name]
    src = orc.source()
    assert src.count(old) == 1, f"mutation site not unique: {old}"
    path = orc.build_variant(src.replace(old, new), str(tmp_path / "liborc_mutant.so"))
    caught = []
    with orc.using_library(path):
        for pin in G.PINS:
            try:
                pin(orc)
            except AssertionError:
                caught.append(pin.__name__)
    assert caught, f"no pin catches the planted mistake '{name}'"
