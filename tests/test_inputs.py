"""The seeded input generator: reproducible, non-overlapping, right sizes."""
import numpy as np

from paper_1711_00336_amd import inputs as I


def _min_gap(p, box, periodic):
    I_, J, dv = I._neighbour_pairs(p.x, box, periodic, float(p.d.max()),
                                   lambda i, j: 0.5 * (p.d[i] + p.d[j]))
    return len(I_)


def test_splitmix64_reference_values():
    # SplitMix64 with state 0 (Steele et al. 2014): first outputs
    z = I.splitmix64(0, 0, np.arange(3))
    assert [hex(int(v)) for v in z] == ["0xe220a8397b1dcdaf", "0x6e789e6aa1b965f4", "0x6c45d188009454f"]


def test_small_walled_case():
    c = I.case_small_walled(0)
    p = c.particles
    assert p.n == 64 and np.all(p.d == 0.5)
    assert _min_gap(p, c.params.n, c.params.periodic) == 0
    assert np.all(p.x[:, 2] > 0.25) and np.all(p.x[:, 2] < 64 - 0.25)
    c2 = I.case_small_walled(0)
    assert np.array_equal(c2.particles.x, p.x)
    assert not np.array_equal(I.case_small_walled(1).particles.x, p.x)


def test_dilute_periodic_fraction():
    c = I.case_dilute_periodic(0, n=32)
    p = c.particles
    eps = (np.pi / 6 * p.d ** 3).sum() / 32 ** 3
    assert abs(eps - 0.05) < 1e-3
    assert _min_gap(p, c.params.n, c.params.periodic) == 0
    assert np.all((p.x >= 0) & (p.x < 32))


def test_dense_polydisperse_relaxed():
    c = I.case_dense_walled(0, n=(12, 12, 16), eps_p=0.4)
    p = c.particles
    eps = (np.pi / 6 * p.d ** 3).sum() / (12 * 12 * 16)
    assert abs(eps - 0.4) < 2e-3
    assert p.d.min() >= 0.9 and p.d.max() <= 1.1
    I_, J, dv = I._neighbour_pairs(p.x, c.params.n, c.params.periodic, float(p.d.max()),
                                   lambda i, j: 0.5 * (p.d[i] + p.d[j]))
    if len(I_):
        ov = 0.5 * (p.d[I_] + p.d[J]) - np.sqrt((dv ** 2).sum(1))
        assert ov.max() < 1e-3 * p.d.min()


def test_dense_packing_does_not_depend_on_the_thread_count():
    """The overlap removal visits cells in 27 colour classes whose
    neighbourhoods are disjoint, so its result is the same with one OpenMP
    thread (as in the parallel input generators) and with several."""
    from paper_1711_00336_amd import inputs as I
    try:
        I.set_relax_threads(1)
        a = I.case_dense_walled(3, n=(24, 24, 32), eps_p=0.4, precision="fp64").particles.x
        I.set_relax_threads(4)
        b = I.case_dense_walled(3, n=(24, 24, 32), eps_p=0.4, precision="fp64").particles.x
    finally:
        I.set_relax_threads(0)
    assert np.array_equal(a, b)
