"""Batching and serving forms: every domain's result is the same alone, in a
batch and in a served mix (bitwise: all kernels are deterministic), the
autotuner does not change results, admission respects the HBM budget."""
import numpy as np
import pytest

from paper_1711_00336_amd import inputs as I
from tests.parity_util import compare_states, load_oracle_state, warm_oracle

pytestmark = pytest.mark.gpu

KEYS = ("df", "uprev", "x", "u", "w", "a")


@pytest.fixture(scope="module")
def L():
    from paper_1711_00336_amd import lbdem
    lbdem.lib()
    return lbdem


def _say(msg):
    print(msg, flush=True)


def _cases():
    out = []
    p = I.Params(n=(24, 20, 28), periodic=(1, 1, 0), tau=0.8, n_int=3, h_c=0.5, precision="fp64")
    out.append(I.Case("walled-fp64", p, I.make_particles(1, p, 40, 0.5, 0.7, 2.5), 1))
    out.append(I.case_settling(2, 20, 0.1, 0.8, 2.5, precision="fp32dev"))
    c = I.case_settling(3, 16, 0.3, 0.8, 1.5, precision="fp64", n_int=5, tau=I.SWEEP_TAU)
    out.append(c)
    p = I.Params(n=(30, 18, 22), periodic=(1, 1, 0), tau=0.7, n_int=4, h_c=0.9, precision="fp32dev")
    out.append(I.Case("walled-fp32", p, I.make_particles(4, p, 0.05, 0.8, 0.9, 3.0), 4))
    p = I.Params(n=(12, 12, 12), periodic=(1, 1, 1), tau=0.9, body_force=(1e-6, 0, 0), precision="fp64")
    out.append(I.Case("empty", p, I.Particles(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)),
                                               np.zeros(0), np.zeros(0)), 0))
    return out


def _alone(L, case, nsteps):
    with L.Domain(case.params) as d:
        if case.particles.n:
            d.add(case.particles)
        d.step(nsteps)
        return d.lbdem_get_state()


@pytest.mark.parametrize("tune", [False, True])
def test_batch_domains_equal_alone(L, tune):
    cases = _cases()
    _say("batch of " + ", ".join(f"{c.name}{c.params.n}" for c in cases) + f" autotune={tune}")
    with L.Batch([c.params for c in cases]) as b:
        for dom, c in zip(b.domains, cases):
            if c.particles.n:
                dom.add(c.particles)
        if tune:
            _say(f"  tile variants {b.lbdem_batch_autotune()}")
        b.step(2)
        b.step(1)
        got = [d.lbdem_get_state() for d in b.domains]
    for c, g in zip(cases, got):
        a = _alone(L, c, 3)
        for k in KEYS:
            assert np.array_equal(a[k], g[k]), (c.name, k)
        assert g["step"] == 3


def test_batch_domain_parity_vs_oracle(L):
    cases = _cases()[:3]
    o = warm_oracle(cases[0], 2)
    with L.Batch([c.params for c in cases]) as b:
        for dom, c in zip(b.domains[1:], cases[1:]):
            dom.add(c.particles)
        load_oracle_state(b.domains[0], o.state)
        b.step(1)
        o.step(1)
        errs, bad = compare_states(b.domains[0].lbdem_get_state(), o.state, cases[0].params, 1e-12)
    _say(f"  batch domain vs oracle {errs}")
    assert not bad, errs


def _plain_ups(L, case, steps, avg_from, chunk):
    """The plain per-domain path with the server's sampling of <u_pS>."""
    with L.Domain(case.params) as d:
        d.add(case.particles)
        done, s, n = 0, 0.0, 0
        while done < steps:
            k = min(chunk, steps - done)
            d.step(k)
            done += k
            if done > avg_from:
                s += d.lbdem_diagnostics()["u_ps"]
                n += 1
        return s / n, d.lbdem_diagnostics()


def test_server_result_same_alone_and_in_mix(L):
    target = I.case_settling(11, 20, 0.08, 0.8, 2.5, precision="fp32dev")
    others = [I.case_settling(20 + i, e, eps, 0.8, 2.0, precision="fp32dev", tau=I.SWEEP_TAU)
              for i, (e, eps) in enumerate([(24, 0.2), (16, 0.05), (28, 0.1), (18, 0.3), (22, 0.02)])]
    steps, avg_from, chunk = 60, 20, 10
    with L.Server(8 << 30, max_slots=16, chunk_steps=chunk) as srv:
        t = srv.lbdem_server_submit(target.params, target.particles, steps, avg_from)
        alone = srv.wait(t)
    with L.Server(8 << 30, max_slots=16, chunk_steps=chunk) as srv:
        tk = [srv.lbdem_server_submit(c.params, c.particles, steps + 10 * i, avg_from) for i, c in enumerate(others[:3])]
        t = srv.lbdem_server_submit(target.params, target.particles, steps, avg_from)
        tk += [srv.lbdem_server_submit(c.params, c.particles, steps, avg_from) for c in others[3:]]
        mix = srv.wait(t)
        rest = [srv.wait(x) for x in tk]
    assert alone["status"] == 0 and mix["status"] == 0 and all(r["status"] == 0 for r in rest)
    _say(f"  alone u_ps {alone['u_ps']:.9e} mix {mix['u_ps']:.9e}")
    assert alone["u_ps"] == mix["u_ps"] and alone["mean_eps_f"] == mix["mean_eps_f"]
    assert np.array_equal(alone["mom"], mix["mom"])
    ups, dg = _plain_ups(L, target, steps, avg_from, chunk)
    assert ups == alone["u_ps"] and dg["mean_eps_f"] == alone["mean_eps_f"]


def test_server_admission_by_budget_and_rejection(L):
    cases = [I.case_settling(30 + i, 16, 0.05, 0.8, 2.5, precision="fp32dev") for i in range(4)]
    # budget for exactly one such domain at a time
    with L.Server(48 << 20, max_slots=8, chunk_steps=5) as srv:
        tks = [srv.lbdem_server_submit(c.params, c.particles, 20, 0) for c in cases]
        peak = 0
        while True:
            st = srv.lbdem_server_stats()
            peak = max(peak, st["active"])
            res = [srv.lbdem_server_poll(t) for t in tks]
            if all(r is not None for r in res):
                break
        assert peak == 1
        assert all(r["status"] == 0 for r in res)
        # admitted in submission order, one after another
        adm = [r["t_admit"] for r in res]
        assert adm == sorted(adm)
        big = I.case_settling(40, 96, 0.05, 0.8, 2.5, precision="fp32dev")
        with pytest.raises(L.LbdemError) as e:
            srv.lbdem_server_submit(big.params, big.particles, 10, 0)
        assert e.value.status == L.E_INVALID


def test_server_cancel(L):
    c = I.case_settling(50, 20, 0.05, 0.8, 2.5, precision="fp32dev")
    with L.Server(8 << 30, max_slots=1, chunk_steps=5) as srv:
        t1 = srv.lbdem_server_submit(c.params, c.particles, 400, 0)
        t2 = srv.lbdem_server_submit(c.params, c.particles, 10, 0)
        assert srv.lbdem_server_cancel(t2) == L.OK
        assert srv.lbdem_server_cancel(t1) == L.OK
        r1, r2 = srv.wait(t1), srv.wait(t2)
        assert r1["status"] == L.E_STATE and r2["status"] == L.E_STATE
        assert r1["steps_done"] < 400


def test_server_unstable_request_fails_alone(L):
    """A request in the unstable corner of the explicit coupling (tau = 0.7,
    light crowded spheres: the FP64 oracle diverges within 50 steps) ends
    with LBDEM_E_UNSTABLE and frees its memory and slot; a request running
    beside it is unaffected (its result equals the same request alone)."""
    bad = I.case_settling(23, 18, 0.3, 0.8, 2.0, precision="fp32dev", tau=0.7)
    good = I.case_settling(11, 20, 0.08, 0.8, 2.5, precision="fp32dev")
    with L.Server(8 << 30, max_slots=4, chunk_steps=10) as srv:
        tg = srv.lbdem_server_submit(good.params, good.particles, 60, 20)
        alone = srv.wait(tg)
    with L.Server(8 << 30, max_slots=4, chunk_steps=10) as srv:
        tb = srv.lbdem_server_submit(bad.params, bad.particles, 300, 0)
        tg = srv.lbdem_server_submit(good.params, good.particles, 60, 20)
        rb, rg = srv.wait(tb), srv.wait(tg)
        st = srv.lbdem_server_stats()
    _say(f"  unstable request: status {rb['status']} after {rb['steps_done']} steps")
    assert rb["status"] == L.E_UNSTABLE and rb["steps_done"] < 300
    assert rg["status"] == 0 and rg["u_ps"] == alone["u_ps"]
    assert st["active"] == 0 and st["queued"] == 0 and st["bytes"] == 0


def test_served_results_match_the_fp64_oracle(L):
    """Served FP32-deviation solves against the FP64 oracle on a sample of
    small requests (edges 16-20, solid fractions 0.05-0.2, the serving tau),
    served together in one mix: <u_pS> sampled at the same chunk ends within
    the FP32 settling tolerance (1e-3 relative), <eps_f> within 1e-6, total
    momentum within 1e-6 of sum m|u_p| + sum rho|u_bar|."""
    from oracle import oracle as O
    reqs = [I.case_settling(61, 16, 0.1, 0.8, 2.5, precision="fp32dev", tau=I.SWEEP_TAU),
            I.case_settling(62, 20, 0.05, 0.7, 2.0, precision="fp32dev", tau=I.SWEEP_TAU),
            I.case_settling(63, 18, 0.2, 0.9, 3.0, precision="fp32dev", tau=I.SWEEP_TAU)]
    steps, avg_from, chunk = 120, 40, 20
    _say("served mix of " + ", ".join(f"{c.name} ({c.particles.n} spheres)" for c in reqs))
    with L.Server(8 << 30, max_slots=8, chunk_steps=chunk) as srv:
        tks = [srv.lbdem_server_submit(c.params, c.particles, steps, avg_from) for c in reqs]
        got = [srv.wait(t) for t in tks]
    for c, g in zip(reqs, got):
        assert g["status"] == 0 and g["steps_done"] == steps
        o = O.Oracle(c.params.copy(precision="fp64"), c.particles)
        s, n, done = 0.0, 0, 0
        while done < steps:
            r = o.step(chunk)
            assert r["status"] == 0
            done += chunk
            if done > avg_from:
                s += o.diagnostics()["u_ps"]
                n += 1
        ups_o = s / n
        do = o.diagnostics()
        m = c.particles.rho_p * np.pi * c.particles.d ** 3 / 6
        aux = o.step(1, aux=True)  # one more step only for the fluid momentum scale
        scale = float(np.sum(m * np.linalg.norm(o.state.u, axis=1))
                      + np.sum(np.linalg.norm(aux["j"] + 0.5 * aux["f_acc"], axis=0)))
        e_ups = abs(g["u_ps"] - ups_o) / abs(ups_o)
        e_eps = abs(g["mean_eps_f"] - do["mean_eps_f"]) / do["mean_eps_f"]
        e_mom = float(np.abs(np.asarray(g["mom"]) - (do["mom_fluid"] + do["mom_part"])).max()) / scale
        _say(f"  {c.name}: <u_pS> served {g['u_ps']:.6e} oracle {ups_o:.6e} rel {e_ups:.2e}; "
             f"<eps_f> rel {e_eps:.2e}; momentum rel {e_mom:.2e}")
        assert e_ups <= 1e-3 and e_eps <= 1e-6 and e_mom <= 1e-6
