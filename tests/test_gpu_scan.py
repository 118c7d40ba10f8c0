"""The paper's scans (Sec. 2, Figs. 1 and 2) with event statistics, at a
small lattice: every scan event is an ordinary coupled run (bitwise the same
as building that event by hand), the first event matches the oracle's run of
all twelve scan species and both correlators, and the jackknife statistics
equal the oracle's on the same per-event series."""
import math

import numpy as np
import pytest

from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

CFG = dict(n_events=4, N=24, L_fm=3.0, sheets=1, g2mu=1.0, m_ir=0.2, n_per=150, precision=64,
           seed=77001, tau_max=0.25)


@pytest.fixture(scope="module")
def scan():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_07999_amd import scan as S
    return S, S.run_scan(keep_events=True, **CFG)


def test_scan_event_equals_a_single_event_run(scan):
    import paper_2307_07999_amd as g
    S, res = scan
    e = 2
    steps = res["coupled_steps"]
    ev = g.Event(CFG["N"], CFG["L_fm"], 0.125, precision=64, max_steps=steps,
                 max_particles=CFG["n_per"] * len(S.scan_points()), static_correlator=True,
                 lightlike_correlator=True)
    ev.init_glasma(CFG["g2mu"], CFG["m_ir"], CFG["sheets"], CFG["seed"] + e)
    for (_, kind, m, p0, tf) in S.scan_points():
        ev.add_species(m, p0, kind, CFG["n_per"], CFG["seed"] + e, tau_form_fm=tf)
    a_fm = CFG["L_fm"] / CFG["N"]
    # static quarks start on the formation step of the beauty quarks at rest
    assert res["static_start_fm"] == res["nform"][0] * 0.125 * a_fm
    ev.static_start(res["static_start_fm"])
    ev.lightlike_start(0.0)
    ev.run(steps)
    assert np.array_equal(ev.series()[:, :12, :], res["series"][e])
    assert np.array_equal(S._correlator_series(ev.static_broadening(), a_fm, steps), res["static_series"][e])
    assert np.array_equal(S._correlator_series(ev.lightlike_broadening(), a_fm, steps), res["lightlike_series"][e])


def test_scan_event_matches_oracle(scan, orc):
    """Event 0: the oracle runs the same MV draw and the twelve species
    (beauty quarks at four p_T, jets at four p_x for two masses) to the same
    time; series to 1e-9 relative per species (chaotic growth over the run)
    and both correlators, which the oracle computes from its own fields (the
    static one from the beauty quarks' formation step, the lightlike one from
    the first step)."""
    S, res = scan
    N, L = CFG["N"], CFG["L_fm"]
    a_fm = L / N
    a_gev = a_fm / H.HBARC
    sigma = CFG["g2mu"] * a_gev / math.sqrt(CFG["sheets"])
    m2 = (CFG["m_ir"] * a_gev) ** 2
    steps = res["coupled_steps"]
    species = []
    for k, (_, kind, m, p0, tf) in enumerate(S.scan_points()):
        species.append(dict(kind=kind, mass=m * a_gev, p0=p0 * a_gev, nform=res["nform"][k], n=CFG["n_per"]))
    st, P, ser_o, rc = orc.run(N, sigma, m2, CFG["sheets"], CFG["seed"], 0.125, steps, species)
    assert rc == 0
    got = res["series"][0]
    assert got.shape == ser_o.shape
    assert np.array_equal(got[:, :, 3], ser_o[:, :, 3])
    for k in range(len(species)):
        assert H.rel_err(got[:, k, :3], ser_o[:, k, :3]) < 1e-9, k
    s, rc, _ = orc.init_glasma(N, sigma, m2, CFG["sheets"], CFG["seed"], 0.125)
    s2 = s.copy()
    stat = orc.static_series(s, 0.125, steps, n0=res["nform"][0])
    ll = orc.lightlike_series(s2, 0.125, steps, n0=1)
    assert H.rel_err(res["static_series"][0], stat) < 1e-9
    assert H.rel_err(res["lightlike_series"][0], ll) < 1e-9


def test_scan_statistics_match_oracle_jackknife(scan, orc):
    S, res = scan
    a_fm = CFG["L_fm"] / CFG["N"]
    dt = 0.125 * a_fm
    for k, (_, kind, m, p0, tf) in enumerate(S.scan_points()):
        want = orc.scan_statistics(res["series"][:, :, k, :], kind, dt, a_fm)
        got = res["stats"][k]
        assert got.shape == want.shape and len(got) > 0
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
        assert np.all(got[:, 3::2] >= 0) and np.any(got[:, 3] > 0)     # events differ: non-zero errors
    for name, kind in (("static", 0), ("lightlike", 1)):
        want = orc.scan_statistics(res[name + "_series"], kind, dt, a_fm)
        assert np.abs(res[name] - want).max() <= 1e-12 * np.abs(want).max()
    summ = S.summary(res)
    assert set(summ) == set(res["points"]) | {"static", "lightlike"}
    for v in summ.values():
        assert v["peak"]["total"] > 0 and v["peak"]["err"] >= 0
