"""GPU parity: every stage of the HIP path against the FP64 CPU oracle on the
same seeded inputs, through the C-ABI.

Tolerances (FP64 path): the two sides differ only by rounding order (the GPU
uses Cayley-Hamilton exponentials, fused multiply-adds and tree reductions,
the oracle power-series exponentials and sequential sums), so single steps
agree to ~1e-15 relative; a full 63-step coupled run amplifies that by the
chaotic growth of classical Yang-Mills over tau <= 1 fm, and we bound the
relative error at 1e-9.  FP32 (configuration with FP32 links and fields): the
target is 1e-3 relative on the observables, err(f) = max|f32 - f64| / max|f64|.
"""
import math

import numpy as np
import pytest

from tests import gpu_helpers as H
from tests import seeded_inputs as si

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07999_amd as g
    g.lib()
    return g


def _event(gl, N, L=4.0, prec=64, max_particles=0, max_steps=128, reunit=16, static_correlator=False,
           lightlike_correlator=False):
    return gl.Event(N, L, 0.125, precision=prec, reunit_every=reunit, max_steps=max_steps,
                    max_particles=max_particles, static_correlator=static_correlator,
                    lightlike_correlator=lightlike_correlator)


def test_charges_match_oracle(gl, orc):
    N = 16
    ev = _event(gl, N)
    for nuc, sheet in ((0, 0), (1, 3)):
        got = ev.draw_charges(77, nuc, sheet, 0.6)
        want = orc.mv_charges(N, 0.6, 77, nuc, sheet)
        assert H.rel_err(got, want.T) < 1e-14


@pytest.mark.parametrize("N,sheets", [(32, 2), (48, 2), (6, 1)])
def test_wilson_lines_match_oracle(gl, orc, N, sheets):
    cfg = dict(H.C1, N=N, sheets=sheets)
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    ev = _event(gl, N, cfg["L"])
    ev.init_glasma(cfg["g2mu"], cfg["m_ir"], sheets, cfg["seed"])
    for nuc in (0, 1):
        want = orc.wilson_line(N, sigma, m2, sheets, cfg["seed"], nuc)
        got = ev.wilson_line(nuc)
        assert np.abs(got - want.T).max() < 1e-12


def test_wilson_lines_with_uv_cut_match_oracle(gl, orc):
    N, sheets, uv = 48, 2, 3.0
    cfg = dict(H.C1, N=N, sheets=sheets)
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    ev = _event(gl, N, cfg["L"])
    ev.init_glasma(cfg["g2mu"], cfg["m_ir"], sheets, cfg["seed"], uv_cut_GeV=uv)
    for nuc in (0, 1):
        want = orc.wilson_line(N, sigma, m2, sheets, cfg["seed"], nuc, uv2=(uv * a_gev) ** 2)
        assert np.abs(ev.wilson_line(nuc) - want.T).max() < 1e-12
        nocut = orc.wilson_line(N, sigma, m2, sheets, cfg["seed"], nuc)
        assert np.abs(want - nocut).max() > 1e-3


@pytest.mark.parametrize("N", [32, 24])
def test_initial_state_matches_oracle(gl, orc, N):
    cfg = dict(H.C1, N=N)
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    ev = _event(gl, N, cfg["L"])
    ev.init_glasma(cfg["g2mu"], cfg["m_ir"], 1, cfg["seed"])
    U, E, phi, pi, n = ev.get_state()
    s, rc, res = orc.init_glasma(N, sigma, m2, 1, cfg["seed"], 0.125)
    assert rc == 0 and n == 1
    Uo, Eo, phio, pio = H.state_oracle_to_soa(s)
    assert np.abs(U - Uo).max() < 1e-12
    assert np.abs(E).max() == 0
    assert np.abs(pi - pio).max() < 1e-12
    assert np.abs(phi - phio).max() < 1e-14


@pytest.mark.parametrize("N", [8, 40, 64])
def test_field_steps_match_oracle(gl, orc, N):
    U, E, phi, pi = si.random_state(100 + N, N, link_kind="near", eps=0.5)
    s = orc.State(N)
    s.U, s.E, s.phi, s.pi, s.n = U, E, phi, pi, 3
    ev = _event(gl, N)
    ev.set_state(*H.state_oracle_to_soa(s), 3)
    ev.evolve_fields(5)
    for _ in range(5):
        orc.field_step(s, 0.125)
    got = ev.get_state()
    assert got[4] == s.n
    for g, w in zip(got[:4], H.state_oracle_to_soa(s)):
        assert np.abs(g - w).max() < 1e-12


@pytest.mark.parametrize("prec,tol", [(64, 1e-12), (32, 2e-5)])
def test_site_fields_on_a_ragged_lattice(gl, orc, prec, tol):
    """Site fields at N = 40: the field-step tiles end inside the lattice in
    both directions, and E_x adds the half transported from x - 1 within
    the workgroup except at x = 0, 16, 32, where it is stored apart and
    added by the reader (E_y likewise at even y).  FP64 and FP32 against the
    oracle; a few particles make the step write the site fields."""
    N = 40
    U, E, phi, pi = si.random_state(700 + prec, N, link_kind="near", eps=0.5)
    s = orc.State(N)
    s.U, s.E, s.phi, s.pi, s.n = U, E, phi, pi, 3
    ev = _event(gl, N, prec=prec, max_particles=64)
    ev.set_state(*H.state_oracle_to_soa(s), 3)
    ev.add_species(1.27, 2.0, gl.KIND_HEAVY_QUARK, 16, 5)
    ev.evolve_fields(1)
    F = orc.field_step(s, 0.125, want_F=True)
    want = np.transpose(F, (1, 2, 0))
    got = ev.site_fields()
    assert np.abs(got - want).max() < tol * max(1.0, np.abs(want).max())


def _oracle_particles(orc, N, seed, specs):
    parts = []
    for sid, (kind, p0, n) in enumerate(specs):
        P = orc.particles_init(N, seed, sid, kind, p0, n)
        parts.append(P)
    tot = sum(p.n for p in parts)
    Pall = orc.Particles(tot)
    for k in ("cell", "off", "eta", "p", "Q", "p0", "species"):
        setattr(Pall, k, np.ascontiguousarray(np.concatenate([getattr(p, k) for p in parts])))
    return Pall


def test_particle_init_matches_oracle(gl, orc):
    N, seed = 32, 4242
    cfg = dict(H.C1)
    a_fm, a_gev, _, _ = H.lattice(cfg)
    ev = _event(gl, N, max_particles=3000)
    ev.init_glasma(1.0, 0.2, 1, seed)
    ev.add_species(1.27, 2.0, gl.KIND_HEAVY_QUARK, 1000, seed)
    ev.add_species(0.0, 10.0, gl.KIND_JET, 700, seed)
    got = ev.get_particles()
    want = _oracle_particles(orc, N, seed, [(0, 2.0 * a_gev, 1000), (1, 10.0 * a_gev, 700)])
    w = H.particles_oracle_to_gpu(want)
    assert np.array_equal(got["cell"], w["cell"])
    assert np.array_equal(got["off"], w["off"])
    assert np.array_equal(got["species"], w["species"])
    assert np.abs(got["p0"] - w["p0"]).max() < 1e-15
    assert np.abs(got["Q"] - w["Q"]).max() < 1e-13


def _setup_coupled(gl, orc, N, prec, seed, specs, cfg):
    """GPU and oracle events with identical fields (oracle init) and particles."""
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    s, rc, _ = orc.init_glasma(N, sigma, m2, cfg["sheets"], seed, 0.125)
    ev = _event(gl, N, cfg["L"], prec=prec, max_particles=sum(n for *_, n in specs) + 10, max_steps=256)
    ev.set_state(*H.state_oracle_to_soa(s), 1)
    descs = []
    lat = []
    for kind, m, p0, n in specs:
        descs.append((m, p0, kind, -1.0))
        lat.append((kind, p0 * a_gev, n))
    P = _oracle_particles(orc, N, seed, lat)
    d = H.particles_oracle_to_gpu(P)
    ev.set_particles(descs, d["cell"], d["off"], d["eta"], d["p"], d["Q"], d["p0"], d["species"])
    mass = [ev.species_info(k)[1] for k in range(len(specs))]
    nform = [ev.species_info(k)[0] for k in range(len(specs))]
    return s, P, ev, mass, nform


def test_site_fields_and_one_push_match_oracle(gl, orc):
    N = 24
    cfg = dict(H.C1, N=N, L=3.0)
    s, P, ev, mass, nform = _setup_coupled(gl, orc, N, 64, 9, [(0, 1.27, 2.0, 300), (1, 0.0, 10.0, 200)], cfg)
    # advance both to n = 6 so that every species is formed and fields are generic
    for _ in range(5):
        ev.evolve_fields(1)
        ev.push_particles()
    for _ in range(5):
        U0, phi0, n = s.U.copy(), s.phi.copy(), s.n
        F = orc.field_step(s, 0.125, want_F=True)
        orc.particle_step(N, n, 0.125, U0, phi0, F, P, mass, nform)
    U0, phi0, n = s.U.copy(), s.phi.copy(), s.n
    F = orc.field_step(s, 0.125, want_F=True)
    ev.evolve_fields(1)
    Fg = ev.site_fields()
    assert np.abs(Fg - np.transpose(F, (1, 2, 0))).max() < 1e-12 * max(1.0, np.abs(F).max())
    orc.particle_step(N, n, 0.125, U0, phi0, F, P, mass, nform)
    ev.push_particles()
    got = ev.get_particles()
    w = H.particles_oracle_to_gpu(P)
    assert np.array_equal(got["cell"], w["cell"])
    for k in ("off", "eta", "p", "Q"):
        assert np.abs(got[k] - w[k]).max() < 1e-12, k


@pytest.mark.parametrize("prec,tol,stol", [(64, 1e-12, 1e-9), (32, 2e-4, 1e-3)])
def test_single_particles_through_a_sort_period_match_oracle(gl, orc, prec, tol, stol):
    """The smallest ensembles: one heavy quark and one jet, each alone in its
    push workgroup (255 padding lanes), through 20 coupled steps of gl_run,
    so that the sort that falls due at step 16 and the push that applies it
    run too."""
    N = 24
    cfg = dict(H.C1, N=N, L=3.0)
    s, P, ev, mass, nform = _setup_coupled(gl, orc, N, prec, 17, [(0, 1.27, 2.0, 1), (1, 0.0, 10.0, 1)], cfg)
    steps = 20
    ev.run(steps)
    rows = []
    for _ in range(steps):
        U0, phi0, n = s.U.copy(), s.phi.copy(), s.n
        F = orc.field_step(s, 0.125, want_F=True)
        rows.append(orc.particle_step(N, n, 0.125, U0, phi0, F, P, mass, nform))
    got = ev.get_particles()
    w = H.particles_oracle_to_gpu(P)
    assert np.array_equal(got["cell"], w["cell"])
    for k in ("off", "eta", "p", "Q"):
        assert np.abs(got[k] - w[k]).max() < tol, k
    # series rows: the count of formed particles exactly (the quark forms at
    # its formation step, the jet at once), the momentum sums to tolerance
    ser, want = ev.series()[:, :2, :], np.array(rows)[:, :2, :]
    assert ser.shape == want.shape == (steps, 2, 4)
    assert np.array_equal(ser[:, :, 3], want[:, :, 3])
    assert want[0, 0, 3] == 0 and want[-1, 0, 3] == 1 and np.all(want[:, 1, 3] == 1)
    assert np.abs(ser[:, :, :3] - want[:, :, :3]).max() <= stol * max(1.0, np.abs(want[:, :, :3]).max())


@pytest.mark.parametrize("prec", [64, 32])
def test_run_without_particles_equals_field_steps(gl, prec):
    """An event with no particles: gl_run is the field leapfrog alone, bitwise
    the state that gl_evolve_fields reaches, and writes no series rows."""
    N = 40
    U, E, phi, pi = si.random_state(41 + prec, N, link_kind="near", eps=0.4)
    evs = []
    for _ in range(2):
        ev = _event(gl, N, prec=prec, max_particles=0, max_steps=16)
        ev.set_state(si.links_to_soa(U), si.links_to_soa(E), si.alg_to_soa(phi), si.alg_to_soa(pi), 2)
        evs.append(ev)
    evs[0].run(7)
    evs[1].evolve_fields(7)
    a, b = evs[0].get_state(), evs[1].get_state()
    assert a[4] == b[4] == 9
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    assert len(evs[0].series()) == 0


def test_c1_full_run_matches_oracle(gl, orc):
    """The 32^2 parity configuration end to end: MV init on the device,
    1000 charm quarks, 63 coupled steps to tau = 1 fm, series and kappa."""
    cfg = H.C1
    N = cfg["N"]
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    steps = H.n_steps(cfg)
    assert steps == 63
    ev = _event(gl, N, cfg["L"], max_particles=1000, max_steps=steps)
    ev.init_glasma(cfg["g2mu"], cfg["m_ir"], cfg["sheets"], cfg["seed"])
    sid = ev.add_species(1.27, 0.0, gl.KIND_HEAVY_QUARK, 1000, cfg["seed"])
    nform, mass = ev.species_info(sid)
    assert nform == 5
    ev.run(steps)
    ser = ev.series()[:, :1, :]
    st, P, ser_o, rc = orc.run(N, sigma, m2, 1, cfg["seed"], 0.125, steps,
                               [dict(kind=0, mass=mass, p0=0.0, nform=nform, n=1000)])
    assert rc == 0
    assert np.array_equal(ser[:, 0, 3], ser_o[:, 0, 3])
    for c in range(3):
        assert H.rel_err(ser[:, 0, c], ser_o[:, 0, c]) < 1e-9
    # kappa rows from the library against the oracle's derivative
    kap = ev.kappa(sid)
    ks, rates = orc.coefficients(ser_o[:, 0, :], 0.125)
    f2, fk = orc.to_physical(a_fm)
    assert len(kap) == len(ks)
    assert H.rel_err(kap[:, 2], (rates[:, 0] + rates[:, 1]) * fk) < 1e-9
    assert H.rel_err(kap[:, 3], rates[:, 2] * fk) < 1e-9
    assert np.allclose(kap[:, 0], (ks + 1) * 0.125 * a_fm)
    d = ev.diagnostics()
    assert d["gauss_max"] < 1e-12 and d["unitarity_max"] < 1e-12
    assert d["casimir2_dev"] < 1e-12 and d["nonfinite"] == 0
    U, E, phi, pi, n = ev.get_state()
    for g, w in zip((U, E, phi, pi), H.state_oracle_to_soa(st)):
        assert H.rel_err(g, w) < 1e-9


def test_fp32_observables_within_target(gl, orc):
    """FP32 links/fields (re-unitarised every 16 steps) with FP64 sums against
    the FP64 oracle on the 32^2 configuration with charm quarks and jets."""
    cfg = H.C1
    N = cfg["N"]
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    steps = H.n_steps(cfg)
    ev = _event(gl, N, cfg["L"], prec=32, max_particles=2000, max_steps=steps)
    ev.init_glasma(cfg["g2mu"], cfg["m_ir"], 1, cfg["seed"])
    c = ev.add_species(1.27, 0.0, gl.KIND_HEAVY_QUARK, 1000, cfg["seed"])
    j = ev.add_species(0.0, 10.0, gl.KIND_JET, 1000, cfg["seed"])
    ev.run(steps)
    sp = [dict(kind=0, mass=ev.species_info(c)[1], p0=0.0, nform=ev.species_info(c)[0], n=1000),
          dict(kind=1, mass=0.0, p0=10.0 * a_gev, nform=ev.species_info(j)[0], n=1000)]
    st, P, ser_o, rc = orc.run(N, sigma, m2, 1, cfg["seed"], 0.125, steps, sp)
    ser = ev.series()
    f2, fk = orc.to_physical(a_fm)
    errs = {}
    mean_o, _ = orc.mean_broadening(ser_o[:, 0])
    mean_g, _ = orc.mean_broadening(ser[:, 0])
    errs["dpT2"] = H.rel_err(mean_g[:, 0] + mean_g[:, 1], mean_o[:, 0] + mean_o[:, 1])
    _, ro = orc.coefficients(ser_o[:, 0], 0.125)
    _, rg = orc.coefficients(ser[:, 0], 0.125)
    errs["kappa_T"] = H.rel_err(rg[:, 0] + rg[:, 1], ro[:, 0] + ro[:, 1])
    errs["kappa_L"] = H.rel_err(rg[:, 2], ro[:, 2])
    _, ro = orc.coefficients(ser_o[:, 1], 0.125)
    _, rg = orc.coefficients(ser[:, 1], 0.125)
    errs["qhat_y"] = H.rel_err(rg[:, 1], ro[:, 1])
    errs["qhat_z"] = H.rel_err(rg[:, 2], ro[:, 2])
    print("FP32 vs FP64 oracle errors:", errs)
    for k, v in errs.items():
        assert v < 1e-3, (k, v)
    # particles whose cell sequence left the FP64 one (a crossing decided the
    # other way near a cell boundary): compared through the final cells
    d = ev.get_particles()
    frac = float(np.mean(np.any(d["cell"].T != P.cell, axis=1)))
    print("FP32: fraction of particles whose final cell differs from FP64: %.4f" % frac)
    assert frac < 0.02


def test_call_order_errors(gl):
    ev = _event(gl, 8, max_particles=10)
    with pytest.raises(gl.GlasmaError) as e:
        ev.evolve_fields(1)
    assert e.value.status == -2
    ev.init_glasma(1.0, 0.2, 1, 1)
    ev.add_species(1.27, 0.0, gl.KIND_HEAVY_QUARK, 10, 1)
    with pytest.raises(gl.GlasmaError):
        ev.push_particles()
    with pytest.raises(gl.GlasmaError):
        ev.evolve_fields(2)
    ev.evolve_fields(1)
    with pytest.raises(gl.GlasmaError):
        ev.evolve_fields(1)
    ev.push_particles()
    ev.run(3)


def test_particle_sort_is_transparent_and_deterministic(gl, orc):
    """Re-sorting particles by cell changes only their storage order: the
    particles returned in creation order and the series are the same with
    sorting every step, every 16 steps, and never, up to FP64 summation order,
    and two identical runs are bitwise equal."""
    N = 32
    results = []
    for every in (1, 16, 0, 1):
        ev = _event(gl, N, 4.0, max_particles=3000, max_steps=40)
        ev.set_sort_period(every)
        ev.init_glasma(1.0, 0.2, 1, 7)
        ev.add_species(1.27, 5.0, gl.KIND_HEAVY_QUARK, 1000, 7)
        ev.add_species(0.0, 10.0, gl.KIND_JET, 1500, 8)
        ev.run(40)
        results.append((ev.get_particles(), ev.series()))
    ref_p, ref_s = results[0]
    for parts, ser in results[1:]:
        assert np.array_equal(parts["cell"], ref_p["cell"])
        for k in ("off", "p", "Q", "eta"):
            assert np.abs(parts[k] - ref_p[k]).max() < 1e-13
        assert H.rel_err(ser, ref_s) < 1e-13
    # identical configuration -> bitwise identical series and particles
    assert np.array_equal(results[3][1], results[0][1])
    assert np.array_equal(results[3][0]["p"], results[0][0]["p"])


@pytest.mark.parametrize("prec", [64, 32])
def test_sort_applied_by_the_next_push_is_bitwise_transparent(gl, prec):
    """Within a run a due sort only computes the sorted order, and the next
    push moves each particle to its sorted slot while pushing it.  That must
    give bitwise the same particles and series as sorting at once (stepwise
    field steps and pushes), also when the run ends right after a sort is due
    and when it is split into two runs."""
    N = 48
    out = []
    for mode in ("run", "stepwise", "split"):
        ev = _event(gl, N, 6.0, prec=prec, max_particles=5000, max_steps=30)
        ev.set_sort_period(3)
        ev.init_glasma(1.0, 0.2, 2, 11)
        ev.add_species(1.27, 5.0, gl.KIND_HEAVY_QUARK, 2000, 3)
        ev.add_species(0.0, 10.0, gl.KIND_JET, 2500, 4)
        if mode == "run":
            ev.run(24)
        elif mode == "split":
            ev.run(9)
            ev.run(15)
        else:
            for _ in range(24):
                ev.evolve_fields(1)
                ev.push_particles()
        out.append((ev.get_particles(), ev.series()))
        ev.close()
    ref_p, ref_s = out[1]
    for parts, ser in (out[0], out[2]):
        assert np.array_equal(ser, ref_s)
        for k in ("cell", "off", "p", "Q", "eta"):
            assert np.array_equal(parts[k], ref_p[k]), k
        assert np.isfinite(parts["Q"]).all()


def test_static_correlator_matches_oracle(gl, orc):
    """Static quarks (Eq. (4)) on the 32^2 configuration: FP64 accumulators
    of the site fields from tau_start on, against the oracle's correlator, in
    FP64 and in FP32 (the FP32 fields against the FP64 oracle at the 1e-3
    observable target).  Fields only: the accumulation needs no particles."""
    cfg = H.C1
    N = cfg["N"]
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    steps = H.n_steps(cfg)
    tau0 = 0.05                          # fm: start after a few steps
    n0 = int(np.ceil(tau0 / (0.125 * a_fm) - 1e-9))
    s, rc, _ = orc.init_glasma(N, sigma, m2, 1, cfg["seed"], 0.125)
    assert rc == 0
    rows = orc.static_series(s, 0.125, steps, n0=n0)
    f2, _ = orc.to_physical(a_fm)
    act = rows[:, 3] > 0
    want = rows[act, :3] / rows[act, 3:4] * f2
    for prec, tol in ((64, 1e-9), (32, 1e-3)):
        ev = _event(gl, N, cfg["L"], prec=prec, max_steps=steps, static_correlator=True)
        ev.init_glasma(cfg["g2mu"], cfg["m_ir"], cfg["sheets"], cfg["seed"])
        ev.static_start(tau0)
        ev.evolve_fields(steps)
        got = ev.static_broadening()
        assert len(got) == int(act.sum()) == steps - n0 + 1
        assert np.allclose(got[:, 0], (np.nonzero(act)[0] + 1.5) * 0.125 * a_fm)
        assert np.all(got[:, 4] == N * N)
        for c in range(3):
            err = H.rel_err(got[:, 1 + c], want[:, c])
            print("static correlator FP%d component %d: rel err %.2e" % (prec, c, err))
            assert err < tol
        ev.close()
    # without the accumulators the calls refuse
    ev = _event(gl, N, cfg["L"], max_steps=steps)
    ev.init_glasma(cfg["g2mu"], cfg["m_ir"], cfg["sheets"], cfg["seed"])
    with pytest.raises(gl.GlasmaError):
        ev.static_start(0.0)


def test_lightlike_correlator_matches_oracle(gl, orc):
    """Lightlike jets (Eq. (5)) on the 32^2 configuration, run together with
    the static correlator and with particles (the site fields are shared):
    transported forces accumulated from tau_start on, against the oracle's
    correlator, in FP64 and FP32."""
    cfg = H.C1
    N = cfg["N"]
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    steps = H.n_steps(cfg)
    tau0 = 0.03
    n0 = int(np.ceil(tau0 / (0.125 * a_fm) - 1e-9))
    s, rc, _ = orc.init_glasma(N, sigma, m2, 1, cfg["seed"], 0.125)
    s2 = s.copy()
    rows = orc.lightlike_series(s, 0.125, steps, n0=n0)
    srows = orc.static_series(s2, 0.125, steps, n0=1)
    f2, _ = orc.to_physical(a_fm)
    act = rows[:, 3] > 0
    want = rows[act, :3] / rows[act, 3:4] * f2
    swant = srows[:, :3] / srows[:, 3:4] * f2
    for prec, tol in ((64, 1e-9), (32, 1e-3)):
        ev = _event(gl, N, cfg["L"], prec=prec, max_steps=steps, max_particles=256, static_correlator=True,
                    lightlike_correlator=True)
        ev.init_glasma(cfg["g2mu"], cfg["m_ir"], cfg["sheets"], cfg["seed"])
        ev.add_species(1.27, 0.0, gl.KIND_HEAVY_QUARK, 256, 7)
        ev.lightlike_start(tau0)
        ev.static_start(0.0)
        ev.run(steps)
        got = ev.lightlike_broadening()
        assert len(got) == int(act.sum()) == steps - n0 + 1
        assert np.all(got[:, 4] == N * N)
        sgot = ev.static_broadening()
        for c in range(3):
            err = H.rel_err(got[:, 1 + c], want[:, c])
            serr = H.rel_err(sgot[:, 1 + c], swant[:, c])
            print("FP%d component %d: lightlike rel err %.2e, static rel err %.2e" % (prec, c, err, serr))
            assert err < tol and serr < tol
        ev.close()


def test_dipole_and_saturation_scale_match_oracle(gl, orc):
    """Dipole correlator of the device Wilson lines against the oracle's, and
    Q_s from the exp(-1/2) crossing computed from the oracle curve."""
    N, L = 48, 4.0
    a_fm = L / N
    a_gev = a_fm / H.HBARC
    g2mu, m_ir, sheets, seed = 2.0, 0.2, 3, 17
    sigma = g2mu * a_gev / math.sqrt(sheets)
    ev = _event(gl, N, L)
    ev.init_glasma(g2mu, m_ir, sheets, seed)
    qs = []
    for nuc in (0, 1):
        D = ev.dipole(nuc, N // 2)
        W = orc.wilson_line(N, sigma, (m_ir * a_gev) ** 2, sheets, seed, nuc)
        Do = orc.dipole(N, W, N // 2)
        assert np.abs(D - Do).max() < 1e-12
        r = int(np.argmax(Do <= np.exp(-0.5)))
        rs = (r - 1) + (Do[r - 1] - np.exp(-0.5)) / (Do[r - 1] - Do[r])
        qs.append(math.sqrt(2.0) / (rs * a_gev))
    assert abs(ev.saturation_scale() - 0.5 * (qs[0] + qs[1])) < 1e-10
    # the calibration reaches its target and leaves the fields alone
    U0 = ev.get_state()[0]
    g, q = ev.calibrate_g2mu(1.0, m_ir, sheets, seed, n_seeds=1)
    assert abs(q - 1.0) < 1e-3 and g > 0
    assert np.array_equal(ev.get_state()[0], U0)


def test_paper_scale_g2mu_gives_qs_2_gev(gl):
    """The 512^2 workload's g^2 mu (2.767 GeV) is the calibrated one: the MV
    Wilson lines of 4 seeds at L = 10 fm, 50 sheets, m_IR = 0.2 GeV have
    Q_s = 2 GeV by the dipole definition."""
    import bench
    ev = gl.Event(512, 10.0, 0.125, precision=64, max_steps=1)
    g, q = ev.calibrate_g2mu(2.0, bench.M_IR, bench.SHEETS, bench.SEED, n_seeds=4)
    ev.close()
    print("calibrated g2mu %.4f GeV (Q_s %.4f GeV)" % (g, q))
    assert abs(g - bench.G2MU) < 5e-3


def test_energy_diagnostics_match_oracle(gl, orc):
    """gl_diagnostics' energy terms (E_T, E_L, B_T, B_L per unit rapidity)
    against the oracle's energy of the same state, right after the MV
    initial condition and after 20 field steps."""
    cfg = H.C1
    N = cfg["N"]
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    ev = _event(gl, N, cfg["L"])
    ev.init_glasma(cfg["g2mu"], cfg["m_ir"], cfg["sheets"], cfg["seed"])
    s, rc, _ = orc.init_glasma(N, sigma, m2, cfg["sheets"], cfg["seed"], 0.125)
    for k in (0, 20):
        if k:
            ev.evolve_fields(k)
            for _ in range(k):
                orc.field_step(s, 0.125)
        got = np.array(ev.diagnostics()["energy"])
        want = orc.energy(s, s.n * 0.125)
        print("energy at n=%d: %s vs %s" % (s.n, got, want))
        # E_T vanishes at n = 1 (E^{1/2} = 0); the other terms start non-zero
        assert np.all(want[1:] > 0) and (k == 0 or want[0] > 0)
        assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_observable_rows_match_oracle(gl, orc):
    """The rows of gl_broadening (GeV^2), gl_kappa and gl_qhat (GeV^2/fm)
    against the oracle's series turned into means and central differences and
    converted with the lattice spacing: heavy quarks (kappa_T, kappa_L and
    tau - tau_form) and jets (qhat_y, qhat_z), with the rows before formation
    left out."""
    N = 24
    cfg = dict(H.C1, N=N, L=3.0)
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    steps = 30
    ev = _event(gl, N, cfg["L"], max_particles=1200, max_steps=steps)
    ev.init_glasma(cfg["g2mu"], cfg["m_ir"], 1, cfg["seed"])
    q = ev.add_species(4.18, 2.0, gl.KIND_HEAVY_QUARK, 600, cfg["seed"])
    j = ev.add_species(0.0, 5.0, gl.KIND_JET, 600, cfg["seed"])
    ev.run(steps)
    sp = [dict(kind=0, mass=ev.species_info(q)[1], p0=2.0 * a_gev, nform=ev.species_info(q)[0], n=600),
          dict(kind=1, mass=0.0, p0=5.0 * a_gev, nform=ev.species_info(j)[0], n=600)]
    _, _, ser_o, rc = orc.run(N, sigma, m2, 1, cfg["seed"], 0.125, steps, sp)
    assert rc == 0
    f2, fk = orc.to_physical(a_fm)
    dt_fm = 0.125 * a_fm
    for sid in (q, j):
        mean, act = orc.mean_broadening(ser_o[:, sid])
        ks = np.nonzero(act)[0]
        br = ev.broadening(sid)
        assert len(br) == len(ks) > 0
        assert np.abs(br[:, 0] - (ks + 1.5) * dt_fm).max() < 1e-14
        assert H.rel_err(br[:, 1:4], mean[ks] * f2) < 1e-9
        assert np.array_equal(br[:, 4], ser_o[ks, sid, 3])
        kk, rates = orc.coefficients(ser_o[:, sid], 0.125)
        if sid == q:
            rows = ev.kappa(sid)
            nform = ev.species_info(sid)[0]
            assert ks[0] == nform - 1          # the first active row is the formation step
            tau_form = 0.1973269804 / (2 * math.hypot(4.18, 2.0))
            assert np.abs(rows[:, 1] - (rows[:, 0] - tau_form)).max() < 1e-14
            assert H.rel_err(rows[:, 2], (rates[:, 0] + rates[:, 1]) * fk) < 1e-9
            assert H.rel_err(rows[:, 3], rates[:, 2] * fk) < 1e-9
        else:
            rows = ev.qhat(sid)
            assert H.rel_err(rows[:, 1], rates[:, 1] * fk) < 1e-9
            assert H.rel_err(rows[:, 2], rates[:, 2] * fk) < 1e-9
        assert len(rows) == len(kk)
        assert np.abs(rows[:, 0] - (kk + 1) * dt_fm).max() < 1e-14


def test_fp32_reunitarisation_runs_and_repairs(gl):
    """FP32 links re-unitarised when n mod 16 = 15: right after that step
    (n = 16) the links are unitary to FP32 rounding, and more so than the
    same run without it, whose rounding drift accumulates over 15 link
    updates.  FP32 keeps the Gauss law to FP32 rounding either way; an FP64
    event ignores the setting."""
    cfg = H.C1
    N = cfg["N"]
    out = {}
    for reunit in (16, 0):
        ev = _event(gl, N, cfg["L"], prec=32, reunit=reunit)
        ev.init_glasma(cfg["g2mu"], cfg["m_ir"], 1, cfg["seed"])
        ev.evolve_fields(15)
        assert ev.info()[2] == 16
        d = ev.diagnostics()
        ev.evolve_fields(16)
        d2 = ev.diagnostics()
        out[reunit] = (d, d2)
        print("FP32 reunit_every=%d: unitarity at n=16 %.2e, n=32 %.2e; gauss_rel %.2e, %.2e"
              % (reunit, d["unitarity_max"], d2["unitarity_max"], d["gauss_rel"], d2["gauss_rel"]))
    (w16, w32), (n16, n32) = out[16], out[0]
    assert w16["unitarity_max"] < 1e-6 and w32["unitarity_max"] < 1e-6
    assert w16["unitarity_max"] < n16["unitarity_max"]
    assert w32["unitarity_max"] < n32["unitarity_max"]
    for d in (w16, w32, n16, n32):
        assert d["gauss_rel"] < 1e-5 and d["nonfinite"] == 0
    ev = _event(gl, N, cfg["L"], prec=64, reunit=16)
    ev.init_glasma(cfg["g2mu"], cfg["m_ir"], 1, cfg["seed"])
    ev.evolve_fields(15)
    e0 = _event(gl, N, cfg["L"], prec=64, reunit=0)
    e0.init_glasma(cfg["g2mu"], cfg["m_ir"], 1, cfg["seed"])
    e0.evolve_fields(15)
    for x, y in zip(ev.get_state()[:4], e0.get_state()[:4]):
        assert np.array_equal(x, y)
