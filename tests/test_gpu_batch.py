"""Batched events: the flattened multi-event kernels, replayed from a captured
hipGraph, reproduce events run one by one bitwise (same per-site and
per-particle arithmetic, same fixed-order reductions), for every tile shape
and grid choice; the autotuner writes and then reads its cache."""
import json
import os

import numpy as np
import pytest

from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

SIZES = [(32, 700), (48, 300), (24, 0), (64, 1500)]


@pytest.fixture(scope="module")
def gl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07999_amd as g
    g.lib()
    return g


def _make(gl, prec, steps):
    evs = []
    for k, (N, npart) in enumerate(SIZES):
        ev = gl.Event(N, N * 0.125, 0.125, precision=prec, max_steps=steps + 2,
                      max_particles=max(npart, 1))
        ev.init_glasma(1.0, 0.2, 1, 100 + k)
        if npart:
            ev.add_species(1.27, 2.0, gl.KIND_HEAVY_QUARK, npart // 2, 200 + k)
            ev.add_species(0.0, 10.0, gl.KIND_JET, npart - npart // 2, 300 + k)
        evs.append(ev)
    return evs


@pytest.mark.parametrize("prec,shape,mult", [(64, 0, 4), (32, 1, 0), (64, 2, 2)])
def test_batch_equals_single_events(gl, prec, shape, mult):
    steps = 45          # one 32-step graph plus 13 ordinary steps
    single = _make(gl, prec, steps)
    for ev in single:
        ev.run(steps)
    batched = _make(gl, prec, steps)
    b = gl.Batch(batched)
    b.config(shape=shape, grid_mult=mult, sort_every=16, graph_steps=32)
    b.run(steps)
    for s, t, (N, npart) in zip(single, batched, SIZES):
        Us, Es, phs, pis, ns = s.get_state()
        Ub, Eb, phb, pib, nb = t.get_state()
        assert ns == nb
        for a, c in ((Us, Ub), (Es, Eb), (phs, phb), (pis, pib)):
            assert np.array_equal(a, c)
        if npart:
            assert np.array_equal(s.series(), t.series())
            ps, pb = s.get_particles(), t.get_particles()
            for k in ("cell", "p", "Q"):
                assert np.array_equal(ps[k], pb[k])
    # the events keep working on their own once the batch releases them
    b.close()
    for t, (N, npart) in zip(batched, SIZES):
        if npart:
            t.evolve_fields(1)
            t.push_particles()


@pytest.mark.parametrize("prec,shape,mult", [(64, 0, 4), (32, 2, 0)])
def test_batch_graph_windows_and_calls_ending_at_a_sort(gl, prec, shape, mult):
    """Each sort's order is applied by the next push.  Two graph windows in a
    row (the second starts with the order of the first one's last sort
    pending, so the two graphs differ), a call that ends on a sort boundary
    (the pending order is applied before the call returns), then a short
    call: bitwise the events run alone."""
    steps = 64 + 16 + 5
    single = _make(gl, prec, steps)
    for ev in single:
        ev.run(steps)
    batched = _make(gl, prec, steps)
    b = gl.Batch(batched)
    b.config(shape=shape, grid_mult=mult, sort_every=16, graph_steps=32)
    for k in (64, 16, 5):
        b.run(k)
    for s, t, (N, npart) in zip(single, batched, SIZES):
        for x, y in zip(s.get_state()[:5], t.get_state()[:5]):
            assert np.array_equal(x, y)
        if npart:
            assert np.array_equal(s.series(), t.series())
            ps, pb = s.get_particles(), t.get_particles()
            for k in ps:
                assert np.array_equal(ps[k], pb[k]), k
    b.close()


def test_autotune_cache_roundtrip(gl, tmp_path):
    evs = _make(gl, 32, 4)
    b = gl.Batch(evs)
    path = str(tmp_path / "tune.json")
    b.autotune(path)
    first = b.info()
    data = json.load(open(path))
    assert len(data) == 1
    (key, val), = data.items()
    assert key.startswith("gfx") and "|p32|" in key
    assert val == [first["shape"], first["grid_mult"]]
    b.close()
    b2 = gl.Batch(evs)
    b2.autotune(path)
    assert b2.info() == first
    b2.run(4)
    b2.close()
    # an entry out of the tuner's range is ignored: the batch is timed again
    # and the entry replaced; a hand configuration out of range is refused
    json.dump({key: [first["shape"], 100]}, open(path, "w"))
    b3 = gl.Batch(evs)
    b3.autotune(path)
    assert b3.info()["grid_mult"] <= 8
    assert json.load(open(path))[key] == [b3.info()["shape"], b3.info()["grid_mult"]]
    with pytest.raises(gl.GlasmaError) as e:
        b3.config(shape=0, grid_mult=65, sort_every=16, graph_steps=32)
    assert e.value.status == gl.GL_EINVAL
    b3.close()


def test_batched_event_matches_oracle(gl, orc):
    """One event of a mixed batch against the oracle directly: the 32^2
    configuration (MV init, 1000 charm quarks, 63 coupled steps to 1 fm) runs
    in a batch beside a 48^2 and a 64^2 event with quarks and jets, and its
    series and final state must match orc.run as a single event does (the
    batched kernels hold the same arithmetic; 1e-9 relative over the chaotic
    63-step evolution)."""
    cfg = H.C1
    N = cfg["N"]
    a_fm, a_gev, sigma, m2 = H.lattice(cfg)
    steps = H.n_steps(cfg)
    ev = gl.Event(N, cfg["L"], 0.125, precision=64, max_steps=steps, max_particles=1000)
    ev.init_glasma(cfg["g2mu"], cfg["m_ir"], cfg["sheets"], cfg["seed"])
    sid = ev.add_species(1.27, 0.0, gl.KIND_HEAVY_QUARK, 1000, cfg["seed"])
    nform, mass = ev.species_info(sid)
    others = []
    for k, (Nk, npart) in enumerate(((48, 900), (64, 2000))):
        o = gl.Event(Nk, Nk * 0.125, 0.125, precision=64, max_steps=steps, max_particles=npart)
        o.init_glasma(1.0, 0.2, 1, 500 + k)
        o.add_species(1.27, 2.0, gl.KIND_HEAVY_QUARK, npart // 2, 600 + k)
        o.add_species(0.0, 10.0, gl.KIND_JET, npart - npart // 2, 700 + k)
        others.append(o)
    b = gl.Batch([others[0], ev, others[1]])
    b.config(shape=2, grid_mult=0, sort_every=16, graph_steps=32)
    b.run(steps)
    b.stream.synchronize()
    st, P, ser_o, rc = orc.run(N, sigma, m2, 1, cfg["seed"], 0.125, steps,
                               [dict(kind=0, mass=mass, p0=0.0, nform=nform, n=1000)])
    assert rc == 0
    ser = ev.series()[:, :1, :]
    assert ser.shape == ser_o.shape
    assert np.array_equal(ser[:, 0, 3], ser_o[:, 0, 3])
    for c in range(3):
        err = H.rel_err(ser[:, 0, c], ser_o[:, 0, c])
        print("batched event vs oracle, series component %d: %.2e" % (c, err))
        assert err < 1e-9
    U, E, phi, pi, n = ev.get_state()
    assert n == 1 + steps
    for g, w in zip((U, E, phi, pi), H.state_oracle_to_soa(st)):
        assert H.rel_err(g, w) < 1e-9
    parts = ev.get_particles()
    assert np.array_equal(parts["cell"], np.ascontiguousarray(P.cell.T))
    b.close()


def test_a_failed_event_is_masked_in_a_batch(gl):
    """One event of a batch gets a NaN momentum (set from the host), another
    a NaN in E and no particles.  The first is masked from the step of its
    first push (its series row turns non-finite there), the second is found
    by the end-of-run check of the field states; gl_batch_run reports
    GL_ENUMERIC and gl_batch_status the steps, while the healthy events run
    bitwise as they do alone."""
    steps = 40
    def make(k, N, npart):
        ev = gl.Event(N, N * 0.125, 0.125, precision=64, max_steps=steps + 2, max_particles=max(npart, 1))
        ev.init_glasma(1.0, 0.2, 1, 900 + k)
        if npart:
            ev.add_species(1.27, 2.0, gl.KIND_HEAVY_QUARK, npart, 910 + k, tau_form_fm=0.0)
        return ev
    spec = [(24, 300), (32, 400), (48, 500), (16, 0)]
    single = [make(k, N, p) for k, (N, p) in enumerate(spec)]
    batched = [make(k, N, p) for k, (N, p) in enumerate(spec)]
    d = batched[1].get_particles()
    d["p"][0, 123] = np.nan
    batched[1].set_particles([(1.27, 2.0, gl.KIND_HEAVY_QUARK, 0.0)], d["cell"], d["off"], d["eta"], d["p"],
                             d["Q"], d["p0"], d["species"])
    U, E, phi, pi, n = batched[3].get_state()
    E[0, 3, 100] = np.nan
    batched[3].set_state(U, E, phi, pi, n)
    for k in (0, 2):
        single[k].run(steps)
    b = gl.Batch(batched)
    b.config(shape=0, grid_mult=0, sort_every=16, graph_steps=32)
    with pytest.raises(gl.GlasmaError) as e:
        b.run(steps)
    assert e.value.status == gl.GL_ENUMERIC
    st = b.status()
    print("batch failure steps:", st)
    assert st[0] == -1 and st[2] == -1
    assert st[1] == 2                  # the first push, 1 -> 2
    assert st[3] == 1 + steps          # the field state at the end of the call
    for k in (0, 2):
        for x, y in zip(single[k].get_state()[:4], batched[k].get_state()[:4]):
            assert np.array_equal(x, y)
        assert np.array_equal(single[k].series(), batched[k].series())
    # the masked event keeps the particles of its one push (1 -> 2); the
    # sorts at steps 16 and 32 still moved them (a masked event's particles
    # follow the batch's buffers without a push), so the getters find each
    # one whole, against the same event stopped after its first push
    ref = make(1, *spec[1])
    ref.set_particles([(1.27, 2.0, gl.KIND_HEAVY_QUARK, 0.0)], d["cell"], d["off"], d["eta"], d["p"],
                      d["Q"], d["p0"], d["species"])
    try:
        ref.run(1)
    except gl.GlasmaError as err:
        assert err.status == gl.GL_ENUMERIC
    pr, pb = ref.get_particles(), batched[1].get_particles()
    for k in pr:
        assert np.array_equal(pr[k], pb[k], equal_nan=True), k
    b.close()


def test_batch_equals_single_events_at_batched_workload_sizes(gl):
    """The bitwise batch == single-event check at the sizes of the 64-event
    FP32 workload: lattices of 128^2, 256^2 and 384^2 at its spacing with
    1e4 to 1e5 particles of its seven species, 40 steps (a graph of 32 and
    8 ordinary steps, two sorts), autotuned configuration."""
    import bench
    steps = 40
    a_fm = bench.L_FM / bench.N

    def make(k, N, per):
        ev = gl.Event(N, N * a_fm, bench.DTAU, precision=32, reunit_every=16, max_steps=steps,
                      max_particles=per * len(bench.SPECIES))
        ev.init_glasma(bench.G2MU, bench.M_IR, 4, 5000 + k)
        for j, (m, p0, kind) in enumerate(bench.SPECIES):
            ev.add_species(m, p0, kind, per, 6000 + 17 * k + j)
        return ev
    spec = [(128, 1500), (256, 4000), (384, 14000)]
    single = [make(k, N, p) for k, (N, p) in enumerate(spec)]
    for ev in single:
        ev.run(steps)
    batched = [make(k, N, p) for k, (N, p) in enumerate(spec)]
    b = gl.Batch(batched)
    b.autotune(None)
    b.run(steps)
    for s, t in zip(single, batched):
        for x, y in zip(s.get_state()[:4], t.get_state()[:4]):
            assert np.array_equal(x, y)
        assert np.array_equal(s.series(), t.series())
        ps, pb = s.get_particles(), t.get_particles()
        for k in ("cell", "p", "Q"):
            assert np.array_equal(ps[k], pb[k])
    b.close()
