"""The boundary's state and failure handling through the C-ABI: checkpoint and
restore resume bitwise, failures forced from the host surface as GL_ENUMERIC
and GL_ENOTCONV, the Casimir diagnostics, and a batch holding its events."""
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


def _blank(gl, prec, correlators=True):
    return gl.Event(32, 4.0, 0.125, precision=prec, max_steps=64, max_particles=3000,
                    static_correlator=correlators, lightlike_correlator=correlators)


def _coupled_event(gl, prec, correlators=True):
    ev = _blank(gl, prec, correlators)
    ev.init_glasma(1.0, 0.2, 2, 61)
    ev.add_species(1.27, 2.0, gl.KIND_HEAVY_QUARK, 1200, 62)
    ev.add_species(0.0, 10.0, gl.KIND_JET, 1300, 63)
    if correlators:
        ev.static_start(0.02)
        ev.lightlike_start(0.05)
    return ev


def _snapshot(ev, correlators=True):
    out = dict(state=ev.get_state(), parts=ev.get_particles(), series=ev.series())
    if correlators:
        out["static"] = ev.static_broadening()
        out["lightlike"] = ev.lightlike_broadening()
    return out


def _assert_bitwise(a, b):
    for x, y in zip(a["state"], b["state"]):
        assert np.array_equal(x, y)
    for k in a["parts"]:
        assert np.array_equal(a["parts"][k], b["parts"][k]), k
    for k in ("series", "static", "lightlike"):
        if k in a:
            assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("prec", [64, 32])
def test_checkpoint_restore_resumes_bitwise(gl, prec, tmp_path):
    """20 steps, checkpoint, restore into a fresh event, 20 more steps: the
    same state, particles, series and correlators bit for bit as 40 steps in
    one go.  The checkpoint falls 4 steps into a 16-step sort period, and
    the sort then falls due in the resumed run."""
    path = str(tmp_path / "ev.ckpt")
    whole = _coupled_event(gl, prec)
    whole.run(40)
    ref = _snapshot(whole)
    first = _coupled_event(gl, prec)
    first.run(20)
    first.checkpoint(path)
    fresh = _blank(gl, prec)
    fresh.restore(path)
    assert fresh.info()[2] == 21
    fresh.run(20)
    _assert_bitwise(ref, _snapshot(fresh))
    # the original event continues identically too
    first.run(20)
    _assert_bitwise(ref, _snapshot(first))


def test_checkpoint_with_a_particle_step_due(gl, tmp_path):
    """A checkpoint between a field step and its particle step keeps the site
    fields, so the restored event can take the pending push."""
    path = str(tmp_path / "due.ckpt")
    a = _coupled_event(gl, 64, correlators=False)
    a.run(5)
    a.evolve_fields(1)
    a.checkpoint(path)
    a.push_particles()
    a.run(3)
    b = _blank(gl, 64, correlators=False)
    b.restore(path)
    with pytest.raises(gl.GlasmaError):
        b.evolve_fields(1)          # the particle step is due, as before the checkpoint
    b.push_particles()
    b.run(3)
    _assert_bitwise(_snapshot(a, False), _snapshot(b, False))


def test_restore_refuses_other_lattices_and_junk(gl, tmp_path):
    path = str(tmp_path / "x.ckpt")
    a = _coupled_event(gl, 64, correlators=False)
    a.run(2)
    a.checkpoint(path)
    other = _blank(gl, 32, correlators=False)
    with pytest.raises(gl.GlasmaError) as e:
        other.restore(path)
    assert e.value.status == gl.GL_EINVAL
    junk = tmp_path / "junk.ckpt"
    junk.write_bytes(b"not a checkpoint at all" * 10)
    with pytest.raises(gl.GlasmaError) as e:
        other.restore(str(junk))
    assert e.value.status == gl.GL_EINVAL
    # a truncated file is refused as well
    data = open(path, "rb").read()
    (tmp_path / "cut.ckpt").write_bytes(data[: len(data) // 2])
    same = _blank(gl, 64, correlators=False)
    with pytest.raises(gl.GlasmaError) as e:
        same.restore(str(tmp_path / "cut.ckpt"))
    assert e.value.status == gl.GL_EINVAL
    with pytest.raises(gl.GlasmaError) as e:
        same.run(1)                 # not initialised by the failed restore
    assert e.value.status == gl.GL_ESTATE
    # a well-formed file whose scalars or species counts are out of range
    import ctypes
    scal = 16 + ctypes.sizeof(gl.glasma.LatticeDesc)     # magic, version words, lattice description
    assert int(np.frombuffer(data, np.int64, 1, scal)[0]) == a.info()[2]   # the step index comes first
    bad = bytearray(data)
    bad[scal:scal + 8] = np.int64(-5).tobytes()
    (tmp_path / "neg.ckpt").write_bytes(bytes(bad))
    with pytest.raises(gl.GlasmaError) as e:
        same.restore(str(tmp_path / "neg.ckpt"))
    assert e.value.status == gl.GL_EINVAL and "inconsistent" in str(e.value)
    words = np.frombuffer(data, np.int64, (len(data) - scal) // 8, scal)
    k = scal + 8 * int(np.nonzero(words == 1200)[0][0])   # the first species' count
    bad = bytearray(data)
    bad[k:k + 8] = np.int64(5000).tobytes()
    (tmp_path / "count.ckpt").write_bytes(bytes(bad))
    with pytest.raises(gl.GlasmaError) as e:
        same.restore(str(tmp_path / "count.ckpt"))
    assert e.value.status == gl.GL_EINVAL and "species" in str(e.value)


def test_nan_set_from_the_host_is_reported(gl):
    """A NaN placed in E through gl_set_state: the diagnostics return
    GL_ENUMERIC, and gl_run with a check period names the first step whose
    state or series held a non-finite value.  Without checks gl_run returns
    GL_OK (nothing is checked)."""
    N = 16
    U, E, phi, pi = si.random_state(5, N, link_kind="near", eps=0.3)
    E[1, 37, 4] = np.nan
    soa = (si.links_to_soa(U), si.links_to_soa(E), si.alg_to_soa(phi), si.alg_to_soa(pi))
    ev = gl.Event(N, 2.0, 0.125, precision=64, max_steps=32, max_particles=256)
    ev.set_state(*soa, 3)
    d = ev.diagnostics()
    assert d["status"] == gl.GL_ENUMERIC and d["nonfinite"] == 1
    ev.set_check_period(4)
    with pytest.raises(gl.GlasmaError) as e:
        ev.run(9)
    assert e.value.status == gl.GL_ENUMERIC
    assert "step n = 7" in str(e.value)        # the first checked state, after 4 steps from n = 3
    # a healthy event passes the same checks, with particles
    U, E, phi, pi = si.random_state(6, N, link_kind="near", eps=0.3)
    ok = gl.Event(N, 2.0, 0.125, precision=64, max_steps=32, max_particles=256)
    ok.set_state(si.links_to_soa(U), si.links_to_soa(E), si.alg_to_soa(phi), si.alg_to_soa(pi), 3)
    ok.add_species(1.27, 1.0, gl.KIND_HEAVY_QUARK, 200, 3)
    ok.set_check_period(4)
    ok.run(9)
    quiet = gl.Event(N, 2.0, 0.125, precision=64, max_steps=32, max_particles=256)
    quiet.set_state(*soa, 3)
    quiet.run(3)


def test_nan_in_the_particles_is_reported_through_the_series(gl):
    """A particle whose momentum is NaN makes its species' series row
    non-finite; the end-of-run check names the step of that row."""
    N = 16
    U, E, phi, pi = si.random_state(8, N, link_kind="near", eps=0.3)
    ev = gl.Event(N, 2.0, 0.125, precision=64, max_steps=32, max_particles=256)
    ev.set_state(si.links_to_soa(U), si.links_to_soa(E), si.alg_to_soa(phi), si.alg_to_soa(pi), 3)
    ev.add_species(1.27, 1.0, gl.KIND_HEAVY_QUARK, 100, 3, tau_form_fm=0.0)
    d = ev.get_particles()
    d["p"][0, 17] = np.nan
    ev.set_particles([(1.27, 1.0, gl.KIND_HEAVY_QUARK, 0.0)], d["cell"], d["off"], d["eta"], d["p"],
                     d["Q"], d["p0"], d["species"])
    ev.set_check_period(100)
    with pytest.raises(gl.GlasmaError) as e:
        ev.run(5)
    assert e.value.status == gl.GL_ENUMERIC
    assert "step n = 4" in str(e.value)        # the first push, 3 -> 4


def test_matching_iteration_cap_gives_enotconv(gl):
    ev = gl.Event(32, 4.0, 0.125, precision=64, max_steps=8)
    ev.set_match_params(1, 1e-13)
    with pytest.raises(gl.GlasmaError) as e:
        ev.init_glasma(1.0, 0.2, 1, 7)
    assert e.value.status == gl.GL_ENOTCONV
    ev.set_match_params(100, 1e-13)
    ev.init_glasma(1.0, 0.2, 1, 7)
    with pytest.raises(gl.GlasmaError):
        ev.set_match_params(0, 1e-13)


@pytest.mark.parametrize("prec,tol", [(64, 1e-12), (32, 1e-4)])
def test_both_casimirs_conserved(gl, prec, tol):
    """q2 = 4 and q3 = 10/3 for every particle after a coupled run (Sec. 1:
    the colour charge's Casimirs are conserved by Wong's equations).  In FP32
    each step's three unitary rotations of Q round at 2^-24 relative, so over
    30 steps the Casimirs may drift by up to about 30 * 3 * 8 * 2^-24 * q2
    (6e-5) in the worst case; 1e-4 bounds that."""
    ev = _coupled_event(gl, prec, correlators=False)
    d0 = ev.diagnostics()
    ev.run(30)
    d = ev.diagnostics()
    print("FP%d casimir deviations: q2 %.2e, q3 %.2e" % (prec, d["casimir2_dev"], d["casimir3_dev"]))
    assert d0["casimir3_dev"] < tol and d0["casimir2_dev"] < tol
    assert d["casimir2_dev"] < tol and d["casimir3_dev"] < tol


def test_batch_holds_its_events(gl):
    evs = []
    for k, N in enumerate((24, 32)):
        ev = gl.Event(N, N * 0.125, 0.125, precision=32, max_steps=40, max_particles=300)
        ev.init_glasma(1.0, 0.2, 1, 70 + k)
        ev.add_species(1.27, 2.0, gl.KIND_HEAVY_QUARK, 300, 80 + k)
        evs.append(ev)
    b = gl.Batch(evs)
    b.run(3)
    ev = evs[0]
    U, E, phi, pi, n = ev.get_state()
    calls = [lambda: ev.run(1), lambda: ev.evolve_fields(1), lambda: ev.push_particles(),
             lambda: ev.add_species(1.27, 0.0, gl.KIND_HEAVY_QUARK, 10, 1),
             lambda: ev.init_glasma(1.0, 0.2, 1, 1), lambda: ev.set_state(U, E, phi, pi, n),
             lambda: ev.set_sort_period(4), lambda: ev.set_match_params(10, 1e-12)]
    for c in calls:
        with pytest.raises(gl.GlasmaError) as e:
            c()
        assert e.value.status == gl.GL_ESTATE
    with pytest.raises(gl.GlasmaError) as e:
        gl.Batch(evs)               # already held
    assert e.value.status == gl.GL_ESTATE
    assert ev.series().shape[0] == 3          # the getters work
    ev.diagnostics()
    with pytest.raises(gl.GlasmaError) as e:
        ev.close()                  # the batch still uses its memory
    assert e.value.status == gl.GL_ESTATE
    b.close()
    ev.run(2)
    assert ev.info()[2] == n + 2


def test_charges_of_the_wrong_shape_are_refused(gl):
    import torch
    ev = gl.Event(16, 2.0, 0.125, precision=64, max_steps=4)
    for shape in ((1, 2, 8, 256), (2, 2, 8, 255), (2, 2, 4, 256), (2, 8, 256), (2, 2, 8, 15, 17)):
        rho = torch.zeros(shape, dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError):
            ev.init_glasma_from_charges(rho, 0.2)
    with pytest.raises(ValueError):
        ev.init_glasma_from_charges(torch.zeros((2, 1, 8, 256), dtype=torch.float32, device="cuda"), 0.2)
    ev.init_glasma_from_charges(torch.zeros((2, 1, 8, 16, 16), dtype=torch.float64, device="cuda"), 0.2)
