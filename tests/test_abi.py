"""The C-ABI library loads without a GPU, exports every symbol the header
declares, and its host-only logic (sizes, argument checks, the derivative of
the broadening series) behaves as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gl_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def gl():
    import paper_2307_07999_amd as g
    return g


def test_every_declared_symbol_is_exported(gl):
    names = _declared("glasma.h")
    assert len(names) > 20
    L = gl.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_required_bytes_and_validation(gl):
    small = gl.required_bytes(32, 4.0, max_steps=64, max_particles=1000)
    big = gl.required_bytes(512, 10.0, max_steps=410, max_particles=700000)
    assert 0 < small < big
    assert gl.required_bytes(512, 10.0, precision=32) < gl.required_bytes(512, 10.0, precision=64)
    for bad in (dict(N=1), dict(N=2000), dict(precision=16), dict(dtau_over_a=0.0)):
        kw = dict(N=16, L_fm=2.0, dtau_over_a=0.125, precision=64)
        kw.update(bad)
        with pytest.raises(gl.GlasmaError) as e:
            gl.required_bytes(kw["N"], kw["L_fm"], kw["dtau_over_a"], kw["precision"])
        assert e.value.status == -1


@pytest.mark.parametrize("prec,rec_bytes", [(64, 14 * 8), (32, 16 * 4)])
def test_particle_capacity_stays_within_32_bit_record_offsets(gl, prec, rec_bytes):
    # the record of every slot spans rec_bytes of chunk planes over all slots;
    # its byte offsets must stay below 2^31
    top = ((2**31 - 256) // rec_bytes) // 256 * 256
    assert top * rec_bytes < 2**31
    assert gl.max_particles(prec) == top
    assert gl.required_bytes(16, 2.0, precision=prec, max_particles=top) > top * rec_bytes
    for bad in (top + 1, 2**28 - 8192):
        with pytest.raises(gl.GlasmaError) as e:
            gl.required_bytes(16, 2.0, precision=prec, max_particles=bad)
        assert e.value.status == -1
    with pytest.raises(gl.GlasmaError):
        gl.max_particles(16)


def test_event_create_checks_workspace_without_touching_device(gl):
    from paper_2307_07999_amd import glasma as G
    d = G.LatticeDesc(16, 2.0, 0.125, 64, 16, 32, 0)
    need = gl.required_bytes(16, 2.0, max_steps=32)
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(need + 512)
    aligned = (ctypes.addressof(buf) + 255) // 256 * 256
    assert G.lib().gl_event_create(ctypes.byref(d), ctypes.c_void_p(aligned), need - 1, None,
                                   ctypes.byref(h)) == G.GL_ENOMEM
    assert G.lib().gl_event_create(ctypes.byref(d), ctypes.c_void_p(aligned + 8), need, None,
                                   ctypes.byref(h)) == G.GL_EINVAL
    assert G.lib().gl_event_create(ctypes.byref(d), ctypes.c_void_p(aligned), need, None,
                                   ctypes.byref(h)) == G.GL_OK
    # calls that need initialised fields are refused before any device work
    assert G.lib().gl_evolve_fields(h, 1) == G.GL_ESTATE
    assert G.lib().gl_run(h, 1) == G.GL_ESTATE
    assert G.lib().gl_push_particles(h) == G.GL_ESTATE
    bad = G.SpeciesDesc(0.0, 0.0, 0, -1.0)
    assert G.lib().gl_add_species(h, ctypes.byref(bad), 10, 1, None) == G.GL_EINVAL
    assert b"massless" in G.lib().gl_last_error() or b"m_T" in G.lib().gl_last_error()
    G.lib().gl_event_destroy(h)


def test_rates_from_series_matches_oracle(gl, orc):
    g = np.random.default_rng(3)
    rows = 40
    series = np.zeros((rows, 4))
    series[7:, 3] = 100
    series[7:, :3] = np.cumsum(g.normal(size=(rows - 7, 3)), axis=0) * 100
    got = gl.rates_from_series(series, 0.125)
    ks, want = orc.coefficients(series, 0.125)
    assert np.allclose(got[ks], want, rtol=0, atol=1e-12)
    assert np.all(got[:7] == 0)


def test_status_strings(gl):
    L = gl.lib()
    for s in range(-6, 1):
        assert L.gl_status_string(s)


def test_binding_checks_arguments_without_asserts():
    """The binding's host-array checks raise real exceptions (they stay on
    under python -O; the C side trusts the sizes it is given)."""
    from paper_2307_07999_amd import glasma as G
    with pytest.raises(TypeError):
        G._d(np.zeros(4, np.float32))
    with pytest.raises(TypeError):
        G._d(np.zeros((4, 4))[:, ::2])            # not contiguous
    with pytest.raises(TypeError):
        G._i(np.zeros(4, np.int64))
    with pytest.raises(TypeError):
        G._f(np.zeros(4))
    with pytest.raises(ValueError):
        G.scan_statistics(np.zeros((2, 5, 3)), G.KIND_HEAVY_QUARK, 0.01, 0.02)
