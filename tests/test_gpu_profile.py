"""Kernel timing through the C-ABI (gl_profile_*): a sampled launch of the
field step or a push goes through the launch form that takes the timing
events itself, the others are bracketed by events on the stream.  Timing
must not change what is computed (the profiled run equals the plain one bit
for bit, with sorts applied by the push and both correlators on), and the
samples follow the period."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07999_amd as g
    g.lib()
    return g


def _event(gl, prec):
    ev = gl.Event(48, 6.0, 0.125, precision=prec, max_steps=64, max_particles=2600,
                  static_correlator=True, lightlike_correlator=True)
    ev.init_glasma(1.0, 0.2, 2, 71)
    ev.add_species(1.27, 2.0, gl.KIND_HEAVY_QUARK, 1200, 72)
    ev.add_species(0.0, 10.0, gl.KIND_JET, 1400, 73)
    ev.static_start(0.0)
    ev.lightlike_start(0.0)
    return ev


@pytest.mark.parametrize("prec", [64, 32])
def test_profiled_run_equals_plain_run_and_samples_follow_the_period(gl, prec):
    steps, period = 40, 3
    plain, timed = _event(gl, prec), _event(gl, prec)
    timed.profile(True, period=period)
    plain.run(steps)
    timed.run(steps)
    ms, cnt = timed.profile_read()
    for x, y in zip(plain.get_state()[:4], timed.get_state()[:4]):
        assert np.array_equal(x, y)
    pa, pb = plain.get_particles(), timed.get_particles()
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k
    assert np.array_equal(plain.series(), timed.series())
    assert np.array_equal(plain.static_broadening(), timed.static_broadening())
    assert np.array_equal(plain.lightlike_broadening(), timed.lightlike_broadening())
    print("profile classes: launches %s, ms %s" % (cnt.tolist(), np.round(ms, 4).tolist()))
    # every field step of the run is one launch of class 0; launches 0, p, 2p, ... are timed
    assert cnt[0] == (steps + period - 1) // period
    # pushes: the plain ones (class 2) and those applying a sort (class 4)
    assert cnt[2] > 0 and cnt[4] > 0 and cnt[1] > 0 and cnt[3] > 0
    assert np.all(ms[cnt > 0] > 0.0)
    # each sampled launch of this small lattice takes well under a millisecond
    assert np.all(ms[cnt > 0] / cnt[cnt > 0] < 1.0)
    # reading clears: a second read without launches returns nothing
    ms2, cnt2 = timed.profile_read()
    assert not cnt2.any() and not ms2.any()
    plain.close()
    timed.close()
