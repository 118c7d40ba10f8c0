"""The initial condition (Sec. 1 "Glasma": MV charges, Poisson solve, Wilson
lines, matching, initial longitudinal field) against the oracle at the sizes
and sheet counts the workloads use: 512^2 (three radix-8 FFT stages), 384^2
(a radix-3 stage, one of the batched event sizes), and 17 sheets per nucleus
(the sheets are drawn and transformed in chunks of 8, so 17 crosses two chunk
boundaries).  Both entry points: charges drawn on the device
(gl_init_glasma) and charges handed in by the caller
(gl_init_glasma_from_charges), here the oracle's own draw uploaded.

Tolerance: 1e-12 absolute on the O(1) link entries and on pi_0, as for the
small lattices (the two sides differ by FFT and exponential rounding, and
each side's Newton solve stops below a 1e-13 residual)."""
import functools
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

G2MU, M_IR, SEED = 2.767, 0.2, 2307079997
A_FM = 10.0 / 512          # the paper-scale lattice spacing, L = N a


@pytest.fixture(scope="module")
def gl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07999_amd as g
    g.lib()
    return g


def _params(N, sheets):
    a_gev = A_FM / 0.1973269804
    return N * A_FM, G2MU * a_gev / math.sqrt(sheets), (M_IR * a_gev) ** 2


@functools.lru_cache(maxsize=None)
def _oracle(N, sheets):
    from oracle import oracle as orc
    L, sigma, m2 = _params(N, sheets)
    V = [orc.wilson_line(N, sigma, m2, sheets, SEED, nuc) for nuc in (0, 1)]
    s, rc, res = orc.init_glasma(N, sigma, m2, sheets, SEED, 0.125)
    assert rc == 0
    rho = np.stack([np.stack([orc.mv_charges(N, sigma, SEED, nuc, sh).T for sh in range(sheets)])
                    for nuc in (0, 1)])
    return V, s, rho


def _compare(gl, ev, N, sheets, label):
    from tests import gpu_helpers as H
    V, s, _ = _oracle(N, sheets)
    errs = {}
    for nuc in (0, 1):
        errs["V%d" % nuc] = np.abs(ev.wilson_line(nuc) - V[nuc].T).max()
    U, E, phi, pi, n = ev.get_state()
    Uo, Eo, phio, pio = H.state_oracle_to_soa(s)
    errs["U"] = np.abs(U - Uo).max()
    errs["pi"] = np.abs(pi - pio).max()
    errs["phi"] = np.abs(phi - phio).max()
    print("%s N=%d sheets=%d: %s" % (label, N, sheets, {k: "%.1e" % v for k, v in errs.items()}))
    assert n == 1 and np.abs(E).max() == 0
    for k, v in errs.items():
        assert v < 1e-12, (k, v)
    assert np.abs(pio).max() > 1e-3         # a non-trivial initial field


@pytest.mark.parametrize("N,sheets", [(512, 1), (384, 1), (32, 17)])
def test_init_from_mv_draw_matches_oracle(gl, N, sheets):
    L, _, _ = _params(N, sheets)
    ev = gl.Event(N, L, 0.125, precision=64, max_steps=1)
    ev.init_glasma(G2MU, M_IR, sheets, SEED)
    _compare(gl, ev, N, sheets, "MV draw")
    ev.close()


@pytest.mark.parametrize("N,sheets,shape5", [(512, 1, False), (384, 1, True), (32, 17, False)])
def test_init_from_caller_charges_matches_oracle(gl, N, sheets, shape5):
    import torch
    L, _, _ = _params(N, sheets)
    _, _, rho = _oracle(N, sheets)
    t = torch.from_numpy(np.ascontiguousarray(rho)).to("cuda")
    if shape5:
        t = t.reshape(2, sheets, 8, N, N)
    ev = gl.Event(N, L, 0.125, precision=64, max_steps=1)
    ev.init_glasma_from_charges(t, M_IR)
    _compare(gl, ev, N, sheets, "caller charges")
    ev.close()


def test_device_draw_equals_caller_charges_bitwise(gl):
    """The row pass that draws the charges itself gives bitwise the state of
    the same charges handed in: 17 sheets cross the chunks at sheets 8, 16."""
    import torch
    N, sheets = 32, 17
    L, sigma, _ = _params(N, sheets)
    a = gl.Event(N, L, 0.125, precision=64, max_steps=1)
    a.init_glasma(G2MU, M_IR, sheets, SEED)
    rho = np.stack([np.stack([a.draw_charges(SEED, nuc, sh, sigma) for sh in range(sheets)]) for nuc in (0, 1)])
    b = gl.Event(N, L, 0.125, precision=64, max_steps=1)
    b.init_glasma_from_charges(torch.from_numpy(rho).to("cuda"), M_IR)
    for x, y in zip(a.get_state()[:4], b.get_state()[:4]):
        assert np.array_equal(x, y)
    for nuc in (0, 1):
        assert np.array_equal(a.wilson_line(nuc), b.wilson_line(nuc))
