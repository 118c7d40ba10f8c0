"""Parity at the paper-scale size (512^2, L = 10 fm, 7 x 1e5 particles) in the
launch configuration the benchmark times, on outputs the oracle computes one
by one: sampled sites of one field step (with site fields) and sampled
particles of one push.  Sample sites include the lattice edges and corners."""
import numpy as np
import pytest

from tests import gpu_helpers as H
from tests import seeded_inputs as si

pytestmark = pytest.mark.gpu

N, L = 512, 10.0
HB = 0.1973269804


@pytest.fixture(scope="module")
def gl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07999_amd as g
    g.lib()
    return g


def _sites(seed, k, n=N):
    g = np.random.default_rng(seed)
    edge = [0, n - 1, n * (n - 1), n * n - 1, n // 2, n * 7 + n - 1, n * (n - 1) + 5]
    return np.array(sorted(set(edge) | set(g.integers(0, n * n, k).tolist())), np.int32)


SPECIES = [(1.27, 0.0, 0), (1.27, 2.0, 0), (1.27, 5.0, 0), (4.18, 0.0, 0), (4.18, 2.0, 0),
           (4.18, 5.0, 0), (0.0, 10.0, 1)]


@pytest.mark.parametrize("prec", [64, 32])
def test_field_step_and_site_fields_sampled(gl, orc, prec):
    U, E, phi, pi = si.random_state(512, N, link_kind="near", eps=0.3, e_scale=0.1,
                                    phi_scale=0.1, pi_scale=0.1)
    s = orc.State(N)
    s.U, s.E, s.phi, s.pi, s.n = U, E, phi, pi, 40
    ev = gl.Event(N, L, 0.125, precision=prec, max_steps=64, max_particles=1000)
    ev.set_state(*H.state_oracle_to_soa(s), 40)
    ev.add_species(1.27, 0.0, gl.KIND_HEAVY_QUARK, 1000, 3)     # so that site fields are made
    ev.evolve_fields(1)
    Ug, Eg, phig, pig, n = ev.get_state()
    Fg = ev.site_fields()
    sites = _sites(prec, 300)
    Un, En, phin, pin, F = orc.field_step_sites(s, 0.125, sites)
    tol = 1e-12 if prec == 64 else 2e-5
    assert np.abs(Ug[:, :, sites] - np.transpose(Un, (1, 2, 0))).max() < tol
    assert np.abs(Eg[:, :, sites] - np.transpose(En, (1, 2, 0))).max() < tol
    assert np.abs(phig[:, sites] - phin.T).max() < tol
    assert np.abs(pig[:, sites] - pin.T).max() < tol
    scale = max(1.0, np.abs(F).max())
    assert np.abs(Fg[:, :, sites] - np.transpose(F, (1, 2, 0))).max() < tol * scale


@pytest.mark.parametrize("prec", [64, 32])
def test_field_step_sampled_on_the_largest_lattice(gl, orc, prec):
    """N = 1024, the largest lattice the library accepts: 2^20 sites, the
    largest byte offsets of the field planes and of the site-field record.
    Sampled sites of one field step with site fields, the lattice's last
    row and column included."""
    n = 1024
    U, E, phi, pi = si.random_state(1024 + prec, n, link_kind="near", eps=0.3, e_scale=0.1,
                                    phi_scale=0.1, pi_scale=0.1)
    s = orc.State(n)
    s.U, s.E, s.phi, s.pi, s.n = U, E, phi, pi, 40
    ev = gl.Event(n, 20.0, 0.125, precision=prec, max_steps=8, max_particles=1000)
    ev.set_state(*H.state_oracle_to_soa(s), 40)
    ev.add_species(1.27, 0.0, gl.KIND_HEAVY_QUARK, 1000, 3)     # so that site fields are made
    ev.evolve_fields(1)
    Ug, Eg, phig, pig, steps = ev.get_state()
    assert steps == 41
    Fg = ev.site_fields()
    sites = _sites(prec + 1, 300, n)
    Un, En, phin, pin, F = orc.field_step_sites(s, 0.125, sites)
    tol = 1e-12 if prec == 64 else 2e-5
    assert np.abs(Ug[:, :, sites] - np.transpose(Un, (1, 2, 0))).max() < tol
    assert np.abs(Eg[:, :, sites] - np.transpose(En, (1, 2, 0))).max() < tol
    assert np.abs(phig[:, sites] - phin.T).max() < tol
    assert np.abs(pig[:, sites] - pin.T).max() < tol
    scale = max(1.0, np.abs(F).max())
    assert np.abs(Fg[:, :, sites] - np.transpose(F, (1, 2, 0))).max() < tol * scale


def test_push_sampled_paper_scale(gl, orc):
    """One coupled step of the 7 x 1e5 ensemble on 512^2 (FP64); 3000
    particles of all species recomputed by the oracle."""
    U, E, phi, pi = si.random_state(513, N, link_kind="near", eps=0.3, e_scale=0.1,
                                    phi_scale=0.1, pi_scale=0.1)
    s = orc.State(N)
    s.U, s.E, s.phi, s.pi, s.n = U, E, phi, pi, 40
    ev = gl.Event(N, L, 0.125, precision=64, max_steps=64, max_particles=700000)
    ev.set_state(*H.state_oracle_to_soa(s), 40)
    for k, (m, p0, kind) in enumerate(SPECIES):
        ev.add_species(m, p0, kind, 100000, 1000 + k)
    before = ev.get_particles()
    mass = [ev.species_info(k)[1] for k in range(len(SPECIES))]
    nform = [ev.species_info(k)[0] for k in range(len(SPECIES))]
    assert max(nform) <= 40
    ev.evolve_fields(1)
    ev.push_particles()
    after = ev.get_particles()
    g = np.random.default_rng(5)
    pick = np.sort(g.choice(700000, 3000, replace=False))
    P = H.particles_gpu_to_oracle(orc, before).subset(pick)
    cells = np.unique(P.cell[:, 0] + N * P.cell[:, 1]).astype(np.int32)
    _, _, _, _, Fs = orc.field_step_sites(s, 0.125, cells)
    Ffull = np.zeros((N * N, 6, 8))
    Ffull[cells] = Fs
    ser = orc.particle_step(N, 40, 0.125, s.U, s.phi, Ffull, P, mass, nform)
    A = H.particles_gpu_to_oracle(orc, after).subset(pick)
    assert np.array_equal(A.cell, P.cell)
    for k in ("off", "eta", "p", "Q"):
        assert np.abs(getattr(A, k) - getattr(P, k)).max() < 1e-12, k
    assert ser[:, 3].sum() == 3000


def test_push_sampled_paper_scale_fp32(gl, orc):
    """The FP32 push of the same step (7 x 1e5 particles on 512^2): the
    FP64 oracle recomputes 3000 particles from the FP32 event's own state
    and particles, read back, so both sides start from the same numbers and
    differ only by one step of FP32 arithmetic (its site fields included).
    Offsets, rapidities, momenta and charges agree to 2e-6 of each
    quantity's largest value (one step: about 2e-7, FP32 rounding).  A crossing may be decided the other way only
    where the oracle's offset lands within 1e-4 of a cell edge, where both
    decisions are valid; every other cell agrees exactly."""
    U, E, phi, pi = si.random_state(513, N, link_kind="near", eps=0.3, e_scale=0.1,
                                    phi_scale=0.1, pi_scale=0.1)
    s = orc.State(N)
    s.U, s.E, s.phi, s.pi, s.n = U, E, phi, pi, 40
    ev = gl.Event(N, L, 0.125, precision=32, max_steps=64, max_particles=700000)
    ev.set_state(*H.state_oracle_to_soa(s), 40)
    for k, (m, p0, kind) in enumerate(SPECIES):
        ev.add_species(m, p0, kind, 100000, 1000 + k)
    before = ev.get_particles()
    mass = [ev.species_info(k)[1] for k in range(len(SPECIES))]
    nform = [ev.species_info(k)[0] for k in range(len(SPECIES))]
    U32, E32, phi32, pi32, n32 = ev.get_state()          # the FP32 state the event holds
    s32 = H.state_soa_to_oracle(orc, U32, E32, phi32, pi32, N, n32)
    assert n32 == 40
    ev.evolve_fields(1)
    ev.push_particles()
    after = ev.get_particles()
    g = np.random.default_rng(7)
    pick = np.sort(g.choice(700000, 3000, replace=False))
    P = H.particles_gpu_to_oracle(orc, before).subset(pick)
    cells = np.unique(P.cell[:, 0] + N * P.cell[:, 1]).astype(np.int32)
    _, _, _, _, Fs = orc.field_step_sites(s32, 0.125, cells)
    Ffull = np.zeros((N * N, 6, 8))
    Ffull[cells] = Fs
    ser = orc.particle_step(N, 40, 0.125, s32.U, s32.phi, Ffull, P, mass, nform)
    assert ser[:, 3].sum() == 3000
    A = H.particles_gpu_to_oracle(orc, after).subset(pick)
    same = np.all(A.cell == P.cell, axis=1)
    edge = np.min(np.abs(0.5 - np.abs(P.off)), axis=1)
    print("FP32 push at 512^2: %d of 3000 cells differ" % int((~same).sum()))
    assert (~same).sum() <= 3 and np.all(edge[~same] < 1e-4)
    for k in ("off", "eta", "p", "Q"):
        a, b = getattr(A, k)[same], getattr(P, k)[same]
        err = np.abs(a - b).max() / np.abs(b).max()
        print("FP32 push at 512^2, %s: %.2e of its largest value" % (k, err))
        assert err < 2e-6, k
    ev.close()


def _pick(d, idx):
    return {k: (v[:, idx] if v.ndim == 2 else v[idx]) for k, v in d.items()}


@pytest.mark.parametrize("prec", [64, 32])
def test_push_at_the_particle_capacity(gl, orc, prec):
    """The largest ensemble an event takes, whose record planes end just
    below 2^31 bytes (the limit of the 32-bit buffer offsets): one coupled
    step on a 64^2 lattice.  FP64: 3000 particles, the last-created ones among
    them (the highest slots before the sort), recomputed by the oracle to
    1e-12.  FP32: every particle formed and counted, charges on their Casimir
    shells, the state finite."""
    n_lat, l_lat = 64, 8.0
    cap = gl.max_particles(prec)
    n = cap // 256 * 256
    U, E, phi, pi = si.random_state(514, n_lat, link_kind="near", eps=0.3, e_scale=0.1,
                                    phi_scale=0.1, pi_scale=0.1)
    s = orc.State(n_lat)
    s.U, s.E, s.phi, s.pi, s.n = U, E, phi, pi, 40
    ev = gl.Event(n_lat, l_lat, 0.125, precision=prec, max_steps=48, max_particles=cap)
    ev.set_state(*H.state_oracle_to_soa(s), 40)
    ev.add_species(1.27, 2.0, gl.KIND_HEAVY_QUARK, n, 1234)
    mass, nform = ev.species_info(0)[1], ev.species_info(0)[0]
    print("capacity %d, particles %d (FP%d)" % (cap, n, prec))
    if prec == 64:
        g = np.random.default_rng(6)
        pick = np.unique(np.concatenate([np.arange(n - 100, n), g.choice(n, 2900, replace=False)]))
        before = _pick(ev.get_particles(), pick)
    ev.evolve_fields(1)
    ev.push_particles()
    ser = ev.series()
    assert ser[-1, 0, 3] == n                     # every particle pushed and counted
    d = ev.diagnostics()
    assert d["nonfinite"] == 0
    assert d["casimir2_dev"] < (1e-12 if prec == 64 else 1e-4)
    assert d["casimir3_dev"] < (1e-12 if prec == 64 else 1e-4)
    if prec == 64:
        after = _pick(ev.get_particles(), pick)
        P = H.particles_gpu_to_oracle(orc, before)
        cells = np.unique(P.cell[:, 0] + n_lat * P.cell[:, 1]).astype(np.int32)
        _, _, _, _, Fs = orc.field_step_sites(s, 0.125, cells)
        Ffull = np.zeros((n_lat * n_lat, 6, 8))
        Ffull[cells] = Fs
        so = orc.particle_step(n_lat, 40, 0.125, s.U, s.phi, Ffull, P, [mass], [nform])
        A = H.particles_gpu_to_oracle(orc, after)
        assert np.array_equal(A.cell, P.cell)
        for k in ("off", "eta", "p", "Q"):
            assert np.abs(getattr(A, k) - getattr(P, k)).max() < 1e-12, k
        assert so[:, 3].sum() == len(pick)
    ev.close()
