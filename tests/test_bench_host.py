"""Host logic of bench.py (CPU only): the workload's step count, the
algorithmic byte counts the roofline line divides by, the rule that stale
traffic figures are reported as null, and the single-GPU refusal."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_coupled_steps_of_the_workloads():
    # dtau = a/8 up to tau = 1 fm, less the first half step of the leapfrog
    assert bench.coupled_steps(32, 4.0) == 63      # a = 0.125 fm: 64 steps of a/8
    assert bench.coupled_steps(512, 10.0) == 409   # a = 10/512 fm: ceil(409.6) - 1
    assert bench.coupled_steps(bench.N, bench.L_FM) == 409


@pytest.mark.parametrize("prec,ts", [(64, 8), (32, 4)])
def test_algorithmic_bytes_follow_the_layouts(prec, ts):
    b = bench.alg_bytes(prec)
    link_rows = 2 * (2 * 3 * 2)          # two links, two stored rows of 3 complex entries
    state = link_rows + 2 * 8 + 8 + 8    # U, E_x and E_y, phi, pi
    site_fields = 6 * 8                  # E and B, eight colours each
    assert b["field_step"] == (2 * state + site_fields) * ts
    record = 2 + 1 + 3 + 8               # offsets in the cell, rapidity, momenta, charge
    cells, species = 8, 4
    assert b["push"] == (cells + species + record * ts) + (site_fields + 8) * ts + (cells + record * ts)
    assert (b["field_step"], b["push"]) == ((1280, 692) if prec == 64 else (640, 356))


def test_recorded_traffic_is_near_the_algorithmic_bytes():
    for prec in (64, 32):
        t = bench.measured_traffic("field_step", prec)
        if t is None:   # bench then reports traffic as null until the counters are taken again
            pytest.skip("traffic figures missing or taken on other kernel sources")
        alg = bench.alg_bytes(prec)["field_step"] * bench.N * bench.N
        assert 1.0 <= sum(t) / alg < 1.2
        p = bench.measured_traffic("push", prec)
        assert p is not None and p[0] > 0 and p[1] > 0


def test_traffic_from_other_kernel_sources_is_null(tmp_path, monkeypatch):
    text = open(bench.TRAFFIC_FILE).read()
    fresh = tmp_path / "fresh.md"
    fresh.write_text(text + "\nsource hash: `%s`\n" % bench.kernel_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(fresh))
    assert bench.measured_traffic("field_step", 64) is not None
    stale = tmp_path / "traffic.md"
    stale.write_text(text + "\nsource hash: `0123456789abcdef`\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.measured_traffic("field_step", 64) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("field_step", 64) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_observable_errors_are_per_curve_maxima_over_species():
    """The FP32 twin's deviation: per curve, max |got - want| / max |want|,
    the largest over species, over the rows both curves have."""
    import numpy as np
    want = [{"a": np.array([1.0, 2.0, 4.0]), "b": np.array([0.0, -2.0])},
            {"a": np.array([10.0, 10.0])}]
    got = [{"a": np.array([1.0, 2.1, 4.0, 99.0]), "b": np.array([0.0, -2.0])},
           {"a": np.array([10.0, 9.0])}]
    err = bench.observable_errors(got, want)
    assert err["a"] == pytest.approx(max(0.1 / 4.0, 1.0 / 10.0))
    assert err["b"] == 0.0
    assert bench.observable_errors([{"c": np.zeros(3)}], [{"c": np.zeros(3)}]) == {"c": 0.0}


def test_valu_counts_are_read_for_the_current_kernel_sources(tmp_path, monkeypatch):
    """The committed SQ-counter summaries hold the kernels' VALU instruction
    counts for the current kernel sources; the issue peak is the chip's (one
    wave64 instruction per SIMD every 4 cycles at 2.4 GHz); a count taken on
    other sources, a missing file or a missing row reads as None."""
    assert bench.VALU_ISSUE_PEAK == 256 * 4 * 2.4e9 / 4
    for prec, t in ((64, "double"), (32, "float")):
        fs, push = bench.measured_valu("gl::k_field_step<%s>" % t, prec), bench.measured_valu("gl::k_push<%s>" % t, prec)
        if fs is None:   # bench then reports the issue fraction as null until the counters are taken again
            pytest.skip("SQ counts missing or taken on other kernel sources")
        assert push and fs != push
        # both kernels run one wave64 per 64 lanes: a few thousand VALU instructions per wave
        assert 1000 < fs / 8192 < 4000
    text = open(bench.SQ_FILES[32]).read()
    stale = tmp_path / "stale.md"
    stale.write_text(text.replace(bench.kernel_source_hash(), "0123456789abcdef"))
    monkeypatch.setitem(bench.SQ_FILES, 32, str(stale))
    assert bench.measured_valu("gl::k_field_step<float>", 32) is None
    monkeypatch.setitem(bench.SQ_FILES, 32, str(tmp_path / "missing.md"))
    assert bench.measured_valu("gl::k_field_step<float>", 32) is None
    monkeypatch.setitem(bench.SQ_FILES, 32, str(bench.SQ_FILES[64]))
    assert bench.measured_valu("gl::k_field_step<float>", 32) is None   # no such row there


def test_issue_fraction_in_the_kernel_rates():
    """kernel_rates reports each kernel's share of the VALU issue peak from
    its counted instructions and the measured duration."""
    ab = bench.alg_bytes(32)
    units = {"field_step": 512 * 512, "push": 700000}
    r = bench.kernel_rates(32, {"field_step": 36.6, "push": 37.4}, units, ab)
    valu = bench.measured_valu("gl::k_field_step<float>", 32)
    if valu is None:
        assert r["field_step"]["valu_issue_frac"] is None
        return
    want = valu / 36.6e-6 / bench.VALU_ISSUE_PEAK
    assert abs(r["field_step"]["valu_issue_frac"] - want) < 1e-12
    assert 0.5 < r["field_step"]["valu_issue_frac"] < 1.0


def test_kernel_rates_alone_and_against_the_ceiling():
    """Each kernel's rate alone is its units over its duration, and the
    ceiling fractions are the GB/s over the measured copy rate."""
    ab = bench.alg_bytes(64)
    units = {"field_step": 512 * 512, "push": 700000}
    avg = {"field_step": 68.0, "push": 65.0}
    r = bench.kernel_rates(64, avg, units, ab, ceiling=6300.0)
    assert abs(r["field_step"]["site_updates_per_s"] - 512 * 512 / 68.0e-6) < 1.0
    assert abs(r["push"]["particle_steps_per_s"] - 700000 / 65.0e-6) < 1.0
    for k in ("field_step", "push"):
        assert abs(r[k]["alg_ceiling_frac"] - r[k]["alg_GBps"] / 6300.0) < 1e-12
        assert r[k]["alg_ceiling_frac"] > r[k]["alg_frac"]
    assert "alg_ceiling_frac" not in bench.kernel_rates(64, avg, units, ab)["push"]


def test_per_source_flags_name_existing_sources_and_enter_the_kernel_hash(monkeypatch):
    """Every per-source flag of the build names a source that exists (a typo
    would drop the flag silently), and the profiles' kernel hash changes
    with the flags of the hot kernels' sources."""
    from paper_2307_07999_amd import build
    srcs = {os.path.basename(s) for s in build.sources()}
    assert set(build.PER_SOURCE) <= srcs, set(build.PER_SOURCE) - srcs
    h0 = bench.kernel_source_hash()
    monkeypatch.setitem(build.PER_SOURCE, "fields_f64.hip", ["-mllvm", "-amdgpu-sched-strategy=max-memory-clause"])
    assert bench.kernel_source_hash() != h0
