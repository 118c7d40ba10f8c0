"""Benchmark of the Glasma + colored-particle-in-cell hot path on one MI355X.

One "step" is one whole event of the 512^2 paper-scale workload: MV charges
drawn on the device (50 sheets per nucleus), Poisson solves, Wilson lines,
matching and pi0, 7 x 1e5 particles (charm and beauty at p_T0 in {0, 2, 5}
GeV, massless jets at 10 GeV, tau_form = 1/(2 m_T)), then the coupled leapfrog
to tau = 1 fm/c (409 field + particle steps after the initial half step) and
the broadening series.  Inputs are synthetic (seeded) and generated on the
device; nothing is read from the host inside the timed region.

Prints ONE JSON line (rank 0).  `value` is lattice site-updates per second of
the whole job; particle-steps per second is reported beside it.  `roofline`
is the dominant kernel (the field step) against the HBM peak and against
`stream_ceiling`, the copy rate the library's own streaming kernel reaches on
this device in the same process; `kernels` gives the field step and the push
each with its rate alone (site updates/s, particle steps/s), algorithmic and
counted GB/s as fractions of both, and their share of the chip's VALU issue
rate (the roofline of a kernel bound by its arithmetic), for the FP64 event
and its FP32 twin.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBARC = 0.1973269804
PEAK_HBM_GBS = 8000.0

# paper-scale workload
N, L_FM, SHEETS, M_IR, QS = 512, 10.0, 50, 0.2, 2.0
# g^2 mu whose MV Wilson lines have Q_s = 2 GeV (D(sqrt(2)/Q_s) = exp(-1/2)):
# gl_calibrate_g2mu at 512^2, L = 10 fm, 50 sheets, m_IR = 0.2 GeV, 4 seeds
# (Q_s / g^2 mu = 0.722); reproduced by the GPU tests
G2MU = 2.767
DTAU = 0.125
N_PER = 100000
SPECIES = ([(1.27, p0, 0) for p0 in (0.0, 2.0, 5.0)] + [(4.18, p0, 0) for p0 in (0.0, 2.0, 5.0)]
           + [(0.0, 10.0, 1)])
SEED = 2307079992
# kernel durations are sampled on every PROFILE_PERIOD-th launch of each
# kernel over the timed region (HIP events on the library's stream); the
# period is coprime with the 16-step particle sort cycle so that the samples
# cover every phase of it (the push is fastest right after a sort).  A
# sampled launch costs a few microseconds of timing events, so the period is
# long: every 7th launch cost 0.6 % of the event's wall time, every 17th
# about 0.25 %, and still gives about 25 samples per kernel and event.
PROFILE_PERIOD = 17


def coupled_steps(N, L, tau_max=1.0):
    a = L / N
    return int(math.ceil(tau_max / (DTAU * a) - 1e-9)) - 1


def alg_bytes(prec):
    ts = 8 if prec == 64 else 4
    return {
        # one pass: U (24: the first two rows of each link) E (16) phi (8)
        # pi (8) read once and written once per site, and the six
        # local-frame site fields (48) written
        "field_step": (2 * 56 + 48) * ts,
        # state read (cell 8 B, species 4 B, 14 reals), site fields 48 + phi 8
        # reals gathered, state written (cell 8 B, 14 reals); the momenta at
        # formation enter only through per-species sums taken once
        "push": 12 + 14 * ts + 56 * ts + 8 + 14 * ts,
    }


def kernel_rates(prec, avg_us, units, ab, ceiling=None):
    """Per dominant kernel: its rate alone (site updates/s of the field step,
    particle steps/s of the push, from the live HIP-event duration);
    algorithmic GB/s (algorithmic bytes over that duration) and counted GB/s
    (the HBM bytes of the counter runs over the same duration, None when those
    are stale), each as a fraction of the 8 TB/s peak and, when `ceiling`
    (GB/s of the library's own copy kernel, measured in the same process) is
    given, of that ceiling; and the fraction of the chip's VALU issue rate its
    instructions take (the SQ-counter count per launch over the same duration
    against VALU_ISSUE_PEAK, None when the counts are stale): the roofline of a
    kernel bound by its arithmetic rather than by HBM."""
    out = {}
    tname = "double" if prec == 64 else "float"
    rate_name = {"field_step": "site_updates_per_s", "push": "particle_steps_per_s"}
    for name in ("field_step", "push"):
        t = avg_us[name] * 1e-6
        alg = ab[name] * units[name] / t / 1e9
        tr = measured_traffic(name, prec)
        cnt = None if tr is None else (tr[0] + tr[1]) / t / 1e9
        valu = measured_valu("gl::k_%s<%s>" % (name, tname), prec)
        out[name] = {"avg_us": avg_us[name], rate_name[name]: units[name] / t,
                     "alg_GBps": alg, "alg_frac": alg / PEAK_HBM_GBS,
                     "counted_GBps": cnt, "counted_frac": None if cnt is None else cnt / PEAK_HBM_GBS,
                     "valu_issue_frac": None if valu is None else valu / t / VALU_ISSUE_PEAK}
        if ceiling:
            out[name]["alg_ceiling_frac"] = alg / ceiling
            out[name]["counted_ceiling_frac"] = None if cnt is None else cnt / ceiling
    return out


def run_event(g, torch, prec, n_per, steps, prof=False):
    ev = g.Event(N, L_FM, DTAU, precision=prec, reunit_every=16, max_steps=steps,
                 max_particles=n_per * len(SPECIES))
    return ev


def one_event(ev, g, n_per, steps):
    ev.init_glasma(G2MU, M_IR, SHEETS, SEED)
    for k, (m, p0, kind) in enumerate(SPECIES):
        ev.add_species(m, p0, kind, n_per, SEED + 17 * k)
    ev.run(steps)


# profile classes of the library's kernel timing (1 is unused: the site
# fields are fused into the field step); class 4 is the push that applies a
# sort, once per sort period
PROFILE_CLASSES = {0: "field_step", 2: "push", 4: "push_applying_sort"}


def timed_events(g, torch, prec, n_per, steps, k, warmup):
    """W untimed warm-up events, then K whole events timed together with
    their kernel durations from HIP events on the library's stream over the
    same region.  Returns (wall s, ms per profile class, launches per class,
    all finite)."""
    ev = run_event(g, torch, prec, n_per, steps)
    for _ in range(warmup):
        one_event(ev, g, n_per, steps)
        ev.close()
        ev = run_event(g, torch, prec, n_per, steps)
    ev.close()
    torch.cuda.synchronize()
    evs = [run_event(g, torch, prec, n_per, steps) for _ in range(k)]
    for e in evs:
        e.profile(True, period=PROFILE_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in evs:
        one_event(e, g, n_per, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [0.0] * 5
    cnt = [0] * 5
    for e in evs:
        m, c = e.profile_read()
        for j in range(5):
            ms[j] += m[j]
            cnt[j] += int(c[j])
    finite = True
    for e in evs:
        finite &= e.diagnostics()["nonfinite"] == 0
    obs = observables(evs[-1])
    # the timed events share every seed: their curves must agree bit for bit
    import numpy as np
    first = observables(evs[0])
    repeat = all(np.array_equal(a[k], b[k]) for a, b in zip(first, obs) for k in a)
    for e in evs:
        e.close()
    return wall, ms, cnt, bool(finite), obs, bool(repeat)


def observables(ev):
    """Per species of an event, the curves the paper plots (library rows):
    <dp_T^2> or <dp_y^2>, <dp_z^2>, and kappa_T, kappa_L (heavy quarks) or
    qhat_y, qhat_z (jets)."""
    out = []
    for s, (_, _, kind) in enumerate(SPECIES):
        b = ev.broadening(s)
        if kind == 0:
            k = ev.kappa(s)
            out.append({"dpT2": b[:, 1] + b[:, 2], "dpz2": b[:, 3], "rate_T": k[:, 2], "rate_L": k[:, 3]})
        else:
            q = ev.qhat(s)
            out.append({"dpy2": b[:, 2], "dpz2": b[:, 3], "rate_y": q[:, 1], "rate_z": q[:, 2]})
    return out


def observable_errors(got, want):
    """Largest over species of max |got - want| / max |want| per curve."""
    import numpy as np
    err = {}
    for g_, w_ in zip(got, want):
        for key in w_:
            a, b = np.asarray(g_[key]), np.asarray(w_[key])
            n = min(len(a), len(b))
            scale = np.abs(b[:n]).max() if n else 0.0
            e = float(np.abs(a[:n] - b[:n]).max() / scale) if n and scale > 0 else 0.0
            err[key] = max(err.get(key, 0.0), e)
    return err


def fp32_event(g, torch, n_per, steps, k, obs64, ceiling=None):
    """The FP32 twin of the headline event (FP32 links, fields and
    particles, FP64 sums; the same charges and particles): one warm-up event,
    then K timed events, with the per-kernel algorithmic and counted HBM rates
    and the error of its observables against the FP64 event's."""
    wall, ms, cnt, finite, obs, repeat = timed_events(g, torch, 32, n_per, steps, k, 1)
    n_part = n_per * len(SPECIES)
    avg_us = {PROFILE_CLASSES[j]: 1e3 * ms[j] / max(cnt[j], 1) for j in PROFILE_CLASSES}
    units = {"field_step": N * N, "push": n_part}
    return {"events": k, "ms_per_event": 1e3 * wall / k, "site_updates_per_s": N * N * steps * k / wall,
            "particle_steps_per_s": n_part * steps * k / wall, "kernel_avg_us": avg_us,
            "kernels": kernel_rates(32, avg_us, units, alg_bytes(32), ceiling), "finite": finite,
            "bitwise_repeatable": repeat,
            "observable_rel_err_vs_fp64": observable_errors(obs, obs64)}


def batch_bench(g, torch, steps, n_events=64, seed=20230718, cache=None, ceiling=None):
    """64 MV events with N uniform on {128, 256, 384, 512} at fixed a = 10/512 fm
    and log-uniform 1e4..1e6 particles each (charm and beauty at p_T0 in
    {0, 2, 5} GeV, jets at 10 GeV), FP32, stepped as one batch: flattened
    multi-event kernels, graph-replayed step loop, autotuned tiles."""
    import numpy as np
    rng = np.random.default_rng(seed)
    Ns = rng.choice([128, 256, 384, 512], size=n_events)
    parts = np.exp(rng.uniform(np.log(1e4), np.log(1e6), size=n_events)).astype(np.int64)
    a_fm = L_FM / N
    evs = []
    t0 = time.perf_counter()
    for e in range(n_events):
        ne = int(Ns[e])
        per = max(1, int(parts[e]) // len(SPECIES))
        ev = g.Event(ne, ne * a_fm, DTAU, precision=32, reunit_every=16, max_steps=steps,
                     max_particles=per * len(SPECIES))
        ev.init_glasma(G2MU, M_IR, SHEETS, SEED + 1000 * e)
        for k, (m, p0, kind) in enumerate(SPECIES):
            ev.add_species(m, p0, kind, per, SEED + 1000 * e + 17 * k)
        evs.append(ev)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    b = g.Batch(evs)
    b.autotune(cache)
    cfg = b.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(steps)
    b.stream.synchronize()
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    sites = int(sum(int(n) * int(n) for n in Ns))
    npart = int(sum(len(SPECIES) * max(1, int(p) // len(SPECIES)) for p in parts))
    ab = alg_bytes(32)
    step_bytes = sites * ab["field_step"] + npart * ab["push"]
    finite = all(e.diagnostics()["nonfinite"] == 0 for e in evs)
    counted = {}
    for kern, alg in (("batch_field", sites * ab["field_step"]), ("batch_push", npart * ab["push"])):
        tr = measured_traffic(kern, 32)
        counted[kern] = {"alg_bytes_per_launch": alg,
                         "counted_bytes_per_launch": None if tr is None else tr[0] + tr[1]}
    b.close()
    for e in evs:
        e.close()
    return {"events": n_events, "sites": sites, "particles": npart, "coupled_steps": steps,
            "init_s": t_init, "run_s": t_run,
            "site_updates_per_s": sites * steps / t_run,
            "particle_steps_per_s": npart * steps / t_run,
            "alg_GBps": step_bytes * steps / t_run / 1e9,
            "frac_hbm": step_bytes * steps / t_run / 1e9 / PEAK_HBM_GBS,
            "frac_ceiling": step_bytes * steps / t_run / 1e9 / ceiling if ceiling else None,
            "tile": cfg["tile"], "grid_mult": cfg["grid_mult"], "graph_steps": cfg["graph_steps"],
            "hbm_traffic": counted, "finite": finite}


def scan_bench(n_events=16, n_per=N_PER, precision=64):
    """The paper's scans (Sec. 2, Figs. 1 and 2) at the 512^2 scale: beauty
    quarks at p_T0 in {0, 2, 5, 10} GeV and jets at p_x in {1, 2, 5, 10} GeV for
    m in {1.27, 4.18} GeV, n_per particles per point, with the static and
    lightlike correlators, over n_events MV events; jackknife errors over the
    events.  Reports the wall time and, per point, the peak of the total
    coefficient (kappa_T + kappa_L or qhat_y + qhat_z) with its error and
    time after formation, the anisotropy 0.3 fm after formation, the lowest
    longitudinal rate after the peak (kappa_L or qhat_z, with its time) and
    the transverse rate at tau_max."""
    from paper_2307_07999_amd import scan
    res = scan.run_scan(n_events=n_events, N=N, L_fm=L_FM, sheets=SHEETS, g2mu=G2MU, m_ir=M_IR, n_per=n_per,
                        precision=precision)
    summ = scan.summary(res)

    def short(v):
        pk = v["peak"]
        return {"peak_total_GeV2_per_fm": [round(pk["total"], 3), round(pk["err"], 3)],
                "peak_dtau_fm": round(pk["dtau_fm"], 4),
                "ratio_B_over_A_at_0.3fm": None if v["ratio_at_0.3fm"] is None else
                [round(x, 4) for x in v["ratio_at_0.3fm"]],
                "min_rate_B_after_peak_GeV2_per_fm": [round(x, 3) for x in v["late"]["rate_B_min"]],
                "min_rate_B_dtau_fm": round(v["late"]["rate_B_min_dtau_fm"], 4),
                "rate_A_end_GeV2_per_fm": [round(x, 3) for x in v["late"]["rate_A_end"]]}
    return {"events": n_events, "particles_per_point": n_per, "points": len(res["points"]),
            "precision": precision, "coupled_steps": res["coupled_steps"], "wall_s": res["wall_s"],
            "s_per_event": res["s_per_event"], "particle_steps_per_s": res["particle_steps_per_s"],
            "results": {k: short(v) for k, v in summ.items()},
            "paper_context": {"kappa_total_peak_GeV2_per_fm": scan.PAPER_KAPPA_PEAK,
                              "kappa_peak_dtau_fm": scan.PAPER_KAPPA_PEAK_DTAU,
                              "qhat_total_peak_GeV2_per_fm": scan.PAPER_QHAT_PEAK,
                              "qhat_peak_tau_fm": scan.PAPER_QHAT_PEAK_TAU}}


def surrogate_bench(mode):
    """Surrogate vs solver: the protocol of paper_2307_07999_amd.surrogate
    (solver-generated training data, BF16 network trained on the GPU,
    evaluated against held-out 512^2 solver runs).  'quick' is a reduced protocol that
    keeps the default run within a few minutes; 'full' is the complete one."""
    from paper_2307_07999_amd import surrogate
    if mode == "full":
        rep = surrogate.protocol(log=lambda *a: None)
    else:
        rep = surrogate.protocol(n_train_coarse=400, n_train_fine=128, n_heldout=16, n_avg=2,
                                 epochs=40, fine_epochs=80, log=lambda *a: None)
    rep["mode"] = mode
    return rep


def oracle_sample(budget_s):
    """The FP64 oracle on a bounded sample of the workload, single thread:
    coupled steps on the full 512^2 lattice from a seeded state (site fields
    included) and the particle push on a 1e5 sample scaled to the 7e5
    ensemble, repeated until the field work alone has taken budget_s."""
    from oracle import oracle as orc
    from tests import seeded_inputs as si
    a_fm = L_FM / N
    a_gev = a_fm / HBARC
    U, E, phi, pi = si.random_state(5, N, link_kind="near", eps=0.3)
    s = orc.State(N)
    s.U, s.E, s.phi, s.pi, s.n = U, E, phi, pi, 40
    P = orc.particles_init(N, SEED, 0, 0, 2.0 * a_gev, N_PER)
    t_field = t_part = 0.0
    steps = 0
    while steps < 2 or t_field < budget_s:
        t0 = time.perf_counter()
        U0, phi0, n = s.U.copy(), s.phi.copy(), s.n
        F = orc.field_step(s, DTAU, want_F=True)
        t_field += time.perf_counter() - t0
        t0 = time.perf_counter()
        orc.particle_step(N, n, DTAU, U0, phi0, F, P, [1.27 * a_gev], [1])
        t_part += (time.perf_counter() - t0) * len(SPECIES)   # scale 1e5 -> 7e5
        steps += 1
    return {"steps": steps, "t_field": t_field, "t_part": t_part}


def cpu_model():
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s=12.0, max_procs=16):
    """The oracle timed on the host's cores: P = min(cores available to this
    process, max_procs) independent single-threaded oracle processes, each
    pinned to its own core and running the same bounded sample
    (oracle_sample); the aggregate rate is the work of all of them over the
    wall time of the slowest.  max_procs is the host-core share of one GPU."""
    import subprocess
    cpus = sorted(os.sched_getaffinity(0))
    P = max(1, min(len(cpus), max_procs))
    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "print(json.dumps(bench.oracle_sample(%r)))" % (ROOT, budget_s))
    procs = []
    t0 = time.perf_counter()
    for k in range(P):
        cpu = cpus[k]
        procs.append(subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, text=True,
                                      env=dict(os.environ, OMP_NUM_THREADS="1"),
                                      preexec_fn=lambda c=cpu: os.sched_setaffinity(0, {c})))
    results = []
    for pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError("oracle process failed with status %d" % pr.returncode)
        results.append(json.loads(out.strip().splitlines()[-1]))
    wall = time.perf_counter() - t0
    # per process: its own rate; aggregate: all sites updated over the wall time
    per = [(N * N * r["steps"], (r["t_field"] + r["t_part"])) for r in results]
    single = per[0][0] / per[0][1]
    total_updates = sum(u for u, _ in per)
    busiest = max(t for _, t in per)
    r0 = results[0]
    return {"value": total_updates / busiest, "unit": "site-updates/s", "cores": P, "kind": "oracle",
            "sample": "per process: %d coupled steps on the 512^2 lattice (seeded state) with site fields, and the "
                      "particle push timed on 1e5 particles scaled x7 to the 7e5 ensemble (init excluded); %d "
                      "independent single-threaded processes, one pinned per core; aggregate = site updates of all "
                      "processes over the longest process time" % (r0["steps"], P),
            "single_core_site_updates_per_s": single,
            "particle_steps_per_s": N_PER * len(SPECIES) * sum(r["steps"] for r in results) / busiest,
            "wall_s": wall, "nproc": os.cpu_count(), "cpus_available": len(cpus), "cpu_model": cpu_model()}


# HBM traffic of the dominant kernels, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs (bench.py --traffic), valid for the kernel sources whose
# hash is recorded beside them; stale figures are reported as null.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "glasma512_hbm_traffic.md")
KERNEL_SOURCES = ["su3.hpp", "internal.hpp", "fields_dev.hpp", "fields.hip", "fields_f64.hip", "push_dev.hpp",
                  "particles.hip"]


def kernel_name(raw):
    """A profiler's kernel name without its return type, anonymous-namespace
    qualifier and parameter list."""
    n = raw.replace("(anonymous namespace)::", "")
    if n.startswith("void "):
        n = n[5:]
    return n.split("(")[0].strip()


def kernel_source_hash():
    """Hash of the hot kernels' sources and of the compiler flags they are
    built with (build.py)."""
    import hashlib
    from paper_2307_07999_amd import build as b
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2307_07999_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(repr((b.COMMON[:-2], sorted((k, v) for k, v in b.PER_SOURCE.items() if k in KERNEL_SOURCES))).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, prec):
    """Bytes per launch (fetch, write) recorded for this kernel and precision,
    or None when missing or taken on other kernel sources."""
    import re
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    src = None
    rows = {}
    for ln in lines:
        if ln.startswith("source hash:"):
            m = re.search(r"`([0-9a-f]+)`", ln)
            src = m.group(1) if m else None
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        if len(cells) >= 4 and cells[0] in ("field_step", "push", "batch_field", "batch_push") and \
                cells[1] in ("32", "64"):
            rows[(cells[0], int(cells[1]))] = (float(cells[2]), float(cells[3]))
    if src != kernel_source_hash():
        return None
    return rows.get((kernel, prec))


SQ_FILES = {p: os.path.join(ROOT, "profiles", "glasma512_fp%d_sq_counters.md" % p) for p in (64, 32)}
# wave64 VALU instructions the chip can issue per second: each of the 1024
# SIMDs (256 CUs x 4) takes one every 4 cycles (64 lanes over 16-wide ALUs,
# FP32 without packing like FP64), at the 2.4 GHz peak clock
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4.0
SQ_KERNELS = ("gl::k_field_step<", "gl::k_push<", "gl::k_push_permuted<", "gl::k_batch_field_flat<",
              "gl::k_batch_push_flat<")


def sq_table(prec, pmc_dir):
    """Rows 'kernel | launches | counter means per launch ... | VALU per wave'
    of the hot-path kernels from one rocprofv3 --pmc run of SQ counters, and
    the kernel-source hash they belong to."""
    import csv
    import glob
    acc = {}
    for fn in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(fn)):
            name = kernel_name(r["Kernel_Name"])
            if not name.startswith(SQ_KERNELS):
                continue
            a = acc.setdefault(name, {}).setdefault(r["Counter_Name"], [0.0, 0])
            a[0] += float(r["Counter_Value"])
            a[1] += 1
    counters = sorted({c for v in acc.values() for c in v})
    print("| kernel | launches | " + " | ".join(counters) + " | VALU per wave |")
    print("|---" * (len(counters) + 3) + "|")
    for name in sorted(acc, key=lambda k: -acc[k].get("SQ_INSTS_VALU", [0, 1])[0] / acc[k].get("SQ_INSTS_VALU", [0, 1])[1]):
        m = {c: v[0] / v[1] for c, v in acc[name].items()}
        waves = m.get("SQ_WAVES")
        vpw = "%.0f" % (m["SQ_INSTS_VALU"] / waves) if waves and "SQ_INSTS_VALU" in m else "-"
        launches = max(v[1] for v in acc[name].values())
        print("| %s | %d | %s | %s |" % (name, launches, " | ".join("%.0f" % m.get(c, float("nan")) for c in counters), vpw))
    print("source hash: `%s`" % kernel_source_hash())


def measured_valu(kernel, prec):
    """SQ_INSTS_VALU per launch of the kernel whose name starts with kernel
    (e.g. "gl::k_field_step<double>"), from the committed SQ-counter summary
    of this precision, or None when missing or taken on other kernel sources."""
    import re
    try:
        lines = open(SQ_FILES[prec]).read().splitlines()
    except (OSError, KeyError):
        return None
    src, col, val = None, None, None
    for ln in lines:
        if ln.startswith("source hash:"):
            m = re.search(r"`([0-9a-f]+)`", ln)
            src = m.group(1) if m else None
        cells = [c.strip() for c in ln.strip().strip("|").split("|")]
        if cells and cells[0] == "kernel" and "SQ_INSTS_VALU" in cells:
            col = cells.index("SQ_INSTS_VALU")
        elif col is not None and cells and cells[0].startswith(kernel) and val is None:
            try:
                val = float(cells[col])
            except (ValueError, IndexError):
                val = None
    if src != kernel_source_hash():
        return None
    return val


def traffic_table(prec, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """Rows 'kernel | precision | fetch bytes | write bytes' per launch from
    two counter runs, each scaled by what the counter reads for the plain
    1 GiB copy (bench.py --copy-calib 1024)."""
    import csv
    import glob

    def counts(d, counter):
        n = {}
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(fn)):
                if r["Counter_Name"] == counter:
                    name = kernel_name(r["Kernel_Name"])
                    n[name] = n.get(name, 0) + 1
        return n

    def means(d, counter):
        acc = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                name = kernel_name(r["Kernel_Name"])
                a = acc.setdefault(name, [0.0, 0])
                a[0] += float(r["Counter_Value"])
                a[1] += 1
        return {k: v[0] / v[1] for k, v in acc.items()}

    copy_bytes = 1024 * (1 << 20)
    cf = means(copy_fetch_dir, "FETCH_SIZE")
    cw = means(copy_write_dir, "WRITE_SIZE")
    kf = copy_bytes / (1024.0 * max(v for k, v in cf.items() if "copyBuffer" in k))
    kw = copy_bytes / (1024.0 * max(v for k, v in cw.items() if "copyBuffer" in k))
    f = means(fetch_dir, "FETCH_SIZE")
    w = means(write_dir, "WRITE_SIZE")
    tname = "double" if prec == 64 else "float"
    print("fetch factor %.4f, write factor %.4f (bytes per KiB counted, from the copy)" % (kf, kw))
    kerns = [("gl::k_field_step<%s>" % tname, "field_step"), ("gl::k_push<%s>" % tname, "push")]
    # the batched kernels of the 64-event FP32 workload, when the run had them
    # (the field kernel of the tile shape the autotuner picked: most launches)
    bf = [k for k in f if k.startswith("gl::k_batch_field_flat<%s" % tname)]
    if bf:
        kerns.append((max(bf, key=lambda k: counts(fetch_dir, "FETCH_SIZE").get(k, 0)), "batch_field"))
    # the batch's plain push (the one that applies a sort's order runs once per period)
    if "gl::k_batch_push_flat<%s, false>" % tname in f:
        kerns.append(("gl::k_batch_push_flat<%s, false>" % tname, "batch_push"))
    for kern, short in kerns:
        print("| %s | %d | %.0f | %.0f |" % (short, prec, f[kern] * 1024 * kf, w[kern] * 1024 * kw))
    print("source hash: `%s`" % kernel_source_hash())


def copy_calibration(mib):
    """A plain device-to-device copy of a known size (read mib MiB, write mib MiB),
    run three times: the reference for scaling the FETCH_SIZE / WRITE_SIZE
    hardware counters to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4,
                      "launches": 3}))


STREAM_KINDS = ("copy", "read", "write")


def stream_ceiling(mib=1024, reps=10, kinds=STREAM_KINDS):
    """The bandwidth the library's own streaming kernels reach (gl_stream_probe):
    a copy, a read and a write of mib MiB in 16-byte accesses, over its access
    patterns and grid sizes; GB/s counts the bytes read plus written.  The best
    of each kind is the ceiling a kernel of this library can be held against."""
    import torch
    import paper_2307_07999_amd as g
    g.lib()
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream
    torch.cuda.synchronize()
    rows, best = [], {}
    for kind, name in enumerate(STREAM_KINDS):
        if name not in kinds:
            continue
        moved = nbytes * (2 if kind == 0 else 1)
        for variant in range(6):
            for blocks in (2048, 8192, 32768):
                ms = g.glasma.stream_probe(kind, variant, blocks, src.data_ptr(), dst.data_ptr(), nbytes,
                                           nbytes, reps, stream)
                gbs = moved / (ms * 1e-3) / 1e9
                rows.append({"kind": name, "variant": variant, "blocks": blocks, "ms": ms, "GBps": gbs})
                if gbs > best.get(name, {}).get("GBps", 0.0):
                    best[name] = {"GBps": gbs, "variant": variant, "blocks": blocks}
    del src, dst
    torch.cuda.empty_cache()
    return {"MiB": mib, "reps": reps, "best": best, "all": rows}


def summarize(path, command):
    """Markdown summary of a rocprofv3 output directory: per-kernel durations
    (kernel_stats.csv) and mean per-dispatch counter values
    (counter_collection.csv), whichever are present."""
    import csv
    import glob
    lines = ["Command:", "", "```", command, "```", ""]
    for f in sorted(glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True)):
        lines += ["| kernel | calls | avg µs | total ms | % |", "|---|---|---|---|---|"]
        for r in csv.DictReader(open(f)):
            name = kernel_name(r["Name"])
            lines.append("| %s | %s | %.2f | %.2f | %.1f |" % (
                name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6,
                float(r["Percentage"])))
        lines.append("")
    for f in sorted(glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)):
        acc = {}
        for r in csv.DictReader(open(f)):
            name = kernel_name(r["Kernel_Name"])
            key = (name, r["Counter_Name"])
            a = acc.setdefault(key, [0.0, 0, r.get("VGPR_Count", ""), r.get("Accum_VGPR_Count", "")])
            a[0] += float(r["Counter_Value"])
            a[1] += 1
        lines += ["| kernel | counter | dispatches | mean per dispatch | VGPR | AGPR |",
                  "|---|---|---|---|---|---|"]
        for (name, cn), (tot, cnt, vg, ag) in sorted(acc.items(), key=lambda kv: -kv[1][0]):
            lines.append("| %s | %s | %d | %.1f | %s | %s |" % (name, cn, cnt, tot / cnt, vg, ag))
        lines.append("")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", type=int, default=64, choices=(64, 32))
    ap.add_argument("--particles-per-species", type=int, default=N_PER)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-event batched FP32 workload")
    ap.add_argument("--tune-cache", default=None, help="autotuner JSON cache for the batch")
    ap.add_argument("--no-fp32-event", action="store_true",
                    help="skip the FP32 twin of the headline event (reported beside the FP64 line)")
    ap.add_argument("--no-scan", action="store_true",
                    help="skip the paper's scans (16 events of 12 scan points at 512^2)")
    ap.add_argument("--surrogate", default="full", choices=("quick", "full", "off"),
                    help="surrogate-vs-solver section: reduced protocol, full protocol or none")
    ap.add_argument("--ceiling", action="store_true",
                    help="only measure the streaming ceiling (copy/read/write kernels of the library) and exit")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--summarize", nargs=2, metavar=("DIR", "COMMAND"),
                    help="print a markdown summary of a rocprofv3 output directory and exit")
    ap.add_argument("--traffic", nargs=5, metavar=("PREC", "FETCH_DIR", "WRITE_DIR", "COPY_FETCH", "COPY_WRITE"),
                    help="print the HBM traffic rows of the dominant kernels from counter runs and exit")
    ap.add_argument("--sq-table", nargs=2, metavar=("PREC", "PMC_DIR"),
                    help="print the SQ-counter rows of the hot-path kernels from a counter run and exit")
    args = ap.parse_args()
    if args.summarize:
        summarize(*args.summarize)
        return
    if args.traffic:
        traffic_table(int(args.traffic[0]), *args.traffic[1:])
        return
    if args.sq_table:
        sq_table(int(args.sq_table[0]), args.sq_table[1])
        return
    if args.copy_calib:
        copy_calibration(args.copy_calib)
        return
    if args.ceiling:
        print(json.dumps(stream_ceiling()))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported "
              "(independent events would shard across GPUs without exchange)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2307_07999_amd as g
    g.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    steps = coupled_steps(N, L_FM)
    n_per = args.particles_per_species
    wall, ms, cnt, kappa_ok, obs, repeat = timed_events(g, torch, args.precision, n_per, steps, args.steps,
                                                        args.warmup)

    # the streaming ceiling of this device, from the library's copy kernel
    ceil = stream_ceiling(reps=5, kinds=("copy",))["best"]["copy"]
    ceiling = ceil["GBps"]

    n_part = n_per * len(SPECIES)
    site_updates = N * N * steps * args.steps
    particle_steps = n_part * steps * args.steps
    ab = alg_bytes(args.precision)
    avg_us = {PROFILE_CLASSES[k]: 1e3 * ms[k] / max(cnt[k], 1) for k in PROFILE_CLASSES}
    units = {"field_step": N * N, "push": n_part}
    dom = max((0, 2), key=lambda k: ms[k])
    dname = PROFILE_CLASSES[dom]
    achieved = ab[dname] * units[dname] / (avg_us[dname] * 1e-6) / 1e9
    tr = measured_traffic(dname, args.precision)
    traffic = None if tr is None else (tr[0] + tr[1]) / (avg_us[dname] * 1e-6) / 1e9
    out = {
        "metric": "particle-steps/s + lattice site-updates/s (SU(3), 512^2, 1 GPU); surrogate vs solver",
        "value": site_updates / wall,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f32",
        "data": "synthetic",
        "config": {"workload": "glasma+cpic event: 512^2, L=10 fm, 50 MV sheets/nucleus, "
                               "g2mu=%.3f GeV, m_IR=0.2 GeV, dtau=a/8 to 1 fm (%d coupled steps), "
                               "7x%d particles" % (G2MU, steps, n_per),
                   "N": N, "coupled_steps": steps, "particles": n_part,
                   "precision": args.precision},
        "particle_steps_per_s": particle_steps / wall,
        "kernel_avg_us": avg_us,
        "finite": bool(kappa_ok),
        "bitwise_repeatable": repeat,
        "kernels": kernel_rates(args.precision, avg_us, units, ab, ceiling),
        "stream_ceiling": {"copy_GBps": ceiling, "variant": ceil["variant"], "blocks": ceil["blocks"]},
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "ceiling": ceiling, "ceiling_frac": achieved / ceiling,
                     "traffic_bytes_per_launch": None if tr is None else tr[0] + tr[1],
                     "alg_bytes_per_unit": ab[dname], "units_per_launch": units[dname]},
    }
    if args.precision == 64 and not args.no_fp32_event:
        out["fp32_event"] = fp32_event(g, torch, n_per, steps, args.steps, obs, ceiling)
    if not args.no_batch:
        out["batch_fp32"] = batch_bench(g, torch, steps, cache=args.tune_cache, ceiling=ceiling)
    if not args.no_scan:
        out["scan"] = scan_bench()
    if args.surrogate != "off":
        out["surrogate"] = surrogate_bench(args.surrogate)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
