"""Host logic of the scan summary (Sec. 2, Figs. 1 and 2) on synthetic
statistics tables: the peak of the total rate, the anisotropy at delta tau =
0.3 fm and the late rates are read at the right rows, with delta tau counted
from each curve's own start (the formation time of a scan point, the start of
a correlator)."""
import math

import numpy as np

from paper_2307_07999_amd import glasma as G
from paper_2307_07999_amd import scan as S

DT = 0.0025


def _table(peak_k, min_k, n=400, seed=0):
    """Rows as gl_scan_statistics gives them: (tau_{k+3/2}, tau_{k+1}, <A>,
    err, <B>, err, ratio, err, rate_A, err, rate_B, err, total, err), with
    a total-rate maximum at row peak_k, a deeper longitudinal-rate dip before
    it (row 2) than the one after it (row min_k), and ratio = 10 tau."""
    r = np.random.default_rng(seed)
    k = np.arange(n)
    t = np.zeros((n, 14))
    t[:, 0] = (k + 1.5) * DT
    t[:, 1] = (k + 1.0) * DT
    t[:, 2::2] = r.uniform(1.0, 2.0, (n, 6))
    t[:, 3::2] = r.uniform(0.0, 0.1, (n, 6))
    t[:, 6] = 10.0 * t[:, 0]
    t[:, 12] = 1.0
    t[peak_k, 12] = 50.0
    t[2, 10] = -99.0
    t[min_k, 10] = -3.0
    return t


def test_summary_reads_peak_ratio_and_late_rates_from_each_start():
    pts = S.scan_points()
    res = {"stats": [_table(20 + k, 300 + k, seed=k) for k in range(len(pts))],
           "static": _table(30, 350, seed=90), "lightlike": _table(10, 200, seed=91),
           "static_start_fm": 0.05}
    summ = S.summary(res)
    assert set(summ) == {p[0] for p in pts} | {"static", "lightlike"}
    starts = [(label, res["stats"][k], 20 + k, 300 + k,
               tf if tf >= 0 else G.HBARC_GEV_FM / (2.0 * math.hypot(m, p0)))
              for k, (label, kind, m, p0, tf) in enumerate(pts)]
    starts += [("static", res["static"], 30, 350, 0.05), ("lightlike", res["lightlike"], 10, 200, 0.0)]
    for label, t, pk, mk, tau0 in starts:
        v = summ[label]
        assert v["peak"]["total"] == 50.0 and v["peak"]["err"] == t[pk, 13]
        assert v["peak"]["dtau_fm"] == t[pk, 1] - tau0
        i = int(np.argmin(np.abs(t[:, 0] - (tau0 + 0.3))))
        assert abs(t[i, 0] - (tau0 + 0.3)) <= DT / 2 + 1e-15
        assert v["ratio_at_0.3fm"] == [t[i, 6], t[i, 7]]
        late = v["late"]
        assert late["rate_B_min"] == [-3.0, t[mk, 11]]        # the dip before the peak is not late
        assert late["rate_B_min_dtau_fm"] == t[mk, 1] - tau0
        assert late["rate_A_end"] == [t[-1, 8], t[-1, 9]]
        assert late["rate_B_end"] == [t[-1, 10], t[-1, 11]]
        assert v["A_end"] == [t[-1, 2], t[-1, 3]] and v["B_end"] == [t[-1, 4], t[-1, 5]]


def test_static_quarks_start_with_the_beauty_quarks_at_rest():
    """The first scan point is the beauty quark with p_T0 = 0, whose
    formation step the static correlator takes as its start."""
    label, kind, m, p0, tf = S.scan_points()[0]
    assert kind == G.KIND_HEAVY_QUARK and m == S.BEAUTY_GEV and p0 == 0.0 and tf < 0


def test_run_scan_refuses_fewer_than_two_events():
    """The jackknife over events needs two; the check comes before any device work."""
    import pytest
    with pytest.raises(ValueError):
        S.run_scan(n_events=1)
