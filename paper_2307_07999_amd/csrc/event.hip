// event.hip -- runtime behind the C-ABI of include/glasma.h: one event holds
// a caller-owned workspace carved into ping-pong field buffers, the site-field
// records, the padded particle arrays, the FP64 broadening series and the
// initial-condition scratch, and orders every launch on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/glasma.h"
#include "internal.hpp"
#include "su3.hpp"

using namespace gl;

namespace {

thread_local std::string g_err;
constexpr double kHbarC = 0.1973269804;   // GeV fm

gl_status fail(gl_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(GL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// The push writes per-workgroup partial rows; their fixed-order reduction
// into the series is deferred and done for up to kReduceSlots steps in one
// launch (the series is only read between runs).
constexpr int kReduceSlots = 16;
inline size_t partial_slot_stride(int64_t slots) {
    return (size_t)std::max<int64_t>(1, slots / kPushBlock) * kMaxSpecies * 4;
}

struct Layout {
    size_t field[2], F, part[2], id[2], sort_keys[2], sort_vals[2], sort_counts, sort_totals, partials,
        series, p0sum, diag, VA, VB, planes, fft_tab, U0, pi0, status, stat, stat_part, stat_series, ll, ll_part,
        ll_series, total;
    int64_t slots;         // particle capacity in slots (padding included)
    size_t n_diag_blocks;  // workgroups of the diagnostics kernel
};

bool valid_N_for_fft(int N) {
    int m = N;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1;
}

// largest particle capacity whose record planes stay below 2^31 bytes
// (the buffer range of the device accesses), in whole push blocks
int64_t max_particles_for(int precision) {
    const int64_t rec = (int64_t)part_rec(precision == 64 ? 8 : 4) * (precision == 64 ? 8 : 4);
    return ((((int64_t)1 << 31) - 256) / rec) / kPushBlock * kPushBlock;
}

gl_status make_layout(const gl_lattice_desc *d, Layout &L) {
    if (!d) return fail(GL_EINVAL, "null lattice description");
    if (d->N < 2 || d->N > 1024) return fail(GL_EINVAL, "N must be in [2, 1024]");
    if (!(d->L_fm > 0) || !(d->dtau_over_a > 0) || d->dtau_over_a > 0.5)
        return fail(GL_EINVAL, "L_fm must be > 0 and 0 < dtau_over_a <= 0.5");
    if (d->precision != 64 && d->precision != 32) return fail(GL_EINVAL, "precision must be 64 or 32");
    if (d->max_steps < 0 || d->max_particles < 0 || d->reunit_every < 0)
        return fail(GL_EINVAL, "negative capacity");
    const size_t n2 = (size_t)d->N * d->N, ts = d->precision == 64 ? 8 : 4;
    // particle arrays are addressed with 32-bit byte offsets on the device;
    // the widest is the particle record, whose chunk planes span all slots
    if (d->max_particles > max_particles_for(d->precision))
        return fail(GL_EINVAL, "max_particles above the 32-bit particle-record range (" +
                                   std::to_string(max_particles_for(d->precision)) + " at this precision)");
    L.slots = (d->max_particles + kPushBlock - 1) / kPushBlock * kPushBlock;
    if (d->max_particles == 0) L.slots = 0;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    for (int b = 0; b < 2; b++) L.field[b] = take(kStateVals * n2 * ts);
    L.F = take((size_t)kSiteRec * n2 * ts);
    for (int b = 0; b < 2; b++) L.part[b] = take((size_t)L.slots * ((part_rec(ts) + 3) * ts + 12));
    for (int b = 0; b < 2; b++) L.id[b] = take((size_t)L.slots * sizeof(int32_t));
    for (int b = 0; b < 2; b++) L.sort_keys[b] = take((size_t)L.slots * sizeof(uint32_t));
    for (int b = 0; b < 2; b++) L.sort_vals[b] = take((size_t)L.slots * sizeof(int32_t));
    L.sort_counts = take((size_t)256 * std::max<int64_t>(1, sort_tiles(L.slots)) * sizeof(uint32_t));
    L.sort_totals = take(256 * sizeof(uint32_t));
    // partial rows of up to kReduceSlots pushes, reduced into the series in one launch
    L.partials = take(kReduceSlots * partial_slot_stride(L.slots) * sizeof(double));
    L.series = take(std::max(1, d->max_steps) * (size_t)kMaxSpecies * 4 * sizeof(double));
    L.p0sum = take((size_t)kMaxSpecies * 4 * sizeof(double));
    L.n_diag_blocks = (size_t)((d->N + 31) / 32) * ((d->N + 7) / 8);
    size_t cas_blocks = (size_t)std::max<int64_t>(1, (L.slots + 255) / 256);
    L.diag = take(std::max(L.n_diag_blocks * 8, 2 * cas_blocks) * sizeof(double));
    L.VA = take(18 * n2 * sizeof(double));
    L.VB = take(18 * n2 * sizeof(double));
    L.planes = take((size_t)kSheetChunk * 4 * n2 * sizeof(double2));
    L.fft_tab = take(kFftTableBytes);
    L.U0 = take(36 * n2 * sizeof(double));
    L.pi0 = take(8 * n2 * sizeof(double));
    L.status = take(256);
    // static-quark accumulators I [24][n2], their per-workgroup partials and series
    const bool stat = d->static_correlator != 0;
    L.stat = take(stat ? 24 * n2 * sizeof(double) : 0);
    L.stat_part = take(stat ? (n2 + 255) / 256 * 4 * sizeof(double) : 0);
    L.stat_series = take(stat ? std::max(1, d->max_steps) * (size_t)kMaxSpecies * 4 * sizeof(double) : 0);
    // lightlike-jet transports W [18][n2] and accumulators I [24][n2], partials and series
    const bool ll = d->lightlike_correlator != 0;
    L.ll = take(ll ? 42 * n2 * sizeof(double) : 0);
    L.ll_part = take(ll ? (n2 + 255) / 256 * 4 * sizeof(double) : 0);
    L.ll_series = take(ll ? std::max(1, d->max_steps) * (size_t)kMaxSpecies * 4 * sizeof(double) : 0);
    L.total = off;
    return GL_OK;
}

struct SpeciesInfo {
    gl_species_desc desc;
    int64_t n;
    int32_t nform;
    double mass_lat, p0_lat, tau_form_fm;
};

}  // namespace

struct gl_event {
    gl_lattice_desc desc;
    Layout L;
    int N;
    size_t n2;
    double a_fm, a_gev, dtau;   // dtau in lattice units
    hipStream_t stream;
    char *ws;
    int cur = 0;
    int64_t n = 0;
    bool ready = false, push_due = false;
    int64_t rows = 0;           // series rows written
    int64_t pend_row0 = 0;      // first series row of the pending partial rows
    int pend = 0;               // pushes whose partial rows are not reduced yet
    int64_t slots_used = 0;
    std::vector<SpeciesInfo> species;
    int pbuf = 0;               // which particle buffer is current
    // a sort whose permutation (in the sort scratch) the next push applies:
    // within a run the particles move to their sorted slots while being
    // pushed; every call returns with none pending
    bool perm_pending = false;
    // the particle set changed since the last sort and formation sums: both
    // are taken once, before the next push (settle_particles), so that
    // adding several species sorts once
    bool set_changed = false;
    int32_t sort_every = 16;    // re-sort particles by cell every this many pushes (0: never)
    int64_t since_sort = 0;
    bool stat_on = false;       // static-quark accumulation running
    int64_t stat_n0 = 0;        // first accumulated field step
    int64_t stat_rows = 0;      // static series rows written
    bool ll_on = false;         // lightlike-jet accumulation running
    int64_t ll_n0 = 0;          // first accumulated field step
    int64_t ll_rows = 0;
    gl_batch *owner = nullptr;  // the batch that holds the event (its mutators refuse)
    int32_t match_max_iter = 100;
    double match_tol = 1e-13;
    int32_t check_every = 0;    // finite-value checks inside gl_run every this many steps (0: off)
    int32_t graph_steps = 0;    // gl_run replays blocks of this many steps from a captured graph (0: off)
    // two executable graphs used in turn, each with the event recorded after
    // its last launch: one is updated or replaced only once that launch is
    // done, while the other's may still run
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipEvent_t gdone[2] = {nullptr, nullptr};
    int gslot = 0;
    int64_t graph_launches = 0, graph_instantiations = 0;

    // kernel timing: pairs of events per launch, grouped by kernel class
    int32_t prof = 0;                       // time every prof-th launch of each class (0: off)
    int64_t prof_count[GL_PROF_KERNELS] = {};
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> prof_marks;   // (class, index of start event)

    bool fp64() const { return desc.precision == 64; }
    template <typename T>
    FieldPtrs<T> fields(int b) const {
        T *base = (T *)(ws + L.field[b]);
        return FieldPtrs<T>{base, base + 2 * kLinkVals * n2, base + (2 * kLinkVals + 16) * n2,
                            base + (2 * kLinkVals + 24) * n2};
    }
    template <typename T>
    PartPtrs<T> parts(int buf = -1) const {
        PartPtrs<T> p;
        int64_t c = L.slots;
        char *b = ws + L.part[buf < 0 ? pbuf : buf];
        p.cx = (int32_t *)b;
        p.cy = p.cx + c;
        p.species = p.cy + c;
        T *t = (T *)(b + 12 * c);   // 16-byte aligned: c is a multiple of kPushBlock
        p.st = t;
        p.px0 = t + kPartRec<T> * c;
        p.py0 = p.px0 + c;
        p.pz0 = p.py0 + c;
        p.cap = c;
        return p;
    }
    template <typename T>
    SpeciesTab<T> tab() const {
        SpeciesTab<T> t;
        for (int s = 0; s < kMaxSpecies; s++) {
            t.mass[s] = s < (int)species.size() ? (T)species[s].mass_lat : T(0);
            t.nform[s] = s < (int)species.size() ? species[s].nform : 0x7fffffff;
        }
        return t;
    }
    int32_t *ids(int buf = -1) const { return (int32_t *)(ws + L.id[buf < 0 ? pbuf : buf]); }
    SortScratch scratch() const {
        SortScratch sc;
        for (int b = 0; b < 2; b++) {
            sc.keys[b] = (uint32_t *)(ws + L.sort_keys[b]);
            sc.vals[b] = (int32_t *)(ws + L.sort_vals[b]);
        }
        sc.counts = (uint32_t *)(ws + L.sort_counts);
        sc.totals = (uint32_t *)(ws + L.sort_totals);
        return sc;
    }
    double *series() const { return (double *)(ws + L.series); }
    double *stat_series() const { return (double *)(ws + L.stat_series); }
    double *ll_series() const { return (double *)(ws + L.ll_series); }
    double *partials(int slot = 0) const {
        return (double *)(ws + L.partials) + (size_t)slot * partial_slot_stride(L.slots);
    }
    double *p0sum() const { return (double *)(ws + L.p0sum); }
};

namespace {

gl_status check_ev(gl_event *ev) {
    if (!ev) return fail(GL_EINVAL, "null event");
    return GL_OK;
}

// the calls that step, initialise or change an event refuse while a batch holds it
gl_status check_free(gl_event *ev) {
    if (!ev) return fail(GL_EINVAL, "null event");
    if (ev->owner) return fail(GL_ESTATE, "the event is held by a batch (destroy the batch first)");
    return GL_OK;
}

// start/stop marks around one launch of kernel class k (no-ops when disabled
// and for the launches between samples)
constexpr size_t kNoMark = ~(size_t)0;
// a pair of pooled events for a sampled launch of class k (kNoMark: this
// launch is not sampled)
gl_status prof_take(gl_event *ev, int k, size_t *idx) {
    *idx = kNoMark;
    if (ev->prof <= 0 || (ev->prof_count[k]++ % ev->prof) != 0) return GL_OK;
    while (ev->ev_pool.size() < ev->ev_used + 2) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        ev->ev_pool.push_back(e);
    }
    *idx = ev->ev_used;
    ev->ev_used += 2;
    ev->prof_marks.push_back({k, *idx});
    return GL_OK;
}

// events recorded on the stream around a launch (classes of more than one
// kernel or of launchers without a KernelTimer)
gl_status prof_begin(gl_event *ev, int k, size_t *idx) {
    gl_status s = prof_take(ev, k, idx);
    if (s || *idx == kNoMark) return s;
    HIP_TRY(hipEventRecord(ev->ev_pool[*idx], ev->stream));
    return GL_OK;
}

// events the launch of a single kernel records at its start and end
gl_status prof_timer(gl_event *ev, int k, KernelTimer *kt) {
    *kt = KernelTimer{};
    size_t idx = kNoMark;
    gl_status s = prof_take(ev, k, &idx);
    if (s || idx == kNoMark) return s;
    kt->start = ev->ev_pool[idx];
    kt->stop = ev->ev_pool[idx + 1];
    return GL_OK;
}

gl_status prof_end(gl_event *ev, size_t idx) {
    if (idx == kNoMark) return GL_OK;
    HIP_TRY(hipEventRecord(ev->ev_pool[idx + 1], ev->stream));
    return GL_OK;
}

#define PROF(ev, k, call)                                       \
    do {                                                        \
        size_t pidx_ = 0;                                       \
        gl_status ps_ = prof_begin(ev, k, &pidx_);              \
        if (ps_) return ps_;                                    \
        HIP_TRY(call);                                          \
        ps_ = prof_end(ev, pidx_);                              \
        if (ps_) return ps_;                                    \
    } while (0)
// a single-kernel launch that takes the KernelTimer kt_ of its sample
#define PROF_KERNEL(ev, k, call)                                \
    do {                                                        \
        KernelTimer kt_;                                        \
        gl_status ps_ = prof_timer(ev, k, &kt_);                \
        if (ps_) return ps_;                                    \
        HIP_TRY(call);                                          \
    } while (0)

// one field step n -> n+1; site fields F^n in the same pass when the event
// has particles
template <typename T>
gl_status field_step(gl_event *ev, bool site_fields) {
    const int nxt = 1 - ev->cur;
    const double tau = ev->n * ev->dtau;
    int reunit = 0;
    if (!ev->fp64() && ev->desc.reunit_every > 0 &&
        ev->n % ev->desc.reunit_every == ev->desc.reunit_every - 1)
        reunit = 1;
    const bool stat = ev->stat_on && ev->n >= ev->stat_n0 && ev->n - 1 < ev->desc.max_steps;
    const bool ll = ev->ll_on && ev->n >= ev->ll_n0 && ev->n - 1 < ev->desc.max_steps;
    PROF_KERNEL(ev, 0, (launch_field_step<T>(ev->stream, ev->N, ev->fields<T>(ev->cur), ev->fields<T>(nxt),
                                             site_fields || stat || ll ? (T *)(ev->ws + ev->L.F) : nullptr, tau,
                                             ev->dtau, reunit, kt_)));
    if (stat) {
        // static quarks: accumulate the site fields at tau_n, series row n - 1 (time tau_{n+1/2})
        int nb = 0;
        double *part = (double *)(ev->ws + ev->L.stat_part);
        PROF(ev, 1, (launch_static_accum<T>(ev->stream, ev->N, (const T *)(ev->ws + ev->L.F),
                                            (double *)(ev->ws + ev->L.stat), ev->dtau, part, &nb)));
        HIP_TRY(launch_series_reduce(ev->stream, part, nb, 1, ev->stat_series() + (ev->n - 1) * kMaxSpecies * 4,
                                     nullptr));
        ev->stat_rows = std::max<int64_t>(ev->stat_rows, ev->n);
    }
    if (ll) {
        // lightlike jets: transported forces at tau_n with the x links of tau_n (state cur)
        int nb = 0;
        double *part = (double *)(ev->ws + ev->L.ll_part);
        double *W = (double *)(ev->ws + ev->L.ll), *I = W + 18 * ev->n2;
        PROF(ev, 1, (launch_lightlike_accum<T>(ev->stream, ev->N, (const T *)(ev->ws + ev->L.F),
                                               ev->fields<T>(ev->cur).U, W, I, ev->n - ev->ll_n0, ev->dtau, part,
                                               &nb)));
        HIP_TRY(launch_series_reduce(ev->stream, part, nb, 1, ev->ll_series() + (ev->n - 1) * kMaxSpecies * 4,
                                     nullptr));
        ev->ll_rows = std::max<int64_t>(ev->ll_rows, ev->n);
    }
    ev->cur = nxt;
    ev->n += 1;
    return GL_OK;
}

// reduce the pending partial rows into their series rows (one launch)
gl_status flush_series(gl_event *ev) {
    if (ev->pend == 0) return GL_OK;
    const int ns = (int)ev->species.size();
    PROF(ev, 3, (launch_series_reduce_steps(ev->stream, ev->partials(), partial_slot_stride(ev->L.slots), ev->pend,
                                            (int)(ev->slots_used / kPushBlock), ns,
                                            ev->series() + ev->pend_row0 * kMaxSpecies * 4, ev->p0sum())));
    ev->pend = 0;
    return GL_OK;
}

template <typename T>
gl_status push(gl_event *ev) {
    const int64_t n_prev = ev->n - 1;   // particles advance n_prev -> n
    const int64_t row = n_prev - 1;
    if (row >= ev->desc.max_steps) return fail(GL_EINVAL, "series capacity (max_steps) exhausted");
    const int ns = (int)ev->species.size();
    if (ev->pend == 0) ev->pend_row0 = row;
    if (ev->perm_pending) {
        const int nb = 1 - ev->pbuf;
        PROF_KERNEL(ev, 4, (launch_push_permuted<T>(ev->stream, ev->N, ev->parts<T>(ev->pbuf), ev->parts<T>(nb),
                                                    sort_perm(ev->scratch()), ev->ids(ev->pbuf), ev->ids(nb),
                                                    ev->slots_used, ev->fields<T>(1 - ev->cur),
                                                    (const T *)(ev->ws + ev->L.F), ev->tab<T>(), ns, (int)n_prev,
                                                    ev->dtau, ev->partials(ev->pend), kt_)));
        ev->pbuf = nb;
        ev->perm_pending = false;
    } else {
        PROF_KERNEL(ev, 2, (launch_push<T>(ev->stream, ev->N, ev->parts<T>(), ev->slots_used,
                                           ev->fields<T>(1 - ev->cur), (const T *)(ev->ws + ev->L.F), ev->tab<T>(),
                                           ns, (int)n_prev, ev->dtau, ev->partials(ev->pend), kt_)));
    }
    ev->pend++;
    if (ev->pend == kReduceSlots) {
        gl_status s = flush_series(ev);
        if (s) return s;
    }
    ev->rows = std::max<int64_t>(ev->rows, row + 1);
    ev->push_due = false;
    ev->since_sort++;
    return GL_OK;
}

template <typename T>
gl_status sort_t(gl_event *ev) {
    const int nb = 1 - ev->pbuf;
    HIP_TRY(launch_sort_particles<T>(ev->stream, ev->N, ev->parts<T>(ev->pbuf), ev->parts<T>(nb), ev->slots_used,
                                     ev->scratch(), ev->ids(ev->pbuf), ev->ids(nb)));
    ev->pbuf = nb;
    ev->since_sort = 0;
    ev->perm_pending = false;   // a full sort supersedes a pending order
    return GL_OK;
}

gl_status sort_particles(gl_event *ev) {
    if (ev->slots_used == 0) return GL_OK;
    return ev->fp64() ? sort_t<double>(ev) : sort_t<float>(ev);
}

// the sorted order only; the next push moves the particles by it
template <typename T>
gl_status sort_order_t(gl_event *ev) {
    HIP_TRY(launch_sort_order<T>(ev->stream, ev->N, ev->parts<T>(ev->pbuf), ev->slots_used, ev->scratch()));
    ev->perm_pending = true;
    ev->since_sort = 0;
    return GL_OK;
}

// apply a pending sort permutation without a push
template <typename T>
gl_status apply_pending_t(gl_event *ev) {
    const int nb = 1 - ev->pbuf;
    HIP_TRY(launch_permute<T>(ev->stream, ev->parts<T>(ev->pbuf), ev->parts<T>(nb), sort_perm(ev->scratch()),
                              ev->slots_used, ev->ids(ev->pbuf), ev->ids(nb)));
    ev->pbuf = nb;
    ev->perm_pending = false;
    return GL_OK;
}

gl_status apply_pending_sort(gl_event *ev) {
    if (!ev->perm_pending) return GL_OK;
    return ev->fp64() ? apply_pending_t<double>(ev) : apply_pending_t<float>(ev);
}

// the per-species sums of the squared momenta at formation, which the
// momentum series subtract (Sec. 2: broadening relative to formation); taken
// once whenever the particle set changes
gl_status p0_sums(gl_event *ev) {
    const int ns = (int)ev->species.size();
    if (ev->slots_used == 0 || ns == 0) return GL_OK;
    if (ev->fp64())
        HIP_TRY(launch_p0_sums<double>(ev->stream, ev->parts<double>(), ev->slots_used, ns, ev->partials(),
                                       ev->p0sum()));
    else
        HIP_TRY(launch_p0_sums<float>(ev->stream, ev->parts<float>(), ev->slots_used, ns, ev->partials(),
                                      ev->p0sum()));
    return GL_OK;
}

// failure detection: the whole field state at the current step
gl_status check_state(gl_event *ev, int *first_bad) {
    const int64_t n = (int64_t)kStateVals * ev->n2;
    const int step = (int)std::min<int64_t>(ev->n, 0x7F7F7F7E);
    if (ev->fp64())
        HIP_TRY(launch_check_finite<double>(ev->stream, ev->fields<double>(ev->cur).U, n, n, step, first_bad));
    else
        HIP_TRY(launch_check_finite<float>(ev->stream, ev->fields<float>(ev->cur).U, n, n, step, first_bad));
    return GL_OK;
}

// the series rows [row0, row_end) the call wrote (row r holds the particle
// step r + 1 -> r + 2), then the verdict of all checks of the call
gl_status check_report(gl_event *ev, int *first_bad, int64_t row0, int64_t row_end) {
    const int64_t vals = (int64_t)kMaxSpecies * 4;
    if (row_end > row0)
        HIP_TRY(launch_check_finite<double>(ev->stream, ev->series() + row0 * vals, (row_end - row0) * vals, vals,
                                            (int)(row0 + 2), first_bad));
    int h = 0;
    HIP_TRY(hipMemcpyAsync(&h, first_bad, sizeof(int), hipMemcpyDeviceToHost, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    if (h != 0x7F7F7F7F)
        return fail(GL_ENUMERIC, "non-finite values in the fields or the broadening sums at step n = " +
                                     std::to_string(h));
    return GL_OK;
}

gl_status do_field_step(gl_event *ev, bool sf) {
    return ev->fp64() ? field_step<double>(ev, sf) : field_step<float>(ev, sf);
}
gl_status do_push(gl_event *ev, bool defer);

// one coupled step of gl_run: the field step, then the push (a due sort only
// computes its order; the next push applies it)
gl_status one_step(gl_event *ev, bool has_particles) {
    gl_status s = do_field_step(ev, has_particles);
    if (s || !has_particles) return s;
    ev->push_due = true;
    return do_push(ev, true);
}

// the executable graphs of gl_run, after the stream has finished with them
void free_graphs(gl_event *ev) {
    if (!ev->gexec[0] && !ev->gexec[1]) return;
    (void)hipStreamSynchronize(ev->stream);
    for (int k = 0; k < 2; k++) {
        if (ev->gexec[k]) (void)hipGraphExecDestroy(ev->gexec[k]);
        ev->gexec[k] = nullptr;
    }
}

// count steps recorded from the stream into a graph with the same launch
// code and replayed.  Blocks alternate between two executable graphs; the
// one due is first waited for (its previous launch, two blocks back), then
// updated in place (same topology, new step-dependent arguments) or
// instantiated anew.  The host state advances while recording, so a failure
// here leaves the event uninitialised rather than out of step.
gl_status graph_block(gl_event *ev, int32_t count, bool has_particles) {
    const int slot = ev->gslot;
    if (!ev->gdone[slot]) HIP_TRY(hipEventCreateWithFlags(&ev->gdone[slot], hipEventDisableTiming));
    HIP_TRY(hipStreamBeginCapture(ev->stream, hipStreamCaptureModeRelaxed));
    gl_status s = GL_OK;
    for (int32_t k = 0; k < count && !s; k++) s = one_step(ev, has_particles);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ev->stream, &g);
    if (s || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        ev->ready = false;
        return s ? s : fail(GL_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    bool updated = false;
    hipError_t le = hipSuccess;
    hipGraphExec_t &x = ev->gexec[slot];
    if (x) {
        le = hipEventSynchronize(ev->gdone[slot]);   // its previous launch is done
        if (le == hipSuccess) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult r = hipGraphExecUpdateError;
            updated = hipGraphExecUpdate(x, g, &bad, &r) == hipSuccess && r == hipGraphExecUpdateSuccess;
            if (!updated) {
                (void)hipGetLastError();   // a refused update is expected here; keep it out of later launch checks
                (void)hipGraphExecDestroy(x);
                x = nullptr;
            }
        }
    }
    if (le == hipSuccess && !updated) {
        le = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (le == hipSuccess) ev->graph_instantiations++;
    }
    if (le == hipSuccess) le = hipGraphLaunch(x, ev->stream);
    if (le == hipSuccess) le = hipEventRecord(ev->gdone[slot], ev->stream);
    (void)hipGraphDestroy(g);
    if (le != hipSuccess) {
        ev->ready = false;
        return fail(GL_EDEVICE, std::string("graph replay: ") + hipGetErrorString(le));
    }
    ev->gslot = slot ^ 1;
    ev->graph_launches++;
    return GL_OK;
}
gl_status sort_particles(gl_event *ev);

// the sort by cell and the formation sums of a changed particle set.  A
// stable sort gives the same order as sorting after each added species (each
// added block follows the earlier ones, particles in creation order).
gl_status settle_particles(gl_event *ev) {
    if (!ev->set_changed) return GL_OK;
    gl_status s = sort_particles(ev);
    if (s) return s;
    s = p0_sums(ev);
    if (s) return s;
    ev->set_changed = false;
    return GL_OK;
}

// the push, then a sort when one is due: with defer, only the sorted order,
// which the next push applies
gl_status do_push(gl_event *ev, bool defer = false) {
    gl_status s = settle_particles(ev);
    if (s) return s;
    s = ev->fp64() ? push<double>(ev) : push<float>(ev);
    if (s) return s;
    if (ev->sort_every > 0 && ev->since_sort >= ev->sort_every && ev->slots_used > 0) {
        if (defer) return ev->fp64() ? sort_order_t<double>(ev) : sort_order_t<float>(ev);
        return sort_particles(ev);
    }
    return GL_OK;
}

int32_t nform_of(double tau_form_fm, double dtau_fm) {
    double r = std::ceil(tau_form_fm / dtau_fm);
    if (!(r >= 1.0)) r = 1.0;
    if (r > 2e9) r = 2e9;
    return (int32_t)r;
}

gl_status fill_species(gl_event *ev, const gl_species_desc *sp, SpeciesInfo &si) {
    if (!(sp->mass_GeV >= 0) || !(sp->p0_GeV >= 0)) return fail(GL_EINVAL, "mass and p0 must be >= 0");
    if (sp->kind != GL_KIND_HEAVY_QUARK && sp->kind != GL_KIND_JET) return fail(GL_EINVAL, "unknown kind");
    double tf = sp->tau_form_fm;
    if (tf < 0) {
        double mT = std::sqrt(sp->mass_GeV * sp->mass_GeV + sp->p0_GeV * sp->p0_GeV);
        if (!(mT > 0)) return fail(GL_EINVAL, "tau_form = 1/(2 m_T) needs m_T > 0");
        tf = kHbarC / (2.0 * mT);
    }
    if (sp->mass_GeV == 0 && sp->p0_GeV == 0) return fail(GL_EINVAL, "massless particle needs p0 > 0");
    si.desc = *sp;
    si.tau_form_fm = tf;
    si.nform = nform_of(tf, ev->dtau * ev->a_fm);
    si.mass_lat = sp->mass_GeV * ev->a_gev;
    si.p0_lat = sp->p0_GeV * ev->a_gev;
    return GL_OK;
}

// new particles of one species occupy slots [slot0, slot0 + n); the slots up
// to the next multiple of the push workgroup are padding (species -1)
template <typename T>
gl_status init_particles(gl_event *ev, const SpeciesInfo &si, int sid, uint64_t seed, int64_t slot0,
                         int64_t slots_end) {
    PartPtrs<T> p = ev->parts<T>();
    HIP_TRY(hipMemsetAsync(p.species + slot0, 0xFF, (slots_end - slot0) * sizeof(int32_t), ev->stream));
    HIP_TRY(launch_particles_init<T>(ev->stream, ev->N, p, slot0, si.n, seed, sid, si.desc.kind, si.p0_lat));
    HIP_TRY(launch_iota(ev->stream, ev->ids() + slot0, slots_end - slot0, si.n, (int32_t)slot0));
    return GL_OK;
}

template <typename T>
gl_status finish_init(gl_event *ev) {
    int *status = (int *)(ev->ws + ev->L.status);
    HIP_TRY(hipMemsetAsync(status, 0, sizeof(int), ev->stream));
    HIP_TRY(launch_match_pi0(ev->stream, ev->N, (double *)(ev->ws + ev->L.VA), (double *)(ev->ws + ev->L.VB),
                             (double *)(ev->ws + ev->L.U0), (double *)(ev->ws + ev->L.pi0), status,
                             ev->match_max_iter, ev->match_tol));
    ev->cur = 0;
    HIP_TRY(launch_first_half_step<T>(ev->stream, ev->N, (double *)(ev->ws + ev->L.U0),
                                      (double *)(ev->ws + ev->L.pi0), ev->fields<T>(0), ev->dtau));
    int h = 0;
    HIP_TRY(hipMemcpyAsync(&h, status, sizeof(int), hipMemcpyDeviceToHost, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    ev->n = 1;
    ev->ready = true;
    ev->push_due = false;
    ev->rows = 0;
    if (ev->desc.max_steps > 0)
        HIP_TRY(hipMemsetAsync(ev->series(), 0, (size_t)ev->desc.max_steps * kMaxSpecies * 4 * sizeof(double),
                               ev->stream));
    if (h) return fail(GL_ENOTCONV, "matching Newton iteration did not converge on some link");
    return GL_OK;
}

// element of value k of site x in chunked planes: ((k / NV) n2 + x) NV + k mod NV
template <typename T>
inline size_t chunk_index(size_t n2, int k, size_t x) {
    const size_t NV = 16 / sizeof(T);
    return ((size_t)k / NV * n2 + x) * NV + (size_t)k % NV;
}

// K host planes [K][n2] (FP64) into a device array in chunked planes
template <typename T>
gl_status copy_in(gl_event *ev, void *dev, const double *host, int K) {
    const size_t n2 = ev->n2;
    std::vector<T> tmp((size_t)K * n2);
    for (int k = 0; k < K; k++)
        for (size_t x = 0; x < n2; x++) tmp[chunk_index<T>(n2, k, x)] = (T)host[(size_t)k * n2 + x];
    HIP_TRY(hipMemcpyAsync(dev, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    return GL_OK;
}

template <typename T>
gl_status copy_out(gl_event *ev, double *host, const void *dev, int K) {
    const size_t n2 = ev->n2;
    std::vector<T> tmp((size_t)K * n2);
    HIP_TRY(hipMemcpyAsync(tmp.data(), dev, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    for (int k = 0; k < K; k++)
        for (size_t x = 0; x < n2; x++) host[(size_t)k * n2 + x] = (double)tmp[chunk_index<T>(n2, k, x)];
    return GL_OK;
}

template <typename T>
gl_status get_site_fields_t(gl_event *ev, double *F) {
    // planes [6][8][n2]; E_x and E_y add their second halves where those are
    // stored apart (half_stored)
    const size_t n2 = ev->n2;
    std::vector<T> tmp((size_t)kSiteRec * n2);
    HIP_TRY(hipMemcpyAsync(tmp.data(), ev->ws + ev->L.F, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    // device records in chunked planes
    auto at = [&](int k, size_t x) { return (double)tmp[chunk_index<T>(n2, k, x)]; };
    for (int k = 0; k < 48; k++)
        for (size_t x = 0; x < n2; x++) F[(size_t)k * n2 + x] = at(k, x);
    for (int k = 0; k < 16; k++)
        for (size_t x = 0; x < n2; x++)
            if (half_stored(k / 8, (int)(x % ev->N), (int)(x / ev->N))) F[(size_t)k * n2 + x] += at(48 + k, x);
    return GL_OK;
}

// links: the host holds all 18 values of each link ([36][n2], U_1 then U_2),
// the state its first two rows; the third row comes back as the conjugate
// cross product of the two
template <typename T>
gl_status copy_in_links(gl_event *ev, void *dev, const double *host) {
    const size_t n2 = ev->n2;
    std::vector<double> rows((size_t)2 * kLinkVals * n2);
    for (int d = 0; d < 2; d++)
        for (int c = 0; c < kLinkVals; c++)
            std::copy(host + (size_t)(18 * d + c) * n2, host + (size_t)(18 * d + c + 1) * n2,
                      rows.begin() + (size_t)(kLinkVals * d + c) * n2);
    return copy_in<T>(ev, dev, rows.data(), 2 * kLinkVals);
}
template <typename T>
gl_status copy_out_links(gl_event *ev, double *host, const void *dev) {
    const size_t n2 = ev->n2;
    std::vector<double> rows((size_t)2 * kLinkVals * n2);
    gl_status s = copy_out<T>(ev, rows.data(), dev, 2 * kLinkVals);
    if (s) return s;
    for (int d = 0; d < 2; d++)
        for (size_t x = 0; x < n2; x++) {
            auto v = [&](int c) { return rows[(size_t)(kLinkVals * d + c) * n2 + x]; };
            for (int c = 0; c < kLinkVals; c++) host[(size_t)(18 * d + c) * n2 + x] = v(c);
            // row 2 = conj(r0 x r1); entry (i, j) at 2(3i + j)
            for (int k = 0; k < 3; k++) {
                const int a = (k + 1) % 3, b = (k + 2) % 3;
                const double r0a = v(2 * a), i0a = v(2 * a + 1), r0b = v(2 * b), i0b = v(2 * b + 1);
                const double r1a = v(2 * (3 + a)), i1a = v(2 * (3 + a) + 1), r1b = v(2 * (3 + b)), i1b = v(2 * (3 + b) + 1);
                const double cr = r0a * r1b - i0a * i1b - (r0b * r1a - i0b * i1a);
                const double ci = r0a * i1b + i0a * r1b - (r0b * i1a + i0b * r1a);
                host[(size_t)(18 * d + 2 * (6 + k)) * n2 + x] = cr;
                host[(size_t)(18 * d + 2 * (6 + k) + 1) * n2 + x] = -ci;
            }
        }
    return GL_OK;
}

template <typename T>
gl_status set_state_t(gl_event *ev, const double *U, const double *E, const double *phi, const double *pi) {
    FieldPtrs<T> f = ev->fields<T>(ev->cur);
    gl_status s;
    if ((s = copy_in_links<T>(ev, f.U, U))) return s;
    if ((s = copy_in<T>(ev, f.E, E, 16))) return s;
    if ((s = copy_in<T>(ev, f.phi, phi, 8))) return s;
    return copy_in<T>(ev, f.pi, pi, 8);
}

template <typename T>
gl_status get_state_t(gl_event *ev, double *U, double *E, double *phi, double *pi) {
    FieldPtrs<T> f = ev->fields<T>(ev->cur);
    gl_status s;
    if (U && (s = copy_out_links<T>(ev, U, f.U))) return s;
    if (E && (s = copy_out<T>(ev, E, f.E, 16))) return s;
    if (phi && (s = copy_out<T>(ev, phi, f.phi, 8))) return s;
    if (pi && (s = copy_out<T>(ev, pi, f.pi, 8))) return s;
    return GL_OK;
}

template <typename T>
gl_status set_particles_t(gl_event *ev, int64_t n, const int32_t *cell, const double *off, const double *eta,
                          const double *p, const double *Q, const double *p0, const int32_t *species) {
    const int64_t c = ev->L.slots;
    std::vector<int32_t> cx(c, 0), cy(c, 0), sp(c, -1), id(c, -1);
    // the record planes followed by px0, py0, pz0 (contiguous on the device)
    std::vector<T> f((kPartRec<T> + 3) * (size_t)c, T(0));
    auto rec = [&](int k, int64_t i) -> T & { return f[chunk_index<T>((size_t)c, k, (size_t)i)]; };
    T *f0 = f.data() + kPartRec<T> * (size_t)c;
    for (int64_t i = 0; i < n; i++) {
        id[i] = (int32_t)i;
        cx[i] = cell[i];
        cy[i] = cell[n + i];
        sp[i] = species[i];
        rec(kOx, i) = (T)off[i];
        rec(kOy, i) = (T)off[n + i];
        rec(kEta, i) = (T)eta[i];
        rec(kPx, i) = (T)p[i];
        rec(kPy, i) = (T)p[n + i];
        rec(kPeta, i) = (T)p[2 * n + i];
        for (int a = 0; a < 8; a++) rec(kQ + a, i) = (T)Q[a * n + i];
        f0[0 * c + i] = (T)p0[i];
        f0[1 * c + i] = (T)p0[n + i];
        f0[2 * c + i] = (T)p0[2 * n + i];
    }
    PartPtrs<T> P = ev->parts<T>();
    HIP_TRY(hipMemcpyAsync(ev->ids(), id.data(), c * 4, hipMemcpyHostToDevice, ev->stream));
    HIP_TRY(hipMemcpyAsync(P.cx, cx.data(), c * 4, hipMemcpyHostToDevice, ev->stream));
    HIP_TRY(hipMemcpyAsync(P.cy, cy.data(), c * 4, hipMemcpyHostToDevice, ev->stream));
    HIP_TRY(hipMemcpyAsync(P.species, sp.data(), c * 4, hipMemcpyHostToDevice, ev->stream));
    HIP_TRY(hipMemcpyAsync(P.st, f.data(), f.size() * sizeof(T), hipMemcpyHostToDevice, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    return GL_OK;
}

template <typename T>
gl_status get_particles_t(gl_event *ev, int64_t n, int32_t *cell, double *off, double *eta, double *p,
                          double *Q, double *p0, int32_t *species) {
    const int64_t c = ev->L.slots;
    std::vector<int32_t> cx(c), cy(c), sp(c), id(c);
    std::vector<T> f((kPartRec<T> + 3) * (size_t)c);
    auto rec = [&](int k, int64_t j) { return (double)f[chunk_index<T>((size_t)c, k, (size_t)j)]; };
    const T *f0 = f.data() + kPartRec<T> * (size_t)c;
    PartPtrs<T> P = ev->parts<T>();
    if (c > 0) {
        HIP_TRY(hipMemcpyAsync(id.data(), ev->ids(), c * 4, hipMemcpyDeviceToHost, ev->stream));
        HIP_TRY(hipMemcpyAsync(cx.data(), P.cx, c * 4, hipMemcpyDeviceToHost, ev->stream));
        HIP_TRY(hipMemcpyAsync(cy.data(), P.cy, c * 4, hipMemcpyDeviceToHost, ev->stream));
        HIP_TRY(hipMemcpyAsync(sp.data(), P.species, c * 4, hipMemcpyDeviceToHost, ev->stream));
        HIP_TRY(hipMemcpyAsync(f.data(), P.st, f.size() * sizeof(T), hipMemcpyDeviceToHost, ev->stream));
        HIP_TRY(hipStreamSynchronize(ev->stream));
    }
    for (int64_t j = 0; j < ev->slots_used; j++) {
        {
            if (id[j] < 0) continue;
            int64_t i = id[j];
            if (i >= n) return fail(GL_EDEVICE, "corrupt particle id");
            if (cell) { cell[i] = cx[j]; cell[n + i] = cy[j]; }
            if (species) species[i] = sp[j];
            if (off) { off[i] = rec(kOx, j); off[n + i] = rec(kOy, j); }
            if (eta) eta[i] = rec(kEta, j);
            if (p) { p[i] = rec(kPx, j); p[n + i] = rec(kPy, j); p[2 * n + i] = rec(kPeta, j); }
            if (p0) { p0[i] = f0[0 * c + j]; p0[n + i] = f0[1 * c + j]; p0[2 * n + i] = f0[2 * c + j]; }
            if (Q)
                for (int a = 0; a < 8; a++) Q[a * n + i] = rec(kQ + a, j);
        }
    }
    return GL_OK;
}

int64_t total_particles(const gl_event *ev) {
    int64_t t = 0;
    for (auto &s : ev->species) t += s.n;
    return t;
}

gl_status read_series_species(gl_event *ev, int32_t species, std::vector<double> &rows4) {
    if (species < 0 || species >= (int32_t)ev->species.size()) return fail(GL_EINVAL, "no such species");
    std::vector<double> all((size_t)ev->rows * kMaxSpecies * 4);
    if (ev->rows > 0) {
        HIP_TRY(hipMemcpyAsync(all.data(), ev->series(), all.size() * sizeof(double), hipMemcpyDeviceToHost,
                               ev->stream));
        HIP_TRY(hipStreamSynchronize(ev->stream));
    }
    rows4.resize((size_t)ev->rows * 4);
    for (int64_t k = 0; k < ev->rows; k++)
        for (int c = 0; c < 4; c++) rows4[k * 4 + c] = all[(k * kMaxSpecies + species) * 4 + c];
    return GL_OK;
}

}  // namespace

// ============================================================================
extern "C" {

const char *gl_last_error(void) { return g_err.c_str(); }

const char *gl_status_string(gl_status s) {
    switch (s) {
        case GL_OK: return "ok";
        case GL_EINVAL: return "invalid argument";
        case GL_ESTATE: return "call not allowed in the current state";
        case GL_ENOTCONV: return "matching did not converge";
        case GL_ENUMERIC: return "non-finite values";
        case GL_EDEVICE: return "HIP runtime error";
        case GL_ENOMEM: return "workspace too small";
        default: return "unknown status";
    }
}

gl_status gl_max_particles(int32_t precision, int64_t *max_particles) {
    if (precision != 64 && precision != 32) return fail(GL_EINVAL, "precision must be 64 or 32");
    if (!max_particles) return fail(GL_EINVAL, "null output");
    *max_particles = max_particles_for(precision);
    return GL_OK;
}

gl_status gl_required_bytes(const gl_lattice_desc *desc, size_t *bytes) {
    Layout L;
    gl_status s = make_layout(desc, L);
    if (s) return s;
    if (!bytes) return fail(GL_EINVAL, "null output");
    *bytes = L.total;
    return GL_OK;
}

gl_status gl_event_create(const gl_lattice_desc *desc, void *workspace, size_t bytes, void *stream,
                          gl_event **out) {
    if (!out) return fail(GL_EINVAL, "null output");
    *out = nullptr;
    Layout L;
    gl_status s = make_layout(desc, L);
    if (s) return s;
    if (!workspace) return fail(GL_EINVAL, "null workspace");
    if (((uintptr_t)workspace & 255) != 0) return fail(GL_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < L.total) return fail(GL_ENOMEM, "workspace smaller than gl_required_bytes()");
    gl_event *ev = new (std::nothrow) gl_event();
    if (!ev) return fail(GL_ENOMEM, "host allocation failed");
    ev->desc = *desc;
    ev->L = L;
    ev->N = desc->N;
    ev->n2 = (size_t)desc->N * desc->N;
    ev->a_fm = desc->L_fm / desc->N;
    ev->a_gev = ev->a_fm / kHbarC;
    ev->dtau = desc->dtau_over_a;
    ev->stream = (hipStream_t)stream;
    ev->ws = (char *)workspace;
    *out = ev;
    return GL_OK;
}

void gl_event_destroy(gl_event *ev) {
    if (!ev) return;
    free_graphs(ev);
    // timing events may still be pending on the stream
    if (!ev->ev_pool.empty()) (void)hipStreamSynchronize(ev->stream);
    for (hipEvent_t e : ev->gdone)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev->ev_pool) (void)hipEventDestroy(e);
    delete ev;
}

// the Wilson lines of both nuclei into VA, VB (steps 1-3 of the MV initialisation)
static gl_status wilson_lines(gl_event *ev, int n_sheets, double m_ir_GeV, double uv_GeV, const double *rho_dev,
                              double sigma, uint64_t seed) {
    const int N = ev->N;
    double m2 = (m_ir_GeV * ev->a_gev) * (m_ir_GeV * ev->a_gev);
    double uv2 = uv_GeV > 0 ? (uv_GeV * ev->a_gev) * (uv_GeV * ev->a_gev) : 0.0;
    if (!(m2 > 0)) return fail(GL_EINVAL, "infrared regulator must be > 0");
    if (!valid_N_for_fft(N)) return fail(GL_EINVAL, "MV initialisation needs N = 2^a 3^b");
    double *V[2] = {(double *)(ev->ws + ev->L.VA), (double *)(ev->ws + ev->L.VB)};
    double2 *planes = (double2 *)(ev->ws + ev->L.planes);
    double2 *tab = (double2 *)(ev->ws + ev->L.fft_tab);
    HIP_TRY(launch_fft_tables(ev->stream, N, tab));
    for (int nuc = 0; nuc < 2; nuc++) {
        HIP_TRY(launch_wilson_init(ev->stream, N, V[nuc]));
        for (int sh0 = 0; sh0 < n_sheets; sh0 += kSheetChunk) {
            const int cnt = std::min(kSheetChunk, n_sheets - sh0);
            if (rho_dev) {
                for (int k = 0; k < cnt; k++)
                    HIP_TRY(launch_charges_to_planes(
                        ev->stream, N, rho_dev + ((size_t)nuc * n_sheets + sh0 + k) * 8 * ev->n2,
                        planes + (size_t)k * 4 * ev->n2));
                HIP_TRY(launch_poisson(ev->stream, N, m2, uv2, planes, cnt, tab));
            } else {
                // the forward row pass draws the charges itself
                const MvDraw mv{sigma, seed, nuc, sh0};
                HIP_TRY(launch_poisson(ev->stream, N, m2, uv2, planes, cnt, tab, &mv));
            }
            HIP_TRY(launch_wilson_accum(ev->stream, N, planes, cnt, V[nuc]));
        }
    }
    return GL_OK;
}

static gl_status init_common(gl_event *ev, int n_sheets, double m_ir_GeV, double uv_GeV, const double *rho_dev,
                             double sigma, uint64_t seed) {
    gl_status s = wilson_lines(ev, n_sheets, m_ir_GeV, uv_GeV, rho_dev, sigma, seed);
    if (s) return s;
    return ev->fp64() ? finish_init<double>(ev) : finish_init<float>(ev);
}

// D(r), r = 0..rmax, of the stored Wilson line of one nucleus (device
// kernels; partials in the initialisation scratch planes)
static gl_status dipole_curve(gl_event *ev, int nucleus, int rmax, std::vector<double> &D) {
    const double *V = (const double *)(ev->ws + (nucleus == 0 ? ev->L.VA : ev->L.VB));
    double *part = (double *)(ev->ws + ev->L.planes);
    const int nb = (int)((ev->n2 + 255) / 256);
    double *Dd = part + (size_t)(rmax + 1) * nb;
    HIP_TRY(launch_dipole(ev->stream, ev->N, V, rmax, part, Dd));
    D.assign(rmax + 1, 0.0);
    HIP_TRY(hipMemcpyAsync(D.data(), Dd, (rmax + 1) * sizeof(double), hipMemcpyDeviceToHost, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    return GL_OK;
}

// Q_s [GeV] from D(sqrt(2)/Q_s) = exp(-1/2), r linearly interpolated between
// the lattice separations around the crossing; 0 if D stays above it
static double qs_from_dipole(const std::vector<double> &D, double a_gev) {
    const double target = std::exp(-0.5);
    for (size_t r = 1; r < D.size(); r++)
        if (D[r] <= target) {
            const double rs = (double)(r - 1) + (D[r - 1] - target) / (D[r - 1] - D[r]);
            return std::sqrt(2.0) / (rs * a_gev);
        }
    return 0.0;
}

gl_status gl_init_glasma(gl_event *ev, const gl_mv_desc *mv, uint64_t seed) {
    if (!mv) return fail(GL_EINVAL, "null argument");
    if (gl_status s = check_free(ev)) return s;
    if (mv->n_sheets < 1) return fail(GL_EINVAL, "n_sheets must be >= 1");
    if (!(mv->g2mu_GeV >= 0)) return fail(GL_EINVAL, "g2mu must be >= 0");
    if (!(mv->uv_cut_GeV >= 0)) return fail(GL_EINVAL, "uv_cut_GeV must be >= 0");
    double sigma = mv->g2mu_GeV * ev->a_gev / std::sqrt((double)mv->n_sheets);
    return init_common(ev, mv->n_sheets, mv->m_ir_GeV, mv->uv_cut_GeV, nullptr, sigma, seed);
}

gl_status gl_init_glasma_from_charges(gl_event *ev, const double *rho_dev, int32_t n_sheets, double m_ir_GeV) {
    if (!rho_dev) return fail(GL_EINVAL, "null argument");
    if (gl_status s = check_free(ev)) return s;
    if (n_sheets < 1) return fail(GL_EINVAL, "n_sheets must be >= 1");
    return init_common(ev, n_sheets, m_ir_GeV, 0.0, rho_dev, 0.0, 0);
}

gl_status gl_add_species(gl_event *ev, const gl_species_desc *sp, int64_t n, uint64_t seed, int32_t *species_id) {
    if (!sp) return fail(GL_EINVAL, "null argument");
    if (gl_status s = check_free(ev)) return s;
    if (n < 1) return fail(GL_EINVAL, "n must be >= 1");
    if ((int)ev->species.size() >= kMaxSpecies) return fail(GL_EINVAL, "too many species");
    if (ev->push_due) return fail(GL_ESTATE, "a particle step is due");
    SpeciesInfo si;
    gl_status s = fill_species(ev, sp, si);
    if (s) return s;
    si.n = n;
    const int64_t slot0 = total_particles(ev);   // valid particles occupy [0, total) (padding sorts last)
    const int64_t end = (slot0 + n + kPushBlock - 1) / kPushBlock * kPushBlock;
    if (end > ev->L.slots) return fail(GL_ENOMEM, "particle capacity exceeded");
    int sid = (int)ev->species.size();
    ev->species.push_back(si);
    ev->slots_used = end;
    s = ev->fp64() ? init_particles<double>(ev, si, sid, seed, slot0, end)
                   : init_particles<float>(ev, si, sid, seed, slot0, end);
    if (s) return s;
    ev->set_changed = true;   // sorted, with its formation sums, before the next push
    if (species_id) *species_id = sid;
    return GL_OK;
}

gl_status gl_evolve_fields(gl_event *ev, int32_t n_steps) {
    if (gl_status s = check_free(ev)) return s;
    if (!ev->ready) return fail(GL_ESTATE, "fields not initialised");
    if (n_steps < 0) return fail(GL_EINVAL, "n_steps must be >= 0");
    bool has_particles = ev->slots_used > 0;
    if (has_particles && (ev->push_due || n_steps > 1))
        return fail(GL_ESTATE, "particles are not at the field time: push them first, one field step at a time");
    for (int32_t k = 0; k < n_steps; k++) {
        gl_status s = do_field_step(ev, has_particles);
        if (s) return s;
        if (has_particles) ev->push_due = true;
    }
    return GL_OK;
}

gl_status gl_push_particles(gl_event *ev) {
    if (gl_status s = check_free(ev)) return s;
    if (!ev->push_due) return fail(GL_ESTATE, "no particle step is due: call gl_evolve_fields(ev, 1) first");
    gl_status s = do_push(ev);
    if (s) return s;
    return flush_series(ev);
}

gl_status gl_run(gl_event *ev, int32_t n_steps) {
    if (gl_status s = check_free(ev)) return s;
    if (!ev->ready) return fail(GL_ESTATE, "fields not initialised");
    if (ev->push_due) return fail(GL_ESTATE, "a particle step is due");
    if (n_steps < 0) return fail(GL_EINVAL, "n_steps must be >= 0");
    bool has_particles = ev->slots_used > 0;
    if (has_particles && ev->n - 1 + n_steps > ev->desc.max_steps)
        return fail(GL_EINVAL, "series capacity (max_steps) too small for this run");
    // this call writes the series rows [n - 1, n - 1 + n_steps) (row r: the
    // particle step r + 1 -> r + 2)
    const int64_t row0 = ev->n - 1, row_end = has_particles ? row0 + n_steps : row0;
    int *first_bad = (int *)(ev->ws + ev->L.status) + 1;
    const bool checks = ev->check_every > 0 && n_steps > 0;
    if (checks) HIP_TRY(hipMemsetAsync(first_bad, 0x7F, sizeof(int), ev->stream));
    // a changed particle set is sorted and summed once, before any recording
    gl_status s = has_particles ? settle_particles(ev) : GL_OK;
    // whole blocks of graph_steps from captured graphs (not while kernels are
    // timed or checked: those keep direct launches), the rest launched directly
    const bool graphs = ev->graph_steps > 0 && ev->prof == 0 && !checks;
    for (int32_t k = 0; k < n_steps && !s;) {
        if (graphs && n_steps - k >= ev->graph_steps) {
            s = graph_block(ev, ev->graph_steps, has_particles);
            k += ev->graph_steps;
            continue;
        }
        s = one_step(ev, has_particles);
        k++;
        if (!s && checks && (k % ev->check_every == 0 || k == n_steps)) s = check_state(ev, first_bad);
    }
    // no sort is left pending, also after an error
    const gl_status sp = apply_pending_sort(ev);
    if (s) return s;
    if (sp) return sp;
    s = flush_series(ev);
    if (s || !checks) return s;
    return check_report(ev, first_bad, row0, row_end);
}

gl_status gl_static_start(gl_event *ev, double tau_start_fm) {
    if (gl_status s = check_free(ev)) return s;
    if (!ev->desc.static_correlator) return fail(GL_ESTATE, "event created without static_correlator");
    if (!ev->ready) return fail(GL_ESTATE, "fields not initialised");
    if (!(tau_start_fm >= 0)) return fail(GL_EINVAL, "tau_start_fm must be >= 0");
    const double r = std::ceil(tau_start_fm / (ev->dtau * ev->a_fm) - 1e-9);
    int64_t n0 = r < 1.0 ? 1 : (r > 2e9 ? (int64_t)2e9 : (int64_t)r);
    ev->stat_n0 = std::max<int64_t>(n0, ev->n);
    HIP_TRY(hipMemsetAsync(ev->ws + ev->L.stat, 0, 24 * ev->n2 * sizeof(double), ev->stream));
    HIP_TRY(hipMemsetAsync(ev->stat_series(), 0,
                           std::max(1, ev->desc.max_steps) * (size_t)kMaxSpecies * 4 * sizeof(double), ev->stream));
    ev->stat_rows = 0;
    ev->stat_on = true;
    return GL_OK;
}

static gl_status correlator_rows(gl_event *ev, const double *series, int64_t rows, double *out, int32_t cap,
                                 int32_t *n_rows) {
    std::vector<double> s4((size_t)std::max<int64_t>(rows, 1) * kMaxSpecies * 4, 0.0);
    if (rows > 0) {
        HIP_TRY(hipMemcpyAsync(s4.data(), series, (size_t)rows * kMaxSpecies * 4 * sizeof(double),
                               hipMemcpyDeviceToHost, ev->stream));
        HIP_TRY(hipStreamSynchronize(ev->stream));
    }
    const double f2 = 1.0 / (ev->a_gev * ev->a_gev), dt_fm = ev->dtau * ev->a_fm;
    int32_t r = 0;
    for (int64_t k = 0; k < rows; k++) {
        const double *row = s4.data() + (size_t)k * kMaxSpecies * 4;
        if (!(row[3] > 0)) continue;
        if (out) {
            if (r >= cap) return fail(GL_EINVAL, "output too small");
            out[r * 5 + 0] = (k + 1.5) * dt_fm;
            for (int c = 0; c < 3; c++) out[r * 5 + 1 + c] = row[c] / row[3] * f2;
            out[r * 5 + 4] = row[3];
        }
        r++;
    }
    *n_rows = r;
    return GL_OK;
}

gl_status gl_static_broadening(gl_event *ev, double *out, int32_t cap, int32_t *n_rows) {
    if (check_ev(ev) || !n_rows) return fail(GL_EINVAL, "null argument");
    if (!ev->desc.static_correlator) return fail(GL_ESTATE, "event created without static_correlator");
    return correlator_rows(ev, ev->stat_series(), ev->stat_rows, out, cap, n_rows);
}

gl_status gl_lightlike_start(gl_event *ev, double tau_start_fm) {
    if (gl_status s = check_free(ev)) return s;
    if (!ev->desc.lightlike_correlator) return fail(GL_ESTATE, "event created without lightlike_correlator");
    if (!ev->ready) return fail(GL_ESTATE, "fields not initialised");
    if (!(tau_start_fm >= 0)) return fail(GL_EINVAL, "tau_start_fm must be >= 0");
    const double r = std::ceil(tau_start_fm / (ev->dtau * ev->a_fm) - 1e-9);
    int64_t n0 = r < 1.0 ? 1 : (r > 2e9 ? (int64_t)2e9 : (int64_t)r);
    ev->ll_n0 = std::max<int64_t>(n0, ev->n);
    double *W = (double *)(ev->ws + ev->L.ll);
    HIP_TRY(launch_wilson_init(ev->stream, ev->N, W));   // W = 1 at every start site
    HIP_TRY(hipMemsetAsync(W + 18 * ev->n2, 0, 24 * ev->n2 * sizeof(double), ev->stream));
    HIP_TRY(hipMemsetAsync(ev->ll_series(), 0,
                           std::max(1, ev->desc.max_steps) * (size_t)kMaxSpecies * 4 * sizeof(double), ev->stream));
    ev->ll_rows = 0;
    ev->ll_on = true;
    return GL_OK;
}

gl_status gl_lightlike_broadening(gl_event *ev, double *out, int32_t cap, int32_t *n_rows) {
    if (check_ev(ev) || !n_rows) return fail(GL_EINVAL, "null argument");
    if (!ev->desc.lightlike_correlator) return fail(GL_ESTATE, "event created without lightlike_correlator");
    return correlator_rows(ev, ev->ll_series(), ev->ll_rows, out, cap, n_rows);
}

gl_status gl_series(gl_event *ev, double *out, int32_t cap_rows, int32_t *n_rows) {
    if (check_ev(ev) || !n_rows) return fail(GL_EINVAL, "null argument");
    *n_rows = (int32_t)ev->rows;
    if (!out || ev->rows == 0) return GL_OK;
    if (cap_rows < ev->rows) return fail(GL_EINVAL, "output too small");
    HIP_TRY(hipMemcpyAsync(out, ev->series(), (size_t)ev->rows * kMaxSpecies * 4 * sizeof(double),
                           hipMemcpyDeviceToHost, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    return GL_OK;
}

gl_status gl_rates_from_series(const double *series, int32_t rows, double dtau, double *rates) {
    if (!series || !rates || rows < 0 || !(dtau > 0)) return fail(GL_EINVAL, "bad argument");
    double prev[3] = {0, 0, 0};
    bool prev_active = false;
    for (int32_t k = 0; k < rows; k++) {
        double cnt = series[k * 4 + 3];
        if (!(cnt > 0)) {
            rates[k * 3] = rates[k * 3 + 1] = rates[k * 3 + 2] = 0.0;
            prev_active = false;
            continue;
        }
        for (int c = 0; c < 3; c++) {
            double m = series[k * 4 + c] / cnt;
            rates[k * 3 + c] = (m - (prev_active ? prev[c] : 0.0)) / dtau;
            prev[c] = m;
        }
        prev_active = true;
    }
    return GL_OK;
}

gl_status gl_scan_statistics(const double *series, int32_t n_events, int32_t rows, int32_t kind, double dtau_fm,
                             double a_fm, double *out, int32_t cap, int32_t *n_rows) {
    if (!series || !n_rows || n_events < 2 || rows < 0 || (kind != GL_KIND_HEAVY_QUARK && kind != GL_KIND_JET) ||
        !(dtau_fm > 0) || !(a_fm > 0))
        return fail(GL_EINVAL, "bad argument (at least two events, kind heavy quark or jet, dtau and a > 0)");
    const int E = n_events;
    const double a_gev = a_fm / kHbarC, f2 = 1.0 / (a_gev * a_gev), fk = f2 / a_fm;
    const double dtau_lat = dtau_fm / a_fm;
    auto at = [&](int e, int k, int c) { return series[((size_t)e * rows + k) * 4 + c]; };
    // the two components: (dp_x^2 + dp_y^2, dp_z^2) for heavy quarks, (dp_y^2, dp_z^2) for jets
    auto comp = [&](int e, int k, int j) {
        if (j == 1) return at(e, k, 2);
        return kind == GL_KIND_HEAVY_QUARK ? at(e, k, 0) + at(e, k, 1) : at(e, k, 1);
    };
    // pooled sums of a row over all events, and over all but event i (i < 0: none left out)
    auto pooled = [&](int k, int skip, double *A, double *B) {
        double sa = 0, sb = 0, n = 0;
        for (int e = 0; e < E; e++) {
            if (e == skip) continue;
            sa += comp(e, k, 0);
            sb += comp(e, k, 1);
            n += at(e, k, 3);
        }
        *A = n > 0 ? sa / n : 0.0;
        *B = n > 0 ? sb / n : 0.0;
        return n > 0;
    };
    // the observables of row k from one (leave-one-out) sample: <A>, <B>,
    // <B>/<A>, dA/dtau, dB/dtau and the total rate d(A + B)/dtau
    auto observables = [&](int k, int skip, double *v) {
        double A = 0, B = 0, Ap = 0, Bp = 0;
        pooled(k, skip, &A, &B);
        const bool prev = k > 0 && pooled(k - 1, skip, &Ap, &Bp);
        v[0] = A * f2;
        v[1] = B * f2;
        v[2] = A != 0 ? B / A : 0.0;
        v[3] = (A - (prev ? Ap : 0.0)) / dtau_lat * fk;
        v[4] = (B - (prev ? Bp : 0.0)) / dtau_lat * fk;
        v[5] = v[3] + v[4];
    };
    int32_t r = 0;
    for (int k = 0; k < rows; k++) {
        int active = 0;
        for (int e = 0; e < E; e++) active += at(e, k, 3) > 0 ? 1 : 0;
        if (active == 0) continue;
        if (active != E) return fail(GL_EINVAL, "the events disagree on which rows hold active particles");
        if (out) {
            if (r >= cap) return fail(GL_EINVAL, "output too small");
            constexpr int NO = 6;
            double full[NO], jk[NO] = {0, 0, 0, 0, 0, 0}, sq[NO] = {0, 0, 0, 0, 0, 0};
            observables(k, -1, full);
            std::vector<double> loo((size_t)E * NO);
            for (int i = 0; i < E; i++) {
                observables(k, i, &loo[(size_t)i * NO]);
                for (int j = 0; j < NO; j++) jk[j] += loo[(size_t)i * NO + j] / E;
            }
            for (int i = 0; i < E; i++)
                for (int j = 0; j < NO; j++) {
                    const double d = loo[(size_t)i * NO + j] - jk[j];
                    sq[j] += d * d;
                }
            double *o = out + (size_t)r * 14;
            o[0] = (k + 1.5) * dtau_fm;
            o[1] = (k + 1) * dtau_fm;
            for (int j = 0; j < NO; j++) {
                o[2 + 2 * j] = full[j];
                o[3 + 2 * j] = std::sqrt((double)(E - 1) / E * sq[j]);
            }
        }
        r++;
    }
    *n_rows = r;
    return GL_OK;
}

gl_status gl_broadening(gl_event *ev, int32_t species, double *out, int32_t cap, int32_t *n_rows) {
    if (check_ev(ev) || !n_rows) return fail(GL_EINVAL, "null argument");
    std::vector<double> s4;
    gl_status s = read_series_species(ev, species, s4);
    if (s) return s;
    const double f2 = 1.0 / (ev->a_gev * ev->a_gev), dt_fm = ev->dtau * ev->a_fm;
    int32_t r = 0;
    for (int64_t k = 0; k < ev->rows; k++) {
        double cnt = s4[k * 4 + 3];
        if (!(cnt > 0)) continue;
        if (out) {
            if (r >= cap) return fail(GL_EINVAL, "output too small");
            out[r * 5 + 0] = (k + 1.5) * dt_fm;
            for (int c = 0; c < 3; c++) out[r * 5 + 1 + c] = s4[k * 4 + c] / cnt * f2;
            out[r * 5 + 4] = cnt;
        }
        r++;
    }
    *n_rows = r;
    return GL_OK;
}

static gl_status coeff_rows(gl_event *ev, int32_t species, double *out, int32_t cap, int32_t *n_rows, bool kappa) {
    if (check_ev(ev) || !n_rows) return fail(GL_EINVAL, "null argument");
    std::vector<double> s4;
    gl_status s = read_series_species(ev, species, s4);
    if (s) return s;
    std::vector<double> rates(ev->rows * 3);
    if (ev->rows > 0) {
        s = gl_rates_from_series(s4.data(), (int32_t)ev->rows, ev->dtau, rates.data());
        if (s) return s;
    }
    const double fk = 1.0 / (ev->a_gev * ev->a_gev * ev->a_fm), dt_fm = ev->dtau * ev->a_fm;
    const double tf = ev->species[species].tau_form_fm;
    int32_t r = 0;
    const int w = kappa ? 4 : 3;
    for (int64_t k = 0; k < ev->rows; k++) {
        if (!(s4[k * 4 + 3] > 0)) continue;
        if (out) {
            if (r >= cap) return fail(GL_EINVAL, "output too small");
            double tau = (k + 1) * dt_fm;
            if (kappa) {
                out[r * w + 0] = tau;
                out[r * w + 1] = tau - tf;
                out[r * w + 2] = (rates[k * 3] + rates[k * 3 + 1]) * fk;
                out[r * w + 3] = rates[k * 3 + 2] * fk;
            } else {
                out[r * w + 0] = tau;
                out[r * w + 1] = rates[k * 3 + 1] * fk;
                out[r * w + 2] = rates[k * 3 + 2] * fk;
            }
        }
        r++;
    }
    *n_rows = r;
    return GL_OK;
}

gl_status gl_kappa(gl_event *ev, int32_t species, double *out, int32_t cap, int32_t *n_rows) {
    return coeff_rows(ev, species, out, cap, n_rows, true);
}

gl_status gl_qhat(gl_event *ev, int32_t species, double *out, int32_t cap, int32_t *n_rows) {
    return coeff_rows(ev, species, out, cap, n_rows, false);
}

gl_status gl_diagnostics(gl_event *ev, gl_diag *out) {
    if (check_ev(ev) || !out) return fail(GL_EINVAL, "null argument");
    if (!ev->ready) return fail(GL_ESTATE, "fields not initialised");
    double *part = (double *)(ev->ws + ev->L.diag);
    int nb = 0;
    double tau = ev->n * ev->dtau;
    if (tau <= 0) tau = ev->dtau;
    if (ev->fp64()) HIP_TRY(launch_diag<double>(ev->stream, ev->N, ev->fields<double>(ev->cur), tau, part, &nb));
    else HIP_TRY(launch_diag<float>(ev->stream, ev->N, ev->fields<float>(ev->cur), tau, part, &nb));
    std::vector<double> h((size_t)nb * 8);
    HIP_TRY(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nb; b++)
        for (int k = 0; k < 8; k++) v[k] = k < 3 ? std::max(v[k], h[b * 8 + k]) : v[k] + h[b * 8 + k];
    out->gauss_max = v[0];
    out->gauss_rel = v[1] > 0 ? v[0] / v[1] : v[0];
    out->unitarity_max = v[2];
    for (int k = 0; k < 4; k++) out->energy[k] = v[3 + k];
    out->nonfinite = v[7] > 0 ? 1 : 0;
    out->casimir2_dev = 0.0;
    out->casimir3_dev = 0.0;
    if (ev->slots_used > 0) {
        int cb = 0;
        if (ev->fp64()) HIP_TRY(launch_casimir<double>(ev->stream, ev->parts<double>(), ev->slots_used, part, &cb));
        else HIP_TRY(launch_casimir<float>(ev->stream, ev->parts<float>(), ev->slots_used, part, &cb));
        std::vector<double> c((size_t)2 * cb);
        HIP_TRY(hipMemcpyAsync(c.data(), part, c.size() * sizeof(double), hipMemcpyDeviceToHost, ev->stream));
        HIP_TRY(hipStreamSynchronize(ev->stream));
        for (int b = 0; b < cb; b++) {
            out->casimir2_dev = std::max(out->casimir2_dev, c[2 * b]);
            out->casimir3_dev = std::max(out->casimir3_dev, c[2 * b + 1]);
        }
    }
    if (out->nonfinite) return fail(GL_ENUMERIC, "non-finite values in the fields");
    return GL_OK;
}

gl_status gl_set_state(gl_event *ev, const double *U, const double *E, const double *phi, const double *pi,
                       int64_t n) {
    if (!U || !E || !phi || !pi) return fail(GL_EINVAL, "null argument");
    if (gl_status s = check_free(ev)) return s;
    if (n < 1) return fail(GL_EINVAL, "time index must be >= 1");
    gl_status s = ev->fp64() ? set_state_t<double>(ev, U, E, phi, pi) : set_state_t<float>(ev, U, E, phi, pi);
    if (s) return s;
    // a new history: the series rows before the first push read as zero
    if (ev->desc.max_steps > 0)
        HIP_TRY(hipMemsetAsync(ev->series(), 0, (size_t)ev->desc.max_steps * kMaxSpecies * 4 * sizeof(double),
                               ev->stream));
    ev->rows = 0;
    ev->n = n;
    ev->ready = true;
    ev->push_due = false;
    return GL_OK;
}

gl_status gl_get_state(gl_event *ev, double *U, double *E, double *phi, double *pi, int64_t *n) {
    if (check_ev(ev)) return GL_EINVAL;
    if (!ev->ready) return fail(GL_ESTATE, "fields not initialised");
    gl_status s = ev->fp64() ? get_state_t<double>(ev, U, E, phi, pi) : get_state_t<float>(ev, U, E, phi, pi);
    if (s) return s;
    if (n) *n = ev->n;
    return GL_OK;
}

gl_status gl_get_site_fields(gl_event *ev, double *F) {
    if (check_ev(ev) || !F) return fail(GL_EINVAL, "null argument");
    if (ev->slots_used == 0) return fail(GL_ESTATE, "site fields are only computed when the event has particles");
    return ev->fp64() ? get_site_fields_t<double>(ev, F) : get_site_fields_t<float>(ev, F);
}

gl_status gl_set_particles(gl_event *ev, int32_t n_species, const gl_species_desc *sp, int64_t n,
                           const int32_t *cell, const double *off, const double *eta, const double *p,
                           const double *Q, const double *p0, const int32_t *species) {
    if (!sp || !cell || !off || !eta || !p || !Q || !p0 || !species) return fail(GL_EINVAL, "null argument");
    if (gl_status s = check_free(ev)) return s;
    if (n_species < 1 || n_species > kMaxSpecies || n < 1) return fail(GL_EINVAL, "bad counts");
    if (ev->push_due) return fail(GL_ESTATE, "a particle step is due");
    std::vector<int64_t> count(n_species, 0);
    for (int64_t i = 0; i < n; i++) {
        if (species[i] < 0 || species[i] >= n_species) return fail(GL_EINVAL, "species id out of range");
        if (cell[i] < 0 || cell[i] >= ev->N || cell[n + i] < 0 || cell[n + i] >= ev->N)
            return fail(GL_EINVAL, "cell out of range");
        count[species[i]]++;
    }
    std::vector<SpeciesInfo> tab;
    const int64_t used = (n + kPushBlock - 1) / kPushBlock * kPushBlock;
    for (int s = 0; s < n_species; s++) {
        SpeciesInfo si;
        gl_status st = fill_species(ev, &sp[s], si);
        if (st) return st;
        si.n = count[s];
        tab.push_back(si);
    }
    if (used > ev->L.slots) return fail(GL_ENOMEM, "particle capacity exceeded");
    ev->species = tab;
    ev->slots_used = used;
    gl_status s = ev->fp64() ? set_particles_t<double>(ev, n, cell, off, eta, p, Q, p0, species)
                             : set_particles_t<float>(ev, n, cell, off, eta, p, Q, p0, species);
    if (s) return s;
    ev->set_changed = true;
    return GL_OK;
}

gl_status gl_set_sort_period(gl_event *ev, int32_t every) {
    if (gl_status s = check_free(ev)) return s;
    if (every < 0) return fail(GL_EINVAL, "sort period must be >= 0");
    ev->sort_every = every;
    return GL_OK;
}

gl_status gl_set_graph_steps(gl_event *ev, int32_t steps) {
    if (gl_status s = check_free(ev)) return s;
    if (steps < 0) return fail(GL_EINVAL, "graph_steps must be >= 0");
    if (steps > 0 && !ev->stream) return fail(GL_EINVAL, "graph replay needs a stream other than the null stream");
    ev->graph_steps = steps;
    if (steps == 0) free_graphs(ev);
    return GL_OK;
}

gl_status gl_graph_stats(const gl_event *ev, int64_t *launches, int64_t *instantiations) {
    if (!ev || !launches || !instantiations) return fail(GL_EINVAL, "null argument");
    *launches = ev->graph_launches;
    *instantiations = ev->graph_instantiations;
    return GL_OK;
}

gl_status gl_set_check_period(gl_event *ev, int32_t every) {
    if (check_ev(ev)) return GL_EINVAL;
    if (every < 0) return fail(GL_EINVAL, "check period must be >= 0");
    ev->check_every = every;
    return GL_OK;
}

gl_status gl_set_match_params(gl_event *ev, int32_t max_iter, double tol) {
    if (gl_status s = check_free(ev)) return s;
    if (max_iter < 1 || !(tol > 0)) return fail(GL_EINVAL, "max_iter must be >= 1 and tol > 0");
    ev->match_max_iter = max_iter;
    ev->match_tol = tol;
    return GL_OK;
}

gl_status gl_get_particles(gl_event *ev, int64_t cap, int64_t *n, int32_t *cell, double *off, double *eta,
                           double *p, double *Q, double *p0, int32_t *species) {
    if (check_ev(ev) || !n) return fail(GL_EINVAL, "null argument");
    int64_t tot = total_particles(ev);
    *n = tot;
    if (!cell && !off && !eta && !p && !Q && !p0 && !species) return GL_OK;
    if (cap < tot) return fail(GL_EINVAL, "output too small");
    return ev->fp64() ? get_particles_t<double>(ev, tot, cell, off, eta, p, Q, p0, species)
                      : get_particles_t<float>(ev, tot, cell, off, eta, p, Q, p0, species);
}

gl_status gl_species_info(gl_event *ev, int32_t species, int32_t *nform, double *mass_lat) {
    if (check_ev(ev)) return GL_EINVAL;
    if (species < 0 || species >= (int32_t)ev->species.size()) return fail(GL_EINVAL, "no such species");
    if (nform) *nform = ev->species[species].nform;
    if (mass_lat) *mass_lat = ev->species[species].mass_lat;
    return GL_OK;
}

gl_status gl_get_wilson_line(gl_event *ev, int32_t nucleus, double *V) {
    if (check_ev(ev) || !V || (nucleus != 0 && nucleus != 1)) return fail(GL_EINVAL, "bad argument");
    HIP_TRY(hipMemcpyAsync(V, ev->ws + (nucleus == 0 ? ev->L.VA : ev->L.VB), 18 * ev->n2 * sizeof(double),
                           hipMemcpyDeviceToHost, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    return GL_OK;
}

gl_status gl_dipole(gl_event *ev, int32_t nucleus, int32_t rmax, double *D) {
    if (check_ev(ev) || !D || (nucleus != 0 && nucleus != 1)) return fail(GL_EINVAL, "bad argument");
    if (rmax < 1 || rmax > ev->N / 2) return fail(GL_EINVAL, "rmax must be in [1, N/2]");
    std::vector<double> d;
    gl_status s = dipole_curve(ev, nucleus, rmax, d);
    if (s) return s;
    std::copy(d.begin(), d.end(), D);
    return GL_OK;
}

gl_status gl_saturation_scale(gl_event *ev, double *qs_GeV) {
    if (check_ev(ev) || !qs_GeV) return fail(GL_EINVAL, "null argument");
    double sum = 0.0;
    for (int nuc = 0; nuc < 2; nuc++) {
        std::vector<double> d;
        gl_status s = dipole_curve(ev, nuc, ev->N / 2, d);
        if (s) return s;
        const double q = qs_from_dipole(d, ev->a_gev);
        if (!(q > 0)) return fail(GL_ENUMERIC, "dipole does not fall to exp(-1/2) within N/2 sites");
        sum += q;
    }
    *qs_GeV = 0.5 * sum;
    return GL_OK;
}

gl_status gl_calibrate_g2mu(gl_event *ev, const gl_mv_desc *mv, double qs_target_GeV, uint64_t seed,
                            int32_t n_seeds, double *g2mu_out, double *qs_out) {
    if (check_ev(ev) || !mv || !g2mu_out) return fail(GL_EINVAL, "null argument");
    if (!(qs_target_GeV > 0) || n_seeds < 1 || mv->n_sheets < 1) return fail(GL_EINVAL, "bad argument");
    double g = mv->g2mu_GeV > 0 ? mv->g2mu_GeV : qs_target_GeV / 0.6, q = 0.0;
    for (int it = 0; it < 12; it++) {
        q = 0.0;
        for (int k = 0; k < n_seeds; k++) {
            const double sigma = g * ev->a_gev / std::sqrt((double)mv->n_sheets);
            gl_status s = wilson_lines(ev, mv->n_sheets, mv->m_ir_GeV, mv->uv_cut_GeV, nullptr, sigma, seed + k);
            if (s) return s;
            double qk = 0.0;
            s = gl_saturation_scale(ev, &qk);
            if (s) return s;
            q += qk / n_seeds;
        }
        if (std::fabs(q - qs_target_GeV) <= 1e-3 * qs_target_GeV) break;
        g *= qs_target_GeV / q;   // Q_s grows about linearly with g^2 mu
    }
    *g2mu_out = g;
    if (qs_out) *qs_out = q;
    return GL_OK;
}

gl_status gl_draw_charges(gl_event *ev, uint64_t seed, int32_t nucleus, int32_t sheet, double sigma, double *rho) {
    if (check_ev(ev) || !rho || sheet < 0 || nucleus < 0) return fail(GL_EINVAL, "bad argument");
    double2 *planes = (double2 *)(ev->ws + ev->L.planes);
    double *tmp = (double *)(ev->ws + ev->L.U0);
    HIP_TRY(launch_mv_charges(ev->stream, ev->N, sigma, seed, nucleus, sheet, 1, planes));
    HIP_TRY(launch_planes_to_charges(ev->stream, ev->N, planes, tmp));
    HIP_TRY(hipMemcpyAsync(rho, tmp, 8 * ev->n2 * sizeof(double), hipMemcpyDeviceToHost, ev->stream));
    HIP_TRY(hipStreamSynchronize(ev->stream));
    return GL_OK;
}

gl_status gl_profile_enable(gl_event *ev, int32_t period) {
    if (check_ev(ev)) return GL_EINVAL;
    if (period < 0) return fail(GL_EINVAL, "profiling period must be >= 0");
    ev->prof = period;
    for (int k = 0; k < GL_PROF_KERNELS; k++) ev->prof_count[k] = 0;
    return GL_OK;
}

gl_status gl_profile_read(gl_event *ev, double *ms, int64_t *launches) {
    if (check_ev(ev) || !ms || !launches) return fail(GL_EINVAL, "null argument");
    for (int k = 0; k < GL_PROF_KERNELS; k++) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    HIP_TRY(hipStreamSynchronize(ev->stream));
    for (auto &m : ev->prof_marks) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, ev->ev_pool[m.second], ev->ev_pool[m.second + 1]));
        ms[m.first] += t;
        launches[m.first] += 1;
    }
    ev->prof_marks.clear();
    ev->ev_used = 0;
    return GL_OK;
}

gl_status gl_event_info(gl_event *ev, double *a_fm, double *dtau_lat, int64_t *n) {
    if (check_ev(ev)) return GL_EINVAL;
    if (a_fm) *a_fm = ev->a_fm;
    if (dtau_lat) *dtau_lat = ev->dtau;
    if (n) *n = ev->n;
    return GL_OK;
}

gl_status gl_sync(gl_event *ev) {
    if (check_ev(ev)) return GL_EINVAL;
    HIP_TRY(hipStreamSynchronize(ev->stream));
    return GL_OK;
}

}  // extern "C"

// ---- checkpoint / restore -----------------------------------------------------
// File: magic, format version, sizeof(gl_lattice_desc), the descriptor, the
// runtime scalars, the species table, then tagged device blobs (tag, bytes,
// raw device bytes).  The blob list follows from the descriptor and the
// scalars, so a restore rebuilds it after reading them and checks each tag
// and size.  Raw device bytes in the device order keep the resumed run
// bitwise identical (the reductions follow the particles' slots).
namespace {

const char kCkptMagic[8] = {'G', 'L', 'C', 'K', 'P', 'T', '0', '1'};
constexpr uint32_t kCkptVersion = 1;

struct CkptScalars {
    int64_t n, rows, slots_used, since_sort, stat_n0, stat_rows, ll_n0, ll_rows;
    int32_t cur, pbuf, push_due, set_changed, sort_every, stat_on, ll_on, match_max_iter, check_every, n_species;
    double match_tol;
};

struct CkptSpecies {
    gl_species_desc desc;
    int64_t n;
    int32_t nform, pad;
    double mass_lat, p0_lat, tau_form_fm;
};

struct Blob {
    uint64_t tag;
    char *dev;
    size_t bytes;
};

std::vector<Blob> ckpt_blobs(gl_event *ev) {
    const size_t ts = ev->fp64() ? 8 : 4, n2 = ev->n2, row = (size_t)kMaxSpecies * 4 * sizeof(double);
    std::vector<Blob> b;
    b.push_back({1, ev->ws + ev->L.field[ev->cur], (size_t)kStateVals * n2 * ts});
    if (ev->push_due) {
        // the pending push reads the site fields and the state at tau_n (links
        // for the crossings, phi for the eta rotation), the other buffer
        b.push_back({2, ev->ws + ev->L.F, (size_t)kSiteRec * n2 * ts});
        b.push_back({11, ev->ws + ev->L.field[1 - ev->cur], (size_t)kStateVals * n2 * ts});
    }
    if (ev->L.slots > 0) {
        b.push_back({3, ev->ws + ev->L.part[ev->pbuf], (size_t)ev->L.slots * ((part_rec(ts) + 3) * ts + 12)});
        b.push_back({4, (char *)ev->ids(), (size_t)ev->L.slots * sizeof(int32_t)});
    }
    b.push_back({5, (char *)ev->series(), (size_t)ev->rows * row});
    b.push_back({6, (char *)ev->p0sum(), row});
    if (ev->stat_on) {
        b.push_back({7, ev->ws + ev->L.stat, 24 * n2 * sizeof(double)});
        b.push_back({8, (char *)ev->stat_series(), (size_t)ev->stat_rows * row});
    }
    if (ev->ll_on) {
        b.push_back({9, ev->ws + ev->L.ll, 42 * n2 * sizeof(double)});
        b.push_back({10, (char *)ev->ll_series(), (size_t)ev->ll_rows * row});
    }
    return b;
}

struct FileCloser {
    std::FILE *f;
    ~FileCloser() {
        if (f) std::fclose(f);
    }
};

bool same_desc(const gl_lattice_desc &a, const gl_lattice_desc &b) {
    return a.N == b.N && a.L_fm == b.L_fm && a.dtau_over_a == b.dtau_over_a && a.precision == b.precision &&
           a.reunit_every == b.reunit_every && a.max_steps == b.max_steps && a.max_particles == b.max_particles &&
           a.static_correlator == b.static_correlator && a.lightlike_correlator == b.lightlike_correlator;
}

}  // namespace

extern "C" {

gl_status gl_checkpoint(gl_event *ev, const char *path) {
    if (check_ev(ev) || !path) return fail(GL_EINVAL, "null argument");
    if (!ev->ready) return fail(GL_ESTATE, "fields not initialised");
    if (ev->pend != 0 || ev->perm_pending) return fail(GL_ESTATE, "the event has deferred device work pending");
    FileCloser fc{std::fopen(path, "wb")};
    if (!fc.f) return fail(GL_EINVAL, std::string("cannot open ") + path + " for writing");
    CkptScalars c{};
    c.n = ev->n;
    c.rows = ev->rows;
    c.slots_used = ev->slots_used;
    c.since_sort = ev->since_sort;
    c.stat_n0 = ev->stat_n0;
    c.stat_rows = ev->stat_rows;
    c.ll_n0 = ev->ll_n0;
    c.ll_rows = ev->ll_rows;
    c.cur = ev->cur;
    c.pbuf = ev->pbuf;
    c.push_due = ev->push_due;
    c.set_changed = ev->set_changed;
    c.sort_every = ev->sort_every;
    c.stat_on = ev->stat_on;
    c.ll_on = ev->ll_on;
    c.match_max_iter = ev->match_max_iter;
    c.check_every = ev->check_every;
    c.n_species = (int32_t)ev->species.size();
    c.match_tol = ev->match_tol;
    std::vector<CkptSpecies> sp(ev->species.size());
    for (size_t k = 0; k < sp.size(); k++) {
        const SpeciesInfo &si = ev->species[k];
        sp[k] = CkptSpecies{si.desc, si.n, si.nform, 0, si.mass_lat, si.p0_lat, si.tau_form_fm};
    }
    const uint32_t head[2] = {kCkptVersion, (uint32_t)sizeof(gl_lattice_desc)};
    bool ok = std::fwrite(kCkptMagic, 1, 8, fc.f) == 8 && std::fwrite(head, sizeof(head), 1, fc.f) == 1 &&
              std::fwrite(&ev->desc, sizeof(ev->desc), 1, fc.f) == 1 && std::fwrite(&c, sizeof(c), 1, fc.f) == 1 &&
              (sp.empty() || std::fwrite(sp.data(), sizeof(CkptSpecies), sp.size(), fc.f) == sp.size());
    std::vector<char> host;
    for (const Blob &b : ckpt_blobs(ev)) {
        if (!ok) break;
        host.resize(b.bytes);
        if (b.bytes) {
            HIP_TRY(hipMemcpyAsync(host.data(), b.dev, b.bytes, hipMemcpyDeviceToHost, ev->stream));
            HIP_TRY(hipStreamSynchronize(ev->stream));
        }
        const uint64_t hb[2] = {b.tag, (uint64_t)b.bytes};
        ok = std::fwrite(hb, sizeof(hb), 1, fc.f) == 1 && (b.bytes == 0 || std::fwrite(host.data(), 1, b.bytes, fc.f) == b.bytes);
    }
    if (!ok || std::fflush(fc.f) != 0) return fail(GL_EINVAL, std::string("write to ") + path + " failed");
    return GL_OK;
}

gl_status gl_restore(gl_event *ev, const char *path) {
    if (!path) return fail(GL_EINVAL, "null argument");
    if (gl_status s = check_free(ev)) return s;
    FileCloser fc{std::fopen(path, "rb")};
    if (!fc.f) return fail(GL_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    uint32_t head[2];
    gl_lattice_desc d;
    CkptScalars c;
    if (std::fread(magic, 1, 8, fc.f) != 8 || std::memcmp(magic, kCkptMagic, 8) != 0 ||
        std::fread(head, sizeof(head), 1, fc.f) != 1 || head[0] != kCkptVersion ||
        head[1] != sizeof(gl_lattice_desc) || std::fread(&d, sizeof(d), 1, fc.f) != 1 ||
        std::fread(&c, sizeof(c), 1, fc.f) != 1)
        return fail(GL_EINVAL, std::string(path) + " is not a checkpoint of this format");
    if (!same_desc(d, ev->desc)) return fail(GL_EINVAL, "the checkpoint's lattice description differs from the event's");
    if (c.n_species < 0 || c.n_species > kMaxSpecies || c.cur < 0 || c.cur > 1 || c.pbuf < 0 || c.pbuf > 1 ||
        c.rows < 0 || c.rows > std::max(0, d.max_steps) || c.stat_rows < 0 || c.stat_rows > std::max(0, d.max_steps) ||
        c.ll_rows < 0 || c.ll_rows > std::max(0, d.max_steps) || c.slots_used < 0 || c.slots_used > ev->L.slots ||
        (c.stat_on && !d.static_correlator) || (c.ll_on && !d.lightlike_correlator) || c.n < 0 ||
        c.since_sort < 0 || c.sort_every < 0 || c.check_every < 0 || c.match_max_iter < 1 || !(c.match_tol > 0) ||
        c.stat_n0 < 0 || c.ll_n0 < 0 || (c.push_due != 0 && c.push_due != 1) || (c.set_changed != 0 && c.set_changed != 1))
        return fail(GL_EINVAL, std::string(path) + ": inconsistent checkpoint");
    std::vector<CkptSpecies> sp(c.n_species);
    if (!sp.empty() && std::fread(sp.data(), sizeof(CkptSpecies), sp.size(), fc.f) != sp.size())
        return fail(GL_EINVAL, std::string(path) + " is truncated");
    // the particles fill [0, total) of whole push blocks, species by species
    int64_t total = 0;
    for (const CkptSpecies &k : sp) {
        if (k.n < 0 || k.n > ev->L.slots || k.nform < 1 || !(k.mass_lat >= 0) ||
            (k.desc.kind != GL_KIND_HEAVY_QUARK && k.desc.kind != GL_KIND_JET))
            return fail(GL_EINVAL, std::string(path) + ": inconsistent species record");
        total += k.n;
    }
    if ((total + kPushBlock - 1) / kPushBlock * kPushBlock != c.slots_used)
        return fail(GL_EINVAL, std::string(path) + ": species counts do not fill the used slots");
    // the event takes the checkpoint's scalars, then its blobs
    ev->n = c.n;
    ev->rows = c.rows;
    ev->slots_used = c.slots_used;
    ev->since_sort = c.since_sort;
    ev->stat_n0 = c.stat_n0;
    ev->stat_rows = c.stat_rows;
    ev->ll_n0 = c.ll_n0;
    ev->ll_rows = c.ll_rows;
    ev->cur = c.cur;
    ev->pbuf = c.pbuf;
    ev->push_due = c.push_due != 0;
    ev->set_changed = c.set_changed != 0;
    ev->sort_every = c.sort_every;
    ev->stat_on = c.stat_on != 0;
    ev->ll_on = c.ll_on != 0;
    ev->match_max_iter = c.match_max_iter;
    ev->match_tol = c.match_tol;
    ev->check_every = c.check_every;
    ev->pend = 0;
    ev->pend_row0 = 0;
    ev->perm_pending = false;
    ev->ready = false;   // until every blob is in
    ev->species.clear();
    for (const CkptSpecies &k : sp) {
        SpeciesInfo si;
        si.desc = k.desc;
        si.n = k.n;
        si.nform = k.nform;
        si.mass_lat = k.mass_lat;
        si.p0_lat = k.p0_lat;
        si.tau_form_fm = k.tau_form_fm;
        ev->species.push_back(si);
    }
    // series rows past the saved ones read as zero, as in a fresh run
    const size_t row = (size_t)kMaxSpecies * 4 * sizeof(double), cap_rows = (size_t)std::max(1, d.max_steps);
    HIP_TRY(hipMemsetAsync(ev->series(), 0, cap_rows * row, ev->stream));
    if (d.static_correlator) HIP_TRY(hipMemsetAsync(ev->stat_series(), 0, cap_rows * row, ev->stream));
    if (d.lightlike_correlator) HIP_TRY(hipMemsetAsync(ev->ll_series(), 0, cap_rows * row, ev->stream));
    std::vector<char> host;
    for (const Blob &b : ckpt_blobs(ev)) {
        uint64_t hb[2];
        if (std::fread(hb, sizeof(hb), 1, fc.f) != 1 || hb[0] != b.tag || hb[1] != b.bytes)
            return fail(GL_EINVAL, std::string(path) + ": unexpected section");
        host.resize(b.bytes);
        if (b.bytes == 0) continue;
        if (std::fread(host.data(), 1, b.bytes, fc.f) != b.bytes) return fail(GL_EINVAL, std::string(path) + " is truncated");
        HIP_TRY(hipMemcpyAsync(b.dev, host.data(), b.bytes, hipMemcpyHostToDevice, ev->stream));
        HIP_TRY(hipStreamSynchronize(ev->stream));
    }
    ev->ready = true;
    return GL_OK;
}

}  // extern "C"

// ============================================================================
// Batches: many events stepped in lock-step by the flattened kernels of
// batch_kernels.hip, the step loop captured once into a hipGraph.
#include <fstream>
#include <map>
#include <sstream>

#include "batch_internal.hpp"

struct gl_batch {
    std::vector<gl_event *> evs;
    std::vector<int> cur0, pbuf0;      // event buffers that parity 0 maps to
    bool fp64 = true;
    double dtau = 0.125;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t desc = 0, tiles[kBatchShapes] = {0, 0, 0}, pblocks = 0, stiles = 0, ctl = 0, fail = 0, checks = 0;
    int64_t total_tiles[kBatchShapes] = {0, 0, 0}, total_pblocks = 0, total_stiles = 0, total_checks = 0;
    int shape = 0, grid_mult = 4, cus = 256;
    int fpar = 0, ppar = 0;
    int64_t since_sort = 0;
    bool sort_pending = false;        // a sorted order waits in the events' scratch; the next push applies it
    int sort_every = 16;
    int graph_steps = 32;             // two sort periods
    bool any_particles = false;
    // captured step loops, keyed by the state they start from, with the
    // state they leave (the parities and the pending sort)
    struct Graph {
        hipGraphExec_t exec = nullptr;
        hipGraph_t def = nullptr;
        int fpar = 0, ppar = 0;
        int64_t since_sort = 0;   // steps since the last sort at the end, if the graph sorts
        bool sorts = false;       // else the count just grows by graph_steps
        bool sort_pending = false;
    };
    std::map<int, Graph> graphs;
};

namespace {

struct BatchSizes {
    size_t desc, tiles[kBatchShapes], pblocks, stiles, ctl, fail, checks, total;
    int64_t n_tiles[kBatchShapes], n_pblocks, n_stiles, n_checks;
};

// (event, chunk) entries of the finite-value check over the events' states
int64_t check_chunks(const gl_event *ev) { return ((int64_t)kStateVals * ev->n2 + kCheckChunk - 1) / kCheckChunk; }

const int kShapeTX[kBatchShapes] = {32, 64, 16}, kShapeTY[kBatchShapes] = {4, 2, 8};

gl_status batch_sizes(gl_event *const *evs, int n, BatchSizes &z) {
    if (!evs || n < 1) return fail(GL_EINVAL, "empty batch");
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off = align256(off + b);
        return o;
    };
    z.desc = take((size_t)n * std::max(sizeof(BatchEv<double>), sizeof(BatchEv<float>)));
    for (int s = 0; s < kBatchShapes; s++) {
        z.n_tiles[s] = 0;
        for (int e = 0; e < n; e++) {
            if (!evs[e]) return fail(GL_EINVAL, "null event in batch");
            int N = evs[e]->N;
            z.n_tiles[s] += (int64_t)((N + kShapeTX[s] - 1) / kShapeTX[s]) * ((N + kShapeTY[s] - 1) / kShapeTY[s]);
        }
        z.tiles[s] = take((size_t)z.n_tiles[s] * sizeof(int2));
    }
    z.n_pblocks = 0;
    for (int e = 0; e < n; e++) z.n_pblocks += evs[e]->L.slots / kPushBlock;
    z.pblocks = take((size_t)std::max<int64_t>(1, z.n_pblocks) * sizeof(int2));
    z.n_stiles = 0;
    for (int e = 0; e < n; e++) z.n_stiles += evs[e]->slots_used > 0 ? sort_tiles(evs[e]->slots_used) : 0;
    z.stiles = take((size_t)std::max<int64_t>(1, z.n_stiles) * sizeof(int2));
    z.ctl = take(sizeof(BatchCtl));
    z.fail = take((size_t)n * sizeof(int32_t));
    z.n_checks = 0;
    for (int e = 0; e < n; e++) z.n_checks += check_chunks(evs[e]);
    z.checks = take((size_t)z.n_checks * sizeof(int2));
    z.total = off;
    return GL_OK;
}

template <typename T>
BatchEv<T> batch_desc(const gl_batch *b, int e) {
    gl_event *ev = b->evs[e];
    BatchEv<T> d;
    d.N = ev->N;
    d.reunit_every = ev->fp64() ? 0 : ev->desc.reunit_every;
    d.n_species = (int)ev->species.size();
    d.max_steps = ev->desc.max_steps;
    d.n_slots = ev->slots_used;
    d.f[0] = ev->fields<T>(b->cur0[e]);
    d.f[1] = ev->fields<T>(1 - b->cur0[e]);
    d.P[0] = ev->parts<T>(b->pbuf0[e]);
    d.P[1] = ev->parts<T>(1 - b->pbuf0[e]);
    d.F = (T *)(ev->ws + ev->L.F);
    d.partials = ev->partials();
    d.p0sum = ev->p0sum();
    d.series = ev->series();
    d.tab = ev->tab<T>();
    d.sort = ev->scratch();
    d.sort_tiles = ev->slots_used > 0 ? sort_tiles(ev->slots_used) : 0;
    d.ids[0] = ev->ids(b->pbuf0[e]);
    d.ids[1] = ev->ids(1 - b->pbuf0[e]);
    d.fail = (int32_t *)(b->ws + b->fail) + e;
    return d;
}

template <typename T>
gl_status batch_step(gl_batch *b) {
    const int grid = b->grid_mult > 0 ? b->grid_mult * b->cus : 0;
    const BatchEv<T> *d = (const BatchEv<T> *)(b->ws + b->desc);
    const BatchCtl *ctl = (const BatchCtl *)(b->ws + b->ctl);
    HIP_TRY(launch_batch_fields<T>(b->stream, b->shape, d, (const int2 *)(b->ws + b->tiles[b->shape]),
                                   b->total_tiles[b->shape], b->fpar, ctl, b->dtau, grid));
    // a pending sort is applied by this push, which moves the particles to the other buffer
    HIP_TRY(launch_batch_push<T>(b->stream, d, (const int2 *)(b->ws + b->pblocks), b->total_pblocks, b->fpar,
                                 b->ppar, ctl, b->dtau, grid, (int)b->evs.size(), b->sort_pending));
    if (b->sort_pending) b->ppar ^= 1;
    b->sort_pending = false;
    b->fpar ^= 1;
    b->since_sort++;
    if (b->any_particles && b->sort_every > 0 && b->since_sort >= b->sort_every) {
        HIP_TRY(launch_batch_sort<T>(b->stream, d, (int)b->evs.size(), (const int2 *)(b->ws + b->pblocks),
                                     b->total_pblocks, (const int2 *)(b->ws + b->stiles), b->total_stiles, b->ppar,
                                     false));
        b->sort_pending = true;
        b->since_sort = 0;
    }
    return GL_OK;
}

// a pending sort applied alone (the particles move to the other buffer), so
// that none is left when a run returns
template <typename T>
gl_status batch_apply_pending(gl_batch *b) {
    if (!b->sort_pending) return GL_OK;
    const BatchEv<T> *d = (const BatchEv<T> *)(b->ws + b->desc);
    HIP_TRY(launch_batch_permute<T>(b->stream, d, (const int2 *)(b->ws + b->pblocks), b->total_pblocks, b->ppar));
    b->ppar ^= 1;
    b->sort_pending = false;
    return GL_OK;
}

gl_status batch_step_any(gl_batch *b) { return b->fp64 ? batch_step<double>(b) : batch_step<float>(b); }

// the batch's graphs, after the stream has finished with them (a launch may
// still be in flight when the batch is reconfigured or destroyed)
void batch_drop_graphs(gl_batch *b) {
    if (!b->graphs.empty()) (void)hipStreamSynchronize(b->stream);
    for (auto &g : b->graphs) {
        (void)hipGraphExecDestroy(g.second.exec);
        (void)hipGraphDestroy(g.second.def);
    }
    b->graphs.clear();
}

// capture graph_steps steps starting at a sort boundary from the batch's
// state (parities, pending sort); the graph records the state it leaves
gl_status batch_graph(gl_batch *b, const gl_batch::Graph **out) {
    const int key = (b->fpar * 2 + b->ppar) * 2 + (b->sort_pending ? 1 : 0);
    auto it = b->graphs.find(key);
    if (it != b->graphs.end()) {
        *out = &it->second;
        return GL_OK;
    }
    const int f0 = b->fpar, p0 = b->ppar;
    const int64_t s0 = b->since_sort;
    const bool q0 = b->sort_pending;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
    gl_status st = GL_OK;
    for (int k = 0; k < b->graph_steps && st == GL_OK; k++) st = batch_step_any(b);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    gl_batch::Graph rec;
    rec.fpar = b->fpar;
    rec.ppar = b->ppar;
    rec.since_sort = b->since_sort;
    rec.sorts = b->since_sort != s0 + b->graph_steps;
    rec.sort_pending = b->sort_pending;
    // capturing ran nothing: the batch is still where it started
    b->fpar = f0;
    b->ppar = p0;
    b->since_sort = s0;
    b->sort_pending = q0;
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(GL_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(GL_EDEVICE, "hipGraphInstantiate failed");
    }
    rec.exec = x;
    rec.def = g;
    *out = &(b->graphs[key] = rec);
    return GL_OK;
}

std::string batch_key(const gl_batch *b) {
    std::vector<int> Ns;
    int64_t parts = 0;
    for (auto *ev : b->evs) {
        Ns.push_back(ev->N);
        parts += total_particles(ev);
    }
    std::sort(Ns.begin(), Ns.end());
    std::ostringstream k;
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "gpu";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    k << arch << "|p" << (b->fp64 ? 64 : 32) << "|N";
    for (int N : Ns) k << "," << N;
    k << "|parts" << parts;
    return k.str();
}

// the largest grid multiple the tuner tries (workgroups per CU of a persistent launch)
constexpr int kMaxGridMult = 8;

bool cache_lookup(const char *path, const std::string &key, int *shape, int *mult) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    std::string s = ss.str(), pat = "\"" + key + "\": [";
    size_t p = s.find(pat);
    if (p == std::string::npos) return false;
    // an entry out of the tuner's own range is ignored (the batch is timed again)
    return std::sscanf(s.c_str() + p + pat.size(), "%d, %d", shape, mult) == 2 && *shape >= 0 &&
           *shape < kBatchShapes && *mult >= 0 && *mult <= kMaxGridMult;
}

void cache_store(const char *path, const std::string &key, int shape, int mult) {
    if (!path) return;
    std::map<std::string, std::pair<int, int>> entries;
    std::ifstream f(path);
    if (f) {
        std::string line;
        while (std::getline(f, line)) {
            size_t a = line.find('"'), bq = line.find("\": [");
            if (a == std::string::npos || bq == std::string::npos) continue;
            int s = 0, m = 0;
            if (std::sscanf(line.c_str() + bq + 4, "%d, %d", &s, &m) == 2) entries[line.substr(a + 1, bq - a - 1)] = {s, m};
        }
    }
    entries[key] = {shape, mult};
    std::ofstream o(path);
    o << "{\n";
    size_t i = 0;
    for (auto &kv : entries)
        o << "  \"" << kv.first << "\": [" << kv.second.first << ", " << kv.second.second << "]"
          << (++i < entries.size() ? "," : "") << "\n";
    o << "}\n";
}

template <typename T>
gl_status time_fields(gl_batch *b, int shape, int mult, float *ms) {
    const int grid = mult > 0 ? mult * b->cus : 0;
    const BatchEv<T> *d = (const BatchEv<T> *)(b->ws + b->desc);
    const BatchCtl *ctl = (const BatchCtl *)(b->ws + b->ctl);
    const int2 *tiles = (const int2 *)(b->ws + b->tiles[shape]);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // the field phases read the state at parity fpar and only write the
    // next-step buffer and the site fields: repeating them changes nothing
    HIP_TRY(launch_batch_fields<T>(b->stream, shape, d, tiles, b->total_tiles[shape], b->fpar, ctl, b->dtau, grid));
    HIP_TRY(hipEventRecord(e0, b->stream));
    const int reps = 3;
    for (int r = 0; r < reps; r++)
        HIP_TRY(launch_batch_fields<T>(b->stream, shape, d, tiles, b->total_tiles[shape], b->fpar, ctl, b->dtau,
                                       grid));
    HIP_TRY(hipEventRecord(e1, b->stream));
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    *ms /= reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return GL_OK;
}

// order the batch stream after the events' own streams (and the reverse at the end)
gl_status batch_fence(gl_batch *b) {
    for (auto *ev : b->evs)
        if (ev->stream != b->stream) HIP_TRY(hipStreamSynchronize(ev->stream));
    return GL_OK;
}

void batch_sync_events(gl_batch *b, int64_t steps) {
    for (size_t e = 0; e < b->evs.size(); e++) {
        gl_event *ev = b->evs[e];
        ev->cur = b->cur0[e] ^ b->fpar;
        ev->pbuf = b->pbuf0[e] ^ b->ppar;
        ev->n += steps;
        if (ev->slots_used > 0) ev->rows = std::max<int64_t>(ev->rows, std::min<int64_t>(ev->n - 1, ev->desc.max_steps));
        ev->since_sort = b->since_sort;
        ev->push_due = false;
    }
}

}  // namespace

extern "C" {

gl_status gl_batch_required_bytes(gl_event *const *evs, int32_t n_events, size_t *bytes) {
    if (!bytes) return fail(GL_EINVAL, "null output");
    BatchSizes z;
    gl_status s = batch_sizes(evs, n_events, z);
    if (s) return s;
    *bytes = z.total;
    return GL_OK;
}

gl_status gl_batch_create(gl_event *const *evs, int32_t n_events, void *workspace, size_t bytes, void *stream,
                          gl_batch **out) {
    if (!out) return fail(GL_EINVAL, "null output");
    *out = nullptr;
    BatchSizes z;
    gl_status s = batch_sizes(evs, n_events, z);
    if (s) return s;
    if (!workspace || ((uintptr_t)workspace & 255)) return fail(GL_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < z.total) return fail(GL_ENOMEM, "workspace smaller than gl_batch_required_bytes()");
    gl_event *e0 = evs[0];
    for (int e = 0; e < n_events; e++) {
        gl_event *ev = evs[e];
        if (!ev->ready) return fail(GL_ESTATE, "every event must be initialised");
        if (ev->push_due) return fail(GL_ESTATE, "an event has a particle step due");
        if (ev->owner) return fail(GL_ESTATE, "an event is already held by another batch");
        if (ev->desc.precision != e0->desc.precision || ev->dtau != e0->dtau || ev->n != e0->n)
            return fail(GL_EINVAL, "events of a batch share precision, dtau and the step index");
        for (int f = 0; f < e; f++)
            if (evs[f] == ev) return fail(GL_EINVAL, "an event appears twice");
    }
    gl_batch *b = new (std::nothrow) gl_batch();
    if (!b) return fail(GL_ENOMEM, "host allocation failed");
    b->evs.assign(evs, evs + n_events);
    b->fp64 = e0->fp64();
    b->dtau = e0->dtau;
    b->stream = (hipStream_t)stream;
    b->ws = (char *)workspace;
    b->desc = z.desc;
    for (int k = 0; k < kBatchShapes; k++) {
        b->tiles[k] = z.tiles[k];
        b->total_tiles[k] = z.n_tiles[k];
    }
    b->pblocks = z.pblocks;
    b->stiles = z.stiles;
    b->ctl = z.ctl;
    b->fail = z.fail;
    b->checks = z.checks;
    b->total_checks = z.n_checks;
    for (auto *ev : b->evs) {
        // the batch reads each event's current particle buffer and formation
        // sums: take a pending sort first (on the event's stream; the batch
        // runs after those streams)
        gl_status st = settle_particles(ev);
        if (st) {
            delete b;
            return st;
        }
        b->cur0.push_back(ev->cur);
        b->pbuf0.push_back(ev->pbuf);
        b->any_particles |= ev->slots_used > 0;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        b->cus = cus;
    // descriptors and work tables
    std::vector<char> dbuf((size_t)n_events * std::max(sizeof(BatchEv<double>), sizeof(BatchEv<float>)));
    for (int e = 0; e < n_events; e++) {
        if (b->fp64) ((BatchEv<double> *)dbuf.data())[e] = batch_desc<double>(b, e);
        else ((BatchEv<float> *)dbuf.data())[e] = batch_desc<float>(b, e);
    }
    auto cleanup = [&](gl_status st) {
        delete b;
        return st;
    };
    if (hipMemcpyAsync(b->ws + b->desc, dbuf.data(), dbuf.size(), hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return cleanup(fail(GL_EDEVICE, "descriptor upload failed"));
    for (int k = 0; k < kBatchShapes; k++) {
        std::vector<int2> t;
        for (int e = 0; e < n_events; e++) {
            int N = evs[e]->N, nt = ((N + kShapeTX[k] - 1) / kShapeTX[k]) * ((N + kShapeTY[k] - 1) / kShapeTY[k]);
            for (int j = 0; j < nt; j++) t.push_back(make_int2(e, j));
        }
        if (!t.empty() && hipMemcpyAsync(b->ws + b->tiles[k], t.data(), t.size() * sizeof(int2),
                                         hipMemcpyHostToDevice, b->stream) != hipSuccess)
            return cleanup(fail(GL_EDEVICE, "tile table upload failed"));
        if (hipStreamSynchronize(b->stream) != hipSuccess) return cleanup(fail(GL_EDEVICE, "sync failed"));
    }
    std::vector<int2> pb;
    for (int e = 0; e < n_events; e++)
        for (int64_t j = 0; j < evs[e]->slots_used / kPushBlock; j++) pb.push_back(make_int2(e, (int)j));
    b->total_pblocks = (int64_t)pb.size();
    std::vector<int2> stl;
    for (int e = 0; e < n_events; e++)
        if (evs[e]->slots_used > 0)
            for (int64_t j = 0; j < sort_tiles(evs[e]->slots_used); j++) stl.push_back(make_int2(e, (int)j));
    b->total_stiles = (int64_t)stl.size();
    if (!stl.empty() && hipMemcpyAsync(b->ws + b->stiles, stl.data(), stl.size() * sizeof(int2), hipMemcpyHostToDevice,
                                       b->stream) != hipSuccess)
        return cleanup(fail(GL_EDEVICE, "sort table upload failed"));
    std::vector<int2> chk;
    for (int e = 0; e < n_events; e++)
        for (int64_t j = 0; j < check_chunks(evs[e]); j++) chk.push_back(make_int2(e, (int)j));
    if (hipMemsetAsync(b->ws + b->fail, 0x7F, (size_t)n_events * sizeof(int32_t), b->stream) != hipSuccess ||
        hipMemcpyAsync(b->ws + b->checks, chk.data(), chk.size() * sizeof(int2), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess)
        return cleanup(fail(GL_EDEVICE, "failure table upload failed"));
    BatchCtl c;
    c.n = e0->n;
    if ((!pb.empty() && hipMemcpyAsync(b->ws + b->pblocks, pb.data(), pb.size() * sizeof(int2), hipMemcpyHostToDevice,
                                       b->stream) != hipSuccess) ||
        hipMemcpyAsync(b->ws + b->ctl, &c, sizeof(c), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return cleanup(fail(GL_EDEVICE, "table upload failed"));
    for (auto *ev : b->evs) ev->owner = b;
    *out = b;
    return GL_OK;
}

void gl_batch_destroy(gl_batch *b) {
    if (!b) return;
    batch_drop_graphs(b);
    for (auto *ev : b->evs)
        if (ev->owner == b) ev->owner = nullptr;
    delete b;
}

gl_status gl_batch_autotune(gl_batch *b, const char *cache_json) {
    if (!b) return fail(GL_EINVAL, "null batch");
    gl_status fs = batch_fence(b);
    if (fs) return fs;
    std::string key = batch_key(b);
    int shape = 0, mult = 0;
    if (!cache_lookup(cache_json, key, &shape, &mult)) {
        float best = 1e30f;
        const int mults[] = {0, 2, 4, 8};
        for (int s = 0; s < kBatchShapes; s++)
            for (int m : mults) {
                float ms = 0;
                gl_status st = b->fp64 ? time_fields<double>(b, s, m, &ms) : time_fields<float>(b, s, m, &ms);
                if (st) return st;
                if (ms < best) {
                    best = ms;
                    shape = s;
                    mult = m;
                }
            }
        cache_store(cache_json, key, shape, mult);
    }
    if (shape != b->shape || mult != b->grid_mult) batch_drop_graphs(b);
    b->shape = shape;
    b->grid_mult = mult;
    return GL_OK;
}

gl_status gl_batch_config(gl_batch *b, int32_t shape, int32_t grid_mult, int32_t sort_every, int32_t graph_steps) {
    if (!b) return fail(GL_EINVAL, "null batch");
    if (shape < 0 || shape >= kBatchShapes || grid_mult < 0 || grid_mult > 64 || sort_every < 0 || graph_steps < 0)
        return fail(GL_EINVAL, "bad batch configuration");
    if (graph_steps > 0 && sort_every > 0 && graph_steps % (2 * sort_every) != 0)
        return fail(GL_EINVAL, "graph_steps must be a multiple of 2*sort_every");
    if (graph_steps > 0 && graph_steps % 2 != 0) return fail(GL_EINVAL, "graph_steps must be even");
    batch_drop_graphs(b);
    b->shape = shape;
    b->grid_mult = grid_mult;
    b->sort_every = sort_every;
    b->graph_steps = graph_steps;
    return GL_OK;
}

gl_status gl_batch_info(gl_batch *b, int32_t *shape, int32_t *tile_x, int32_t *tile_y, int32_t *grid_mult,
                        int32_t *graph_steps) {
    if (!b) return fail(GL_EINVAL, "null batch");
    if (shape) *shape = b->shape;
    if (tile_x) *tile_x = kShapeTX[b->shape];
    if (tile_y) *tile_y = kShapeTY[b->shape];
    if (grid_mult) *grid_mult = b->grid_mult;
    if (graph_steps) *graph_steps = b->graph_steps;
    return GL_OK;
}

gl_status gl_batch_run(gl_batch *b, int32_t n_steps) {
    if (!b) return fail(GL_EINVAL, "null batch");
    if (n_steps < 0) return fail(GL_EINVAL, "n_steps must be >= 0");
    for (auto *ev : b->evs)
        if (ev->slots_used > 0 && ev->n - 1 + n_steps > ev->desc.max_steps)
            return fail(GL_EINVAL, "series capacity (max_steps) too small for this run");
    gl_status fs = batch_fence(b);
    if (fs) return fs;
    int64_t left = n_steps;
    while (left > 0) {
        bool aligned = b->since_sort == 0 || !b->any_particles || b->sort_every == 0;
        if (b->graph_steps > 0 && aligned && left >= b->graph_steps) {
            const gl_batch::Graph *g = nullptr;
            gl_status s = batch_graph(b, &g);
            if (s) return s;
            HIP_TRY(hipGraphLaunch(g->exec, b->stream));
            b->fpar = g->fpar;
            b->ppar = g->ppar;
            b->since_sort = g->sorts ? g->since_sort : b->since_sort + b->graph_steps;
            b->sort_pending = g->sort_pending;
            left -= b->graph_steps;
            continue;
        }
        gl_status s = batch_step_any(b);
        if (s) return s;
        left--;
    }
    // no sort is left pending when the run returns
    gl_status ap = b->fp64 ? batch_apply_pending<double>(b) : batch_apply_pending<float>(b);
    if (ap) return ap;
    batch_sync_events(b, n_steps);
    // the events' states, checked once per call (their series every step)
    const BatchCtl *ctl = (const BatchCtl *)(b->ws + b->ctl);
    if (b->fp64)
        HIP_TRY(launch_batch_check<double>(b->stream, (const BatchEv<double> *)(b->ws + b->desc),
                                           (const int2 *)(b->ws + b->checks), b->total_checks, b->fpar, ctl));
    else
        HIP_TRY(launch_batch_check<float>(b->stream, (const BatchEv<float> *)(b->ws + b->desc),
                                          (const int2 *)(b->ws + b->checks), b->total_checks, b->fpar, ctl));
    std::vector<int32_t> f(b->evs.size());
    HIP_TRY(hipMemcpyAsync(f.data(), b->ws + b->fail, f.size() * sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    std::string bad;
    for (size_t e = 0; e < f.size(); e++)
        if (f[e] != kNotFailed) bad += (bad.empty() ? "" : ", ") + std::to_string(e) + " at step " + std::to_string(f[e]);
    if (!bad.empty())
        return fail(GL_ENUMERIC, "non-finite values in batch event(s) " + bad +
                                     " (masked from that step on; gl_batch_status lists them)");
    return GL_OK;
}

gl_status gl_batch_status(gl_batch *b, int32_t *fail_step) {
    if (!b || !fail_step) return fail(GL_EINVAL, "null argument");
    std::vector<int32_t> f(b->evs.size());
    HIP_TRY(hipMemcpyAsync(f.data(), b->ws + b->fail, f.size() * sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (size_t e = 0; e < f.size(); e++) fail_step[e] = f[e] == kNotFailed ? -1 : f[e];
    return GL_OK;
}

}  // extern "C"
