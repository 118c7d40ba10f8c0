// batch_kernels.hip -- many events of uneven lattice and ensemble size in one
// launch per phase.  Work is flattened over events: the field phases walk a
// table of (event, tile) entries, the push a table of (event, particle block)
// entries.  Kernels are persistent: a grid sized to the chip walks its table
// with a stride, and the table is split into eight contiguous chunks, one per
// XCD (workgroup b runs on XCD b mod 8), so that neighbouring tiles of one
// lattice share an XCD's L2.  The step index lives in device memory (the
// batch control block), so one captured hipGraph of the step loop can be
// replayed without changing kernel arguments.
#include "batch_internal.hpp"
#include "fields_dev.hpp"
#include "push_dev.hpp"

namespace gl {

// First entry, stride and end of workgroup b's walk: the table is cut into
// nx = 8 contiguous chunks; chunk x is shared by the workgroups b = x mod 8
// (there are per = ceil((g - x) / 8) of them, j = b / 8 numbers them), so
// every entry is visited by exactly one workgroup for any grid size g.
__device__ __forceinline__ int64_t xcd_first(int64_t total, int64_t &stride, int64_t &end) {
    const int64_t g = gridDim.x, b = blockIdx.x;
    const int64_t nx = g >= 8 ? 8 : 1;
    const int64_t x = b % nx, j = b / nx, per = (g - x + nx - 1) / nx;
    const int64_t chunk = (total + nx - 1) / nx;
    const int64_t lo = x * chunk;
    end = lo + chunk < total ? lo + chunk : total;
    stride = per;
    return lo + j;
}

// one tile of an event: stage its links and phi, then the step of its sites
template <typename T, int TX, int TY>
__device__ __forceinline__ void batch_field_tile(LinkTile<T, TX, TY> &tile, const BatchEv<T> &e, int2 w, int fpar,
                                                 int64_t n, T tau, T dtau, T tau_h) {
    const int lx = threadIdx.x >> 1, ly = threadIdx.y;
    const int tx = (e.N + TX - 1) / TX;
    const int x0 = (w.y % tx) * TX, y0 = (w.y / tx) * TY;
    const int tid = threadIdx.x + 2 * TX * threadIdx.y;
    stage_tile(tile, e.N, e.f[fpar], x0, y0, tid, 2 * TX * TY);
    __syncthreads();
    // every thread takes part (the step synchronises the workgroup)
    const bool active = x0 + lx < e.N && y0 + ly < e.N;
    const int reunit = e.reunit_every > 0 && (n % e.reunit_every) == e.reunit_every - 1;
    // a batch's working set overflows the last-level cache in either
    // precision: its streamed arrays take the non-temporal hint
    field_step_link<T, TX, TY, true>(tile, e.N, e.f[fpar], e.f[fpar ^ 1], e.n_species > 0 ? e.F : nullptr, x0, y0,
                                     lx, ly, threadIdx.x & 1, tid, active, tau, dtau, tau_h, reunit);
}

template <typename T, int TX, int TY>
__global__ void __launch_bounds__(2 * TX *TY)
k_batch_field(const BatchEv<T> *__restrict__ evs, const int2 *__restrict__ tiles, int64_t total, int fpar,
              const BatchCtl *__restrict__ ctl, T dtau) {
    __shared__ LinkTile<T, TX, TY> tile;
    const int64_t n = ctl->n;
    const T tau = dtau * (T)n, tau_h = dtau * ((T)n + T(0.5));
    int64_t stride, end;
    for (int64_t t = xcd_first(total, stride, end); t < end; t += stride) {
        const int2 w = tiles[t];
        if (*evs[w.x].fail != kNotFailed) continue;   // a failed event is masked (uniform per workgroup)
        __syncthreads();   // the previous tile's reads are done
        batch_field_tile(tile, evs[w.x], w, fpar, n, tau, dtau, tau_h);
    }
}

// One workgroup per table entry (grid = entries), numbered so that each XCD
// takes one contiguous run of the table: the walk of the persistent kernel
// without its loop, which holds registers the step can use.
template <typename T, int TX, int TY>
__global__ void __launch_bounds__(2 * TX *TY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 2 : 4, 8)))
k_batch_field_flat(const BatchEv<T> *__restrict__ evs, const int2 *__restrict__ tiles, int64_t total, int fpar,
                   const BatchCtl *__restrict__ ctl, T dtau) {
    __shared__ LinkTile<T, TX, TY> tile;
    const int64_t n = ctl->n;
    const T tau = dtau * (T)n, tau_h = dtau * ((T)n + T(0.5));
    const int2 w = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    if (*evs[w.x].fail != kNotFailed) return;   // a failed event is masked (uniform per workgroup)
    batch_field_tile(tile, evs[w.x], w, fpar, n, tau, dtau, tau_h);
}

// one block of an event's particles; with PERM, position i takes the particle
// in slot perm[i] of buffer parity ppar (the pending sort) and the pushed
// particle goes, with its species, momenta at formation and id, to slot i of
// parity ppar ^ 1, as the single-event push that applies a sort does
template <typename T, bool PERM>
__device__ __forceinline__ void batch_push_block(const BatchEv<T> &e, int2 w, int fpar, int ppar, int n, T dtau) {
    const int64_t i = (int64_t)w.y * kPushBlock + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int s = -1;
    if (i < e.n_slots) {
        if constexpr (PERM) {
            const PartPtrs<T> &P = e.P[ppar], &W = e.P[ppar ^ 1];
            const int64_t src = e.sort.vals[1][i];
            // the arrays that only move go first, so that nothing of them
            // stays live through the push
            W.species[i] = P.species[src];
            W.px0[i] = P.px0[src];
            W.py0[i] = P.py0[src];
            W.pz0[i] = P.pz0[src];
            e.ids[ppar ^ 1][i] = e.ids[ppar][src];
            __builtin_amdgcn_sched_barrier(0);
            s = push_particle<T, true, true>(e.N, P, src, W, i, e.f[fpar], e.F, e.tab, n, dtau, acc);
        } else {
            s = push_particle<T, false, true>(e.N, e.P[ppar], i, e.P[ppar], i, e.f[fpar], e.F, e.tab, n, dtau, acc);
        }
    }
    block_species_reduce(s, acc, e.n_species, e.partials + (size_t)w.y * e.n_species * 4);
}

// a masked (failed) event is not pushed, but a pending sort still moves its
// particles, so that its buffers follow the batch's parity
template <typename T, bool PERM>
__device__ __forceinline__ void batch_masked_block(const BatchEv<T> &e, int2 w, int ppar) {
    if constexpr (PERM) {
        const int64_t j = (int64_t)w.y * kPushBlock + threadIdx.x;
        if (j < e.n_slots) permute_one(e.P[ppar], e.P[ppar ^ 1], e.sort.vals[1], j, e.ids[ppar], e.ids[ppar ^ 1]);
    }
}

template <typename T, bool PERM>
__global__ void __launch_bounds__(kPushBlock)
k_batch_push(const BatchEv<T> *__restrict__ evs, const int2 *__restrict__ blocks, int64_t total, int fpar,
             int ppar, const BatchCtl *__restrict__ ctl, T dtau) {
    const int n = (int)ctl->n;
    int64_t stride, end;
    for (int64_t t = xcd_first(total, stride, end); t < end; t += stride) {
        const int2 w = blocks[t];
        if (*evs[w.x].fail != kNotFailed) {
            batch_masked_block<T, PERM>(evs[w.x], w, ppar);
            continue;
        }
        batch_push_block<T, PERM>(evs[w.x], w, fpar, ppar, n, dtau);
    }
}

template <typename T, bool PERM>
__global__ void __launch_bounds__(kPushBlock)
k_batch_push_flat(const BatchEv<T> *__restrict__ evs, const int2 *__restrict__ blocks, int64_t total, int fpar,
                  int ppar, const BatchCtl *__restrict__ ctl, T dtau) {
    const int2 w = blocks[xcd_remap(blockIdx.x, gridDim.x)];
    if (*evs[w.x].fail != kNotFailed) {
        batch_masked_block<T, PERM>(evs[w.x], w, ppar);
        return;
    }
    batch_push_block<T, PERM>(evs[w.x], w, fpar, ppar, (int)ctl->n, dtau);
}

// one workgroup per (event, species): fixed-order sum of the event's partial
// rows into its series row n - 1, n taken from the control block
template <typename T>
__global__ void __launch_bounds__(256)
k_batch_reduce(const BatchEv<T> *__restrict__ evs, const BatchCtl *__restrict__ ctl) {
    const BatchEv<T> &e = evs[blockIdx.x];
    const int s = blockIdx.y;
    if (s >= e.n_species) return;
    const int64_t row = ctl->n - 1;
    if (row < 0 || row >= e.max_steps) return;
    // masked since an earlier step: that push skipped the event, its partial
    // rows are stale.  Blocks of this launch lower fail to n + 1 at most, so
    // the test reads the same for every thread of the workgroup.
    if (*e.fail <= ctl->n) return;
    const int nb = (int)(e.n_slots / kPushBlock);
    __shared__ double red[256][4];
    double acc[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += 256)
#pragma unroll
        for (int k = 0; k < 4; k++) acc[k] += e.partials[((size_t)b * e.n_species + s) * 4 + k];
#pragma unroll
    for (int k = 0; k < 4; k++) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < 4; k++) red[threadIdx.x][k] += red[threadIdx.x + w][k];
        __syncthreads();
    }
    if (threadIdx.x < 4) {
        double v = red[0][threadIdx.x];
        if (threadIdx.x < 3 && red[0][3] > 0.0) v -= e.p0sum[s * 4 + threadIdx.x];
        e.series[((size_t)row * kMaxSpecies + s) * 4 + threadIdx.x] = v;
        // a non-finite sum fails the event at the step this push reached (n + 1)
        if (!isfinite(v)) atomicMin(e.fail, (int32_t)(ctl->n + 1 < kNotFailed ? ctl->n + 1 : kNotFailed - 1));
    }
}

// the batch's finite-value check: entry (event, chunk) tests values
// [chunk * kCheckChunk, ...) of the event's whole field state at parity fpar
template <typename T>
__global__ void __launch_bounds__(256)
k_batch_check(const BatchEv<T> *__restrict__ evs, const int2 *__restrict__ entries, int fpar,
              const BatchCtl *__restrict__ ctl) {
    const int2 w = entries[blockIdx.x];
    const BatchEv<T> &e = evs[w.x];
    const int64_t nvals = (int64_t)kStateVals * e.N * e.N;
    const int64_t lo = (int64_t)w.y * kCheckChunk, hi = lo + kCheckChunk < nvals ? lo + kCheckChunk : nvals;
    const T *a = e.f[fpar].U;   // the state's arrays lie contiguous from U on
    bool bad = false;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) bad |= !isfinite(a[i]);
    if (bad) atomicMin(e.fail, (int32_t)(ctl->n < kNotFailed ? ctl->n : kNotFailed - 1));
}

__global__ void k_batch_advance(BatchCtl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->n = ctl->n + 1;
}

template <typename T>
hipError_t launch_batch_fields(hipStream_t st, int shape, const BatchEv<T> *evs, const int2 *tiles, int64_t total,
                               int fpar, const BatchCtl *ctl, double dtau, int grid) {
    if (total <= 0) return hipSuccess;
    unsigned g = (unsigned)(grid > 0 && grid < total ? grid : total);
#define GL_SHAPE(TXv, TYv)                                                                                    \
    {                                                                                                         \
        if (g == total)                                                                                       \
            hipLaunchKernelGGL((k_batch_field_flat<T, TXv, TYv>), dim3(g), dim3(2 * TXv, TYv), 0, st, evs,    \
                               tiles, total, fpar, ctl, (T)dtau);                                             \
        else                                                                                                  \
            hipLaunchKernelGGL((k_batch_field<T, TXv, TYv>), dim3(g), dim3(2 * TXv, TYv), 0, st, evs, tiles,  \
                               total, fpar, ctl, (T)dtau);                                                    \
    }
    switch (shape) {
        case 0: GL_SHAPE(32, 4) break;
        case 1: GL_SHAPE(64, 2) break;
        case 2: GL_SHAPE(16, 8) break;
        default: return hipErrorInvalidValue;
    }
#undef GL_SHAPE
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_push(hipStream_t st, const BatchEv<T> *evs, const int2 *blocks, int64_t total, int fpar,
                             int ppar, const BatchCtl *ctl, double dtau, int grid, int n_events, bool permuted) {
    if (total > 0) {
        unsigned g = (unsigned)(grid > 0 && grid < total ? grid : total);
#define GL_PUSH(PERM)                                                                                          \
    {                                                                                                          \
        if (g == total)                                                                                        \
            hipLaunchKernelGGL((k_batch_push_flat<T, PERM>), dim3(g), dim3(kPushBlock), 0, st, evs, blocks, total, \
                               fpar, ppar, ctl, (T)dtau);                                                      \
        else                                                                                                   \
            hipLaunchKernelGGL((k_batch_push<T, PERM>), dim3(g), dim3(kPushBlock), 0, st, evs, blocks, total,   \
                               fpar, ppar, ctl, (T)dtau);                                                      \
    }
        if (permuted)
            GL_PUSH(true)
        else
            GL_PUSH(false)
#undef GL_PUSH
        hipLaunchKernelGGL(k_batch_reduce<T>, dim3(n_events, kMaxSpecies), dim3(256), 0, st, evs, ctl);
    }
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, st, (BatchCtl *)ctl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_check(hipStream_t st, const BatchEv<T> *evs, const int2 *entries, int64_t total, int fpar,
                              const BatchCtl *ctl) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_check<T>, dim3((unsigned)total), dim3(256), 0, st, evs, entries, fpar, ctl);
    return hipGetLastError();
}

#define GL_INST(T)                                                                                          \
    template hipError_t launch_batch_check<T>(hipStream_t, const BatchEv<T> *, const int2 *, int64_t, int,      \
                                              const BatchCtl *);                                             \
    template hipError_t launch_batch_fields<T>(hipStream_t, int, const BatchEv<T> *, const int2 *, int64_t, int, \
                                               const BatchCtl *, double, int);                               \
    template hipError_t launch_batch_push<T>(hipStream_t, const BatchEv<T> *, const int2 *, int64_t, int, int,  \
                                             const BatchCtl *, double, int, int, bool);
GL_INST(double)
GL_INST(float)
#undef GL_INST

}  // namespace gl
