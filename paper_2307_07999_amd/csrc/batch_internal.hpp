// batch_internal.hpp -- device descriptors of a batch of events stepped in
// lock-step by the flattened multi-event kernels (batch_kernels.hip).
#pragma once
#include "internal.hpp"
#include "su3.hpp"

namespace gl {

template <typename T>
struct BatchEv {
    int N;
    int reunit_every;
    int n_species;
    int max_steps;
    int64_t n_slots;
    FieldPtrs<T> f[2];     // f[p] and f[p ^ 1]: state at step n and at n + 1 for parity p
    PartPtrs<T> P[2];      // particle buffers; the current one alternates at each sort
    T *F;                  // site-field records (chunked planes), written by the field phase when n_species > 0
    double *partials;      // [n_slots / kPushBlock][n_species][4]
    const double *p0sum;   // [kMaxSpecies][4]: sums of the squared momenta at formation
    double *series;        // [max_steps][kMaxSpecies][4]
    SpeciesTab<T> tab;
    SortScratch sort;      // the event's radix-sort scratch
    int64_t sort_tiles;    // sort tiles over n_slots
    int32_t *ids[2];       // particle ids, alternating with P
    int32_t *fail;         // first step at which the event failed (kNotFailed: none); failed events are skipped
};

constexpr int32_t kNotFailed = 0x7F7F7F7F;   // the value of bytes 0x7F, as hipMemsetAsync writes it
constexpr int64_t kCheckChunk = 65536;       // state values per entry of the batch's finite-value check

struct BatchCtl {
    int64_t n;             // common step index of all events
};

constexpr int kBatchShapes = 3;   // field-kernel site tiles 32x4, 64x2, 16x8 (two lanes per site)

// position j of dst takes every array of slot perm[j] of src
template <typename T>
__device__ __forceinline__ void permute_one(const PartPtrs<T> &src, const PartPtrs<T> &dst,
                                            const int32_t *__restrict__ perm, int64_t j,
                                            const int32_t *__restrict__ id_src, int32_t *__restrict__ id_dst) {
    int64_t i = perm[j];
    dst.cx[j] = src.cx[i];
    dst.cy[j] = src.cy[i];
    dst.species[j] = src.species[i];
#pragma unroll
    for (int k = 0; k < kPartRec<T>; k += 16 / (int)sizeof(T)) {
        T v[16 / sizeof(T)];
        chunk_ld16(src.st, (size_t)src.cap, (size_t)i, k, v);
        chunk_st16(dst.st, (size_t)dst.cap, (size_t)j, k, v);
    }
    dst.px0[j] = src.px0[i];
    dst.py0[j] = src.py0[i];
    dst.pz0[j] = src.pz0[i];
    id_dst[j] = id_src[i];
}

template <typename T>
hipError_t launch_batch_fields(hipStream_t st, int shape, const BatchEv<T> *evs, const int2 *tiles, int64_t total,
                               int fpar, const BatchCtl *ctl, double dtau, int grid);
// the particle sort of every event, one launch per phase; pblocks (event,
// particle block) and stiles (event, sort tile) cover each event's used
// slots.  The sorted order of buffer parity ppar goes to each event's sort
// scratch; with permute the particles then move to parity ppar ^ 1, else the
// next push moves them (launch_batch_push with permuted) or
// launch_batch_permute does.
template <typename T>
hipError_t launch_batch_sort(hipStream_t st, const BatchEv<T> *evs, int n_events, const int2 *pblocks,
                             int64_t n_pblocks, const int2 *stiles, int64_t n_stiles, int ppar, bool permute);
template <typename T>
hipError_t launch_batch_permute(hipStream_t st, const BatchEv<T> *evs, const int2 *pblocks, int64_t n_pblocks,
                                int ppar);
// the push of every event from buffer parity ppar; with permuted, position j
// takes the particle in slot perm[j] of ppar (the pending sort) and the pushed
// particles go to parity ppar ^ 1 (a masked event's particles are moved
// without a push)
template <typename T>
hipError_t launch_batch_push(hipStream_t st, const BatchEv<T> *evs, const int2 *blocks, int64_t total, int fpar,
                             int ppar, const BatchCtl *ctl, double dtau, int grid, int n_events, bool permuted);
// every event's field state at parity fpar checked for NaN/Inf in chunks of
// kCheckChunk values ((event, chunk) entries); a failing event's fail slot
// is lowered to the current step
template <typename T>
hipError_t launch_batch_check(hipStream_t st, const BatchEv<T> *evs, const int2 *entries, int64_t total, int fpar,
                              const BatchCtl *ctl);

}  // namespace gl
