// sort.hip -- keeps the particle arrays ordered by cell so that the particles
// of one workgroup gather site fields of neighbouring cells (a few cache
// lines per plane per wave, L2 reuse).  Stable LSD radix sort on 20-bit cell
// keys (padding slots get 0xFFFFF and stay at the end), three 8-bit digit
// passes, deterministic: counts per (digit, workgroup), a per-digit scan over
// workgroups, and a stable scatter whose in-workgroup ranks come from wave64
// ballots.
#include "batch_internal.hpp"
#include "su3.hpp"

namespace gl {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;                              // keys per thread
constexpr int kSortTile = kSortThreads * kSortItems;       // keys per workgroup
constexpr int kDigits = 256;

int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

// ---- the phases, for one tile (workgroup) of one sort ---------------------

// key and initial value of slot i < n
template <typename T>
__device__ __forceinline__ void sort_key_one(const PartPtrs<T> &P, int64_t i, int N, uint32_t *__restrict__ keys,
                                             int32_t *__restrict__ vals) {
    keys[i] = P.species[i] >= 0 ? (uint32_t)(P.cx[i] + N * P.cy[i]) : 0xFFFFFu;
    vals[i] = (int32_t)i;
}

// per-digit counts of tile `tile` (kSortTile keys), stored digit-major:
// counts[d * tiles + tile]
__device__ __forceinline__ void radix_count_tile(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                 int64_t tiles, int64_t tile, uint32_t *__restrict__ counts) {
    __shared__ uint32_t h[kDigits];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = tile * kSortTile + (int64_t)threadIdx.x * kSortItems;
#pragma unroll
    for (int k = 0; k < kSortItems; k++) {
        int64_t i = base + k;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    counts[(size_t)threadIdx.x * tiles + tile] = h[threadIdx.x];
}

// exclusive scan of one digit's row of per-tile counts in place (256
// threads), and the digit's total
__device__ __forceinline__ void scan_row(uint32_t *__restrict__ row, int64_t tiles, uint32_t *__restrict__ total) {
    __shared__ uint32_t part[256];
    const int t = threadIdx.x;
    int64_t chunk = (tiles + 255) / 256;
    int64_t lo = t * chunk, hi = lo + chunk < tiles ? lo + chunk : tiles;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; i++) s += row[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
    for (int64_t i = lo; i < hi; i++) {
        uint32_t v = row[i];
        row[i] = run;
        run += v;
    }
    if (t == 255) *total = part[255];
}

// stable scatter of tile `tile` by the digit at `shift`
__device__ __forceinline__ void radix_scatter_tile(const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin,
                                                   int64_t n, int shift, int64_t tiles, int64_t tile,
                                                   const uint32_t *__restrict__ offs,
                                                   const uint32_t *__restrict__ totals, uint32_t *__restrict__ kout,
                                                   int32_t *__restrict__ vout) {
    __shared__ uint32_t wcount[kSortThreads / 64][kDigits];
    __shared__ uint32_t running[kDigits];
    __shared__ uint32_t gstart[kDigits];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    // exclusive scan of the digit totals gives each digit's base
    gstart[t] = totals[t];
    __syncthreads();
    for (int off = 1; off < kDigits; off <<= 1) {
        uint32_t v = t >= off ? gstart[t - off] : 0u;
        __syncthreads();
        gstart[t] += v;
        __syncthreads();
    }
    uint32_t base = (t > 0 ? gstart[t - 1] : 0u) + offs[(size_t)t * tiles + tile];
    __syncthreads();
    gstart[t] = base;
    running[t] = 0;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kSortItems; r++) {
#pragma unroll
        for (int w = 0; w < kSortThreads / 64; w++) wcount[w][t] = 0;
        __syncthreads();
        int64_t i = tile * kSortTile + (int64_t)r * kSortThreads + t;
        bool valid = i < n;
        uint32_t key = valid ? kin[i] : 0u;
        uint32_t d = (key >> shift) & 0xFF;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint64_t m = __ballot(valid && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rank == 0) wcount[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t before = running[d];
            for (int w = 0; w < wave; w++) before += wcount[w][d];
            uint32_t pos = gstart[d] + before + rank;
            kout[pos] = key;
            vout[pos] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kSortThreads / 64; w++) add += wcount[w][t];
        running[t] += add;
        __syncthreads();
    }
}

// ---- single-sort kernels ----------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256)
k_sort_keys(PartPtrs<T> P, int64_t n, int N, uint32_t *__restrict__ keys, int32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) sort_key_one(P, i, N, keys, vals);
}

__global__ void __launch_bounds__(kSortThreads)
k_radix_count(const uint32_t *__restrict__ keys, int64_t n, int shift, int64_t tiles,
              uint32_t *__restrict__ counts) {
    radix_count_tile(keys, n, shift, tiles, blockIdx.x, counts);
}

// per digit d (one workgroup each): exclusive scan of counts[d][0..tiles) in
// place, and the digit's total
__global__ void __launch_bounds__(256)
k_scan_rows(uint32_t *__restrict__ counts, int64_t tiles, uint32_t *__restrict__ totals) {
    scan_row(counts + (size_t)blockIdx.x * tiles, tiles, totals + blockIdx.x);
}

__global__ void __launch_bounds__(kSortThreads)
k_radix_scatter(const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin, int64_t n,
                int shift, int64_t tiles, const uint32_t *__restrict__ offs,
                const uint32_t *__restrict__ totals, uint32_t *__restrict__ kout,
                int32_t *__restrict__ vout) {
    radix_scatter_tile(kin, vin, n, shift, tiles, blockIdx.x, offs, totals, kout, vout);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_permute(PartPtrs<T> src, PartPtrs<T> dst, const int32_t *__restrict__ perm, int64_t n,
          int32_t *__restrict__ id_src, int32_t *__restrict__ id_dst) {
    int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) permute_one(src, dst, perm, j, id_src, id_dst);
}

// ---- batched kernels: one launch per phase for all events of a batch -------
// Work tables: pblocks (event, block of kPushBlock slots) over each event's
// used slots, stiles (event, sort tile); an event's particles move from
// buffer parity ppar to ppar ^ 1.

template <typename T>
__global__ void __launch_bounds__(256)
k_batch_sort_keys(const BatchEv<T> *__restrict__ evs, const int2 *__restrict__ pblocks, int ppar) {
    const int2 w = pblocks[blockIdx.x];
    const BatchEv<T> &e = evs[w.x];
    const int64_t i = (int64_t)w.y * kPushBlock + threadIdx.x;
    if (i < e.n_slots) sort_key_one(e.P[ppar], i, e.N, e.sort.keys[0], e.sort.vals[0]);
}

template <typename T>
__global__ void __launch_bounds__(kSortThreads)
k_batch_radix_count(const BatchEv<T> *__restrict__ evs, const int2 *__restrict__ stiles, int shift, int cur) {
    const int2 w = stiles[blockIdx.x];
    const BatchEv<T> &e = evs[w.x];
    radix_count_tile(e.sort.keys[cur], e.n_slots, shift, e.sort_tiles, w.y, e.sort.counts);
}

// workgroup e * 256 + d scans digit d of event e
template <typename T>
__global__ void __launch_bounds__(256) k_batch_scan_rows(const BatchEv<T> *__restrict__ evs) {
    const BatchEv<T> &e = evs[blockIdx.x >> 8];
    const int d = blockIdx.x & 255;
    if (e.n_slots <= 0) return;
    scan_row(e.sort.counts + (size_t)d * e.sort_tiles, e.sort_tiles, e.sort.totals + d);
}

template <typename T>
__global__ void __launch_bounds__(kSortThreads)
k_batch_radix_scatter(const BatchEv<T> *__restrict__ evs, const int2 *__restrict__ stiles, int shift, int cur) {
    const int2 w = stiles[blockIdx.x];
    const BatchEv<T> &e = evs[w.x];
    radix_scatter_tile(e.sort.keys[cur], e.sort.vals[cur], e.n_slots, shift, e.sort_tiles, w.y, e.sort.counts,
                       e.sort.totals, e.sort.keys[cur ^ 1], e.sort.vals[cur ^ 1]);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_batch_permute(const BatchEv<T> *__restrict__ evs, const int2 *__restrict__ pblocks, int ppar) {
    const int2 w = pblocks[blockIdx.x];
    const BatchEv<T> &e = evs[w.x];
    const int64_t j = (int64_t)w.y * kPushBlock + threadIdx.x;
    if (j < e.n_slots) permute_one(e.P[ppar], e.P[ppar ^ 1], e.sort.vals[1], j, e.ids[ppar], e.ids[ppar ^ 1]);
}

// The sorted order of the n slots of src by cell: perm[j] is the slot that
// goes to position j (in the sort scratch, see sort_perm).
template <typename T>
hipError_t launch_sort_order(hipStream_t st, int N, PartPtrs<T> src, int64_t n, SortScratch s) {
    if (n <= 0) return hipSuccess;
    const int64_t tiles = sort_tiles(n);
    unsigned b256 = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_sort_keys<T>, dim3(b256), dim3(256), 0, st, src, n, N, s.keys[0], s.vals[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int cur = 0;
    for (int pass = 0; pass < 3; pass++) {
        int shift = 8 * pass;
        hipLaunchKernelGGL(k_radix_count, dim3((unsigned)tiles), dim3(kSortThreads), 0, st, s.keys[cur], n,
                           shift, tiles, s.counts);
        hipLaunchKernelGGL(k_scan_rows, dim3(kDigits), dim3(256), 0, st, s.counts, tiles, s.totals);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)tiles), dim3(kSortThreads), 0, st, s.keys[cur],
                           s.vals[cur], n, shift, tiles, s.counts, s.totals, s.keys[cur ^ 1],
                           s.vals[cur ^ 1]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur ^= 1;
    }
    return hipSuccess;
}

// three digit passes leave the permutation in the second value buffer
const int32_t *sort_perm(SortScratch s) { return s.vals[1]; }

template <typename T>
hipError_t launch_permute(hipStream_t st, PartPtrs<T> src, PartPtrs<T> dst, const int32_t *perm, int64_t n,
                          int32_t *id_src, int32_t *id_dst) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, perm, n, id_src,
                       id_dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sort_particles(hipStream_t st, int N, PartPtrs<T> src, PartPtrs<T> dst, int64_t n,
                                 SortScratch s, int32_t *id_src, int32_t *id_dst) {
    hipError_t e = launch_sort_order<T>(st, N, src, n, s);
    if (e != hipSuccess) return e;
    return launch_permute<T>(st, src, dst, sort_perm(s), n, id_src, id_dst);
}

// the sorted order of every event of a batch by cell, of buffer parity ppar:
// keys and three digit passes (count, scan, scatter), one launch each for all
// events, leaving each event's permutation in its sort scratch (vals[1]);
// with permute, then the permutation itself (ppar to ppar ^ 1), else the next
// push applies it (launch_batch_push with permuted)
template <typename T>
hipError_t launch_batch_sort(hipStream_t st, const BatchEv<T> *evs, int n_events, const int2 *pblocks,
                             int64_t n_pblocks, const int2 *stiles, int64_t n_stiles, int ppar, bool permute) {
    if (n_pblocks <= 0 || n_stiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_sort_keys<T>, dim3((unsigned)n_pblocks), dim3(256), 0, st, evs, pblocks, ppar);
    int cur = 0;
    for (int pass = 0; pass < 3; pass++) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_batch_radix_count<T>, dim3((unsigned)n_stiles), dim3(kSortThreads), 0, st, evs, stiles,
                           shift, cur);
        hipLaunchKernelGGL(k_batch_scan_rows<T>, dim3((unsigned)n_events * kDigits), dim3(256), 0, st, evs);
        hipLaunchKernelGGL(k_batch_radix_scatter<T>, dim3((unsigned)n_stiles), dim3(kSortThreads), 0, st, evs,
                           stiles, shift, cur);
        cur ^= 1;
    }
    if (permute) return launch_batch_permute<T>(st, evs, pblocks, n_pblocks, ppar);
    return hipGetLastError();
}

// every event's pending permutation (left by launch_batch_sort) applied alone,
// buffer parity ppar to ppar ^ 1
template <typename T>
hipError_t launch_batch_permute(hipStream_t st, const BatchEv<T> *evs, const int2 *pblocks, int64_t n_pblocks,
                                int ppar) {
    if (n_pblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_permute<T>, dim3((unsigned)n_pblocks), dim3(256), 0, st, evs, pblocks, ppar);
    return hipGetLastError();
}

#define GL_INST(T)                                                                                            \
    template hipError_t launch_sort_particles<T>(hipStream_t, int, PartPtrs<T>, PartPtrs<T>, int64_t, SortScratch, \
                                                 int32_t *, int32_t *);                                          \
    template hipError_t launch_sort_order<T>(hipStream_t, int, PartPtrs<T>, int64_t, SortScratch);                \
    template hipError_t launch_permute<T>(hipStream_t, PartPtrs<T>, PartPtrs<T>, const int32_t *, int64_t,        \
                                          int32_t *, int32_t *);                                                  \
    template hipError_t launch_batch_sort<T>(hipStream_t, const BatchEv<T> *, int, const int2 *, int64_t,         \
                                             const int2 *, int64_t, int, bool);                                   \
    template hipError_t launch_batch_permute<T>(hipStream_t, const BatchEv<T> *, const int2 *, int64_t, int);
GL_INST(double)
GL_INST(float)
#undef GL_INST

}  // namespace gl
