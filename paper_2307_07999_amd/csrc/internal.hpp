// internal.hpp -- device-side data descriptions shared by the kernels and the
// runtime of the Glasma + colored-particle-in-cell library (not installed).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gl {

constexpr int kMaxSpecies = 16;
constexpr int kPushBlock = 256;   // particles per push workgroup
// site-field record of kSiteRec reals per site in chunked planes (16-byte
// chunks of consecutive values, one chunk plane per chunk index over all
// sites): slots of 8 reals Ex, Ey, Ez, Bx, By, Bz (local frame), then two
// slots for the second halves of Ex and Ey.  E_i at a site is the sum of
// the half from the link U_i(x) and the half transported from U_i(x - i).
// Where both links fall in one field-step workgroup the step adds them and
// stores the sum in slot i; at the sites of half_stored (a fixed lattice
// rule that every tile shape respects) the half from x - i is stored apart
// in slot 6 + i, and readers add it: E_i = slot i + slot 6 + i there, slot
// i elsewhere (slot 6 + i is not written).  Either way it is the same sum
// of the same two halves.  A particle reads its cell's record in 16-byte
// loads, and the field step's lanes store neighbouring chunks.
constexpr int kSiteRec = 64;
constexpr int kHalfX = 16, kHalfY = 2;   // tile widths and heights are multiples of these
// whether site (ix, iy) keeps the half of E_{d+1} from x - (d+1) apart
__host__ __device__ __forceinline__ bool half_stored(int d, int ix, int iy) {
    return d == 0 ? ix % kHalfX == 0 : iy % kHalfY == 0;
}

// distance between consecutive planes of a lattice quantity, in elements
// (packed: a padded pitch against L2 set aliasing of the power-of-two planes
// measured no faster)
__host__ __device__ __forceinline__ size_t plane_pitch(int N) { return (size_t)N * N; }

// Workgroup b of a grid of nb runs on XCD b mod 8.  Renumber the grid so
// that every XCD gets one contiguous run of logical blocks (row bands of a
// lattice, neighbouring particle blocks), and the stencil's neighbour reads
// hit that XCD's L2: XCD x owns nb/8 (+1 for x < nb mod 8) blocks.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t x = b & 7, j = b >> 3, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + j;
}

// One field state, each array in chunked planes over the n2 = N*N sites
// (16-byte chunks of consecutive values; value k of site x at element
// ((k / NV) n2 + x) NV + k mod NV, NV = 16 / sizeof(T)):
//   U: 24 values per site, the first two rows of link U_i at 12 (i - 1)
//   (entry (a,b) real at + 2(3a+b), imaginary next to it, a = 0, 1; the
//   third row is rebuilt where a link is read); E: 16, E_i at 8 (i - 1);
//   phi: 8; pi: 8.  kStateVals reals per site in all.
constexpr int kStateVals = 2 * 12 + 16 + 8 + 8;

template <typename T>
struct FieldPtrs {
    T *U;
    T *E;
    T *phi;
    T *pi;
};

// Particle arrays, capacity cap (padded per species to kPushBlock).  The
// state the push reads and writes every step is one record of
// kPartRec<T> values per slot in chunked planes over the slots (value k of
// slot i at element ((k / NV) cap + i) NV + k mod NV): offsets within the
// cell, the rapidity, p_x, p_y, P_eta = tau^2 p^eta and the colour charge
// Q^a, 14 values: seven whole chunks in FP64; FP32 pads them to four chunks
// (values 14, 15 unused).
constexpr int kOx = 0, kOy = 1, kEta = 2, kPx = 3, kPy = 4, kPeta = 5, kQ = 6;
constexpr int part_rec(size_t value_bytes) { return value_bytes == 8 ? 14 : 16; }
template <typename T>
constexpr int kPartRec = part_rec(sizeof(T));
template <typename T>
struct PartPtrs {
    int32_t *cx, *cy;
    T *st;               // [kPartRec<T>] record per slot, chunked planes
    T *px0, *py0, *pz0;  // momenta at formation (pz0 in the lab frame)
    int32_t *species;    // -1 for padding
    int64_t cap;
};

// radix-sort scratch: double-buffered keys and values, per-(digit, tile)
// counts and per-digit totals
struct SortScratch {
    uint32_t *keys[2];
    int32_t *vals[2];
    uint32_t *counts;
    uint32_t *totals;
};
int64_t sort_tiles(int64_t n);
template <typename T>
hipError_t launch_sort_particles(hipStream_t st, int N, PartPtrs<T> src, PartPtrs<T> dst, int64_t n,
                                 SortScratch s, int32_t *id_src, int32_t *id_dst);
// the two halves of launch_sort_particles: the sorted order (its
// permutation then at sort_perm), and moving every particle array by it
template <typename T>
hipError_t launch_sort_order(hipStream_t st, int N, PartPtrs<T> src, int64_t n, SortScratch s);
const int32_t *sort_perm(SortScratch s);
template <typename T>
hipError_t launch_permute(hipStream_t st, PartPtrs<T> src, PartPtrs<T> dst, const int32_t *perm, int64_t n,
                          int32_t *id_src, int32_t *id_dst);

template <typename T>
struct SpeciesTab {
    T mass[kMaxSpecies];
    int32_t nform[kMaxSpecies];
};

// ---- launchers (stream-ordered, no synchronisation) --------------------------
// Events that a launch records itself at its kernel's start and end
// (hipExtLaunchKernelGGL): the kernel's own duration, without the dispatch
// gap that events recorded on the stream around a launch also cover.  Both
// null: an ordinary launch.
struct KernelTimer {
    hipEvent_t start = nullptr, stop = nullptr;
};
#define GL_LAUNCH_TIMED(kt, kernel, grid, block, shmem, st, ...)                                        \
    do {                                                                                                \
        if ((kt).start)                                                                                 \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, (kt).start, (kt).stop, 0u, __VA_ARGS__); \
        else                                                                                            \
            hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__);                            \
    } while (0)
// a launch with nothing to do still closes its sample (an empty interval)
inline hipError_t timer_skip(hipStream_t st, const KernelTimer &kt) {
    if (!kt.start) return hipSuccess;
    hipError_t e = hipEventRecord(kt.start, st);
    return e != hipSuccess ? e : hipEventRecord(kt.stop, st);
}

// F: site-field records at tau_n in chunked planes, written when non-null
template <typename T>
hipError_t launch_field_step(hipStream_t st, int N, FieldPtrs<T> in, FieldPtrs<T> out, T *F,
                             double tau, double dtau, int reunit, const KernelTimer &kt);
template <typename T>
hipError_t launch_push(hipStream_t st, int N, PartPtrs<T> p, int64_t n_slots, FieldPtrs<T> f,
                       const T *F, SpeciesTab<T> tab, int n_species, int n, double dtau,
                       double *partials, const KernelTimer &kt);
// the push of particles still to be moved by a sort permutation: position j
// is pushed from slot perm[j] of p and written, with the particle's other
// arrays and id, to slot j of dst
template <typename T>
hipError_t launch_push_permuted(hipStream_t st, int N, PartPtrs<T> p, PartPtrs<T> dst, const int32_t *perm,
                                const int32_t *id_src, int32_t *id_dst, int64_t n_slots, FieldPtrs<T> f,
                                const T *F, SpeciesTab<T> tab, int n_species, int n, double dtau,
                                double *partials, const KernelTimer &kt);
hipError_t launch_iota(hipStream_t st, int32_t *id, int64_t n, int64_t n_valid, int32_t base);
// fixed-order sum of per-workgroup partial rows into a series row; a
// non-null sub [kMaxSpecies][4] is subtracted from the first three terms of
// every species with a non-zero count
hipError_t launch_series_reduce(hipStream_t st, const double *partials, int n_blocks, int n_species,
                                double *row, const double *sub);
// the same for n_rows consecutive steps at once: step r reads the partial
// rows at partials + r * slot_stride and writes row + r * kMaxSpecies * 4
hipError_t launch_series_reduce_steps(hipStream_t st, const double *partials, size_t slot_stride, int n_rows,
                                      int n_blocks, int n_species, double *row, const double *sub);
// per-species sums (p_x0^2, p_y0^2, p_z0^2, count) of the momenta at
// formation into out [kMaxSpecies][4], through the partial rows
template <typename T>
hipError_t launch_p0_sums(hipStream_t st, PartPtrs<T> p, int64_t n_slots, int n_species, double *partials,
                          double *out);
// static-quark accumulators I [24][n2] FP64; partials [blocks][4]
template <typename T>
hipError_t launch_static_accum(hipStream_t st, int N, const T *F, double *I, double dtau, double *partials,
                               int *n_blocks_out);
// lightlike-jet transports W [18][n2] and accumulators I [24][n2] FP64; U the x links at tau_n
template <typename T>
hipError_t launch_lightlike_accum(hipStream_t st, int N, const T *F, const T *U, double *W, double *I, int64_t j,
                                  double dtau, double *partials, int *n_blocks_out);
template <typename T>
hipError_t launch_diag(hipStream_t st, int N, FieldPtrs<T> f, double tau, double *partials,
                       int *n_blocks_out);
// lowers *first_bad to step0 + i / vals_per_step for every non-finite value i
// of a [0, n) (16-byte aligned; the int is not reset here)
template <typename T>
hipError_t launch_check_finite(hipStream_t st, const T *a, int64_t n, int64_t vals_per_step, int step0,
                               int *first_bad);

// initial conditions (always FP64 internally)
constexpr int kSheetChunk = 8;   // MV sheets per initialisation launch
// the MV charges of one nucleus drawn for sheets sheet0.. (seeded, counter
// based): colours 2j, 2j + 1 of sheet s at site x from one draw
struct MvDraw {
    double sigma;
    uint64_t seed;
    int nucleus;
    int sheet0;
};
hipError_t launch_mv_charges(hipStream_t st, int N, double sigma, uint64_t seed, int nucleus,
                             int sheet0, int n_sheets, double2 *planes /* [n_sheets][4][n2] */);
hipError_t launch_charges_to_planes(hipStream_t st, int N, const double *rho /* [8][n2] */,
                                 double2 *planes);
hipError_t launch_planes_to_charges(hipStream_t st, int N, const double2 *planes, double *rho);
// the twiddle and sin^2 tables of one solve size into tab (kFftTableBytes)
constexpr size_t kFftTableBytes = 1024 * (sizeof(double2) + sizeof(double));
hipError_t launch_fft_tables(hipStream_t st, int N, double2 *tab);
hipError_t launch_poisson(hipStream_t st, int N, double m2, double uv2, double2 *planes, int n_sheets,
                          const double2 *tab, const MvDraw *draw = nullptr);
hipError_t launch_wilson_init(hipStream_t st, int N, double *V);
// dipole correlator D[0..rmax] of a Wilson line; partials [(rmax+1)][ceil(N^2/256)]
hipError_t launch_dipole(hipStream_t st, int N, const double *V, int rmax, double *partials, double *D);
hipError_t launch_wilson_accum(hipStream_t st, int N, const double2 *planes, int n_sheets, double *V);
hipError_t launch_match_pi0(hipStream_t st, int N, const double *VA, const double *VB,
                           double *U0 /* [2][18][n2] FP64 */, double *pi0 /* [8][n2] */,
                           int *status, int max_iter, double tol);
// per workgroup max |q2 - 4| and max |q3 - 10/3| of the particles' charges:
// partials [blocks][2]
template <typename T>
hipError_t launch_casimir(hipStream_t st, PartPtrs<T> p, int64_t n_slots, double *partials,
                          int *n_blocks_out);
template <typename T>
hipError_t launch_first_half_step(hipStream_t st, int N, const double *U0, const double *pi0,
                                  FieldPtrs<T> out, double dtau);
template <typename T>
hipError_t launch_particles_init(hipStream_t st, int N, PartPtrs<T> p, int64_t slot0, int64_t n,
                                 uint64_t seed, int species_id, int kind, double p0);

}  // namespace gl
