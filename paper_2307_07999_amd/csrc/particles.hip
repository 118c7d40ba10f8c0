// particles.hip -- colored particles in the Glasma: initialisation, the push
// of Wong's equations (Eq. (2)) and the FP64 momentum-broadening sums.
//
// Push (one thread per particle, reading the site-field record F^n of its
// cell -- the six local-frame fields, E_x and E_y plus the half stored apart
// where half_stored holds, in 16-byte chunks -- and phi^n from the field
// state; the particles are kept
// sorted by cell so that a wave's gathers hit neighbouring addresses):
//   e_k = Q^a E_k^a, b_k = Q^a B_k^a in the local frame at tau_n
//   Boris kick of dp/dtau = e + v x b on (p_x, p_y, P_eta/tau_n), P_eta = tau^2 p^eta
//   drift with velocities at tau_{n+1/2}; rapidity step d_eta
//   color: Q <- W Q W^dag, W = exp(-i phi^n(cell) d_eta) (eta component of the
//   Wilson line), then on a cell crossing Q <- U^dag Q U (forward) or
//   U Q U^dag (backward) with the crossed link: the link-built particle
//   Wilson line of the colored-particle-in-cell method, which conserves the
//   Casimirs of Q.
//   broadening at tau_{n+1/2}: p_x^2, p_y^2 and the lab-frame p_z^2, less the
//   species' sums of the squares at formation (taken once, see k_p0_sums).
// Each workgroup writes one FP64 partial row per species into the step's
// slot; a second kernel sums the rows of each species in a fixed order for
// up to 16 steps at once, so the series is deterministic for a given
// particle order.
#include "philox.hpp"
#include "push_dev.hpp"

namespace gl {

template <typename T>
__global__ void __launch_bounds__(kPushBlock)
k_push(int N, PartPtrs<T> P, int64_t n_slots, FieldPtrs<T> f, const T *__restrict__ F,
       SpeciesTab<T> tab, int n_species, int n, T dtau, double *__restrict__ partials) {
    // neighbouring blocks (neighbouring cells, the particles being sorted) on one XCD
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t i = blk * kPushBlock + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int s = -1;
    if (i < n_slots) s = push_particle<T>(N, P, i, P, i, f, F, tab, n, dtau, acc);
    block_species_reduce(s, acc, n_species, partials + (size_t)blk * n_species * 4);
}

// The push that also applies a pending sort: position j takes the particle
// in slot perm[j] of P, pushes it and writes it, with its species, momenta at
// formation and id, to slot j of W.  The blocks (and so the partial rows) are
// those of a push after the permutation.
template <typename T>
__global__ void __launch_bounds__(kPushBlock)
k_push_permuted(int N, PartPtrs<T> P, PartPtrs<T> W, const int32_t *__restrict__ perm,
                const int32_t *__restrict__ id_src, int32_t *__restrict__ id_dst, int64_t n_slots, FieldPtrs<T> f,
                const T *__restrict__ F, SpeciesTab<T> tab, int n_species, int n, T dtau,
                double *__restrict__ partials) {
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t j = blk * kPushBlock + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int s = -1;
    if (j < n_slots) {
        const int64_t i = perm[j];
        // the fields that only move go first, so that nothing of them stays
        // live through the push
        W.species[j] = P.species[i];
        W.px0[j] = P.px0[i];
        W.py0[j] = P.py0[i];
        W.pz0[j] = P.pz0[i];
        id_dst[j] = id_src[i];
        __builtin_amdgcn_sched_barrier(0);
        s = push_particle<T, true>(N, P, i, W, j, f, F, tab, n, dtau, acc);
    }
    block_species_reduce(s, acc, n_species, partials + (size_t)blk * n_species * 4);
}

// series row [kMaxSpecies][4]: species s sums the partial rows of all push
// workgroups in a fixed order; with sub, a species with active particles
// then has sub[s][k] (k < 3) subtracted from its three momentum sums.
__global__ void __launch_bounds__(256)
k_series_reduce(const double *__restrict__ partials, int n_blocks, int n_species, const double *__restrict__ sub,
                double *__restrict__ row, size_t slot_stride) {
    // blockIdx.y: one of several steps reduced in one launch
    const int s = blockIdx.x;
    partials += (size_t)blockIdx.y * slot_stride;
    row += (size_t)blockIdx.y * kMaxSpecies * 4;
    __shared__ double red[256][4];
    double acc[4] = {0, 0, 0, 0};
    if (s < n_species) {
        for (int b = threadIdx.x; b < n_blocks; b += 256)
#pragma unroll
            for (int k = 0; k < 4; k++) acc[k] += partials[((size_t)b * n_species + s) * 4 + k];
    }
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
        if (sub && threadIdx.x < 3 && red[0][3] > 0.0) v -= sub[s * 4 + threadIdx.x];
        row[s * 4 + threadIdx.x] = v;
    }
}

// Particle initialisation (Sec. 2 toy model, Sec. 1 color charges): counter
// (i, j, 2 + species, 0) with j = 0 position, j = 1 azimuth, j = 2..10 the nine
// Gaussian pairs of a complex matrix whose Gram-Schmidt factor is Haar on U(3)
// (Mezzadri 2007); Q = U Q0 U^dag with Q0 = diag of the roots of
// l^3 - l - 5/18 (q2 = 4, q3 = 10/3).
template <typename T>
__global__ void __launch_bounds__(256)
k_particles_init(int N, PartPtrs<T> P, int64_t slot0, int64_t n, uint64_t seed, int species,
                 int kind, double p0) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t j = slot0 + i;
    const uint32_t stream = 2u + (uint32_t)species;
    U4 w = draw(seed, (uint32_t)i, 0u, stream);
    double X = uniform53(w.v[0], w.v[1]) * N, Y = uniform53(w.v[2], w.v[3]) * N;
    double fx = floor(X + 0.5), fy = floor(Y + 0.5);
    int cx = (int)fx, cy = (int)fy;
    P.cx[j] = cx >= N ? cx - N : cx;
    P.cy[j] = cy >= N ? cy - N : cy;
    T r[kPartRec<T>];
#pragma unroll
    for (int k = 0; k < kPartRec<T>; k++) r[k] = T(0);
    r[kOx] = (T)(X - fx);
    r[kOy] = (T)(Y - fy);
    w = draw(seed, (uint32_t)i, 1u, stream);
    double az = 6.283185307179586476925286766559 * uniform53(w.v[0], w.v[1]);
    double px, py;
    if (kind == 0) {
        double sa, ca;
        sincos(az, &sa, &ca);
        px = p0 * ca;
        py = p0 * sa;
    } else {
        px = p0;
        py = 0.0;
    }
    r[kPx] = (T)px;
    r[kPy] = (T)py;
    P.px0[j] = (T)px; P.py0[j] = (T)py; P.pz0[j] = T(0);
    P.species[j] = species;
    // Gaussian complex matrix, columns orthonormalised in order
    double zr[3][3], zi[3][3];
#pragma unroll
    for (int k = 0; k < 9; k++) {
        U4 v = draw(seed, (uint32_t)i, (uint32_t)(2 + k), stream);
        double g0, g1;
        box_muller(v, g0, g1);
        zr[k / 3][k % 3] = g0;
        zi[k / 3][k % 3] = g1;
    }
    double ur[3][3], ui[3][3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        double vr[3], vi[3];
#pragma unroll
        for (int r = 0; r < 3; r++) { vr[r] = zr[r][c]; vi[r] = zi[r][c]; }
#pragma unroll
        for (int q = 0; q < c; q++) {
            // (u_q^dag v) u_q, modified Gram-Schmidt
            double dr = 0, di = 0;
#pragma unroll
            for (int r = 0; r < 3; r++) {
                dr += ur[r][q] * vr[r] + ui[r][q] * vi[r];
                di += ur[r][q] * vi[r] - ui[r][q] * vr[r];
            }
#pragma unroll
            for (int r = 0; r < 3; r++) {
                vr[r] -= dr * ur[r][q] - di * ui[r][q];
                vi[r] -= dr * ui[r][q] + di * ur[r][q];
            }
        }
        double nr = sqrt(vr[0] * vr[0] + vi[0] * vi[0] + vr[1] * vr[1] + vi[1] * vi[1] +
                         vr[2] * vr[2] + vi[2] * vi[2]);
#pragma unroll
        for (int r = 0; r < 3; r++) { ur[r][c] = vr[r] / nr; ui[r][c] = vi[r] / nr; }
    }
    // roots of l^3 - l - 5/18 = 0 (trigonometric form of the depressed cubic)
    const double qd[3] = {1.1174041524913475, -0.30659898226164492, -0.81080517022970258};
    // Q = U diag(qd) U^dag, hermitian; components x^a = 2 Re Tr(T^a Q)
    M3<double> Qm;
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            double sr = 0, si = 0;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                // U[r][k] qd[k] conj(U[c][k])
                sr += qd[k] * (ur[r][k] * ur[c][k] + ui[r][k] * ui[c][k]);
                si += qd[k] * (ui[r][k] * ur[c][k] - ur[r][k] * ui[c][k]);
            }
            Qm.re[r][c] = sr;
            Qm.im[r][c] = si;
        }
    double q[8];
    alg_from_herm(Qm, q);
#pragma unroll
    for (int a = 0; a < 8; a++) r[kQ + a] = (T)q[a];
#pragma unroll
    for (int k = 0; k < kPartRec<T>; k += 16 / (int)sizeof(T)) chunk_st16(P.st, (size_t)P.cap, (size_t)j, k, r + k);
}

// Per-species partial sums of the squared momenta at formation (p_x0^2,
// p_y0^2, p_z0^2, count) over the particles of each kPushBlock workgroup,
// with the push's fixed-order block reduction; the series reduction of
// these rows gives the sums the momentum series subtract.
template <typename T>
__global__ void __launch_bounds__(kPushBlock)
k_p0_sums(PartPtrs<T> P, int64_t n_slots, int n_species, double *__restrict__ partials) {
    const int64_t i = (int64_t)blockIdx.x * kPushBlock + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int s = -1;
    if (i < n_slots && P.species[i] >= 0) {
        s = P.species[i];
        const double x0 = P.px0[i], y0 = P.py0[i], z0 = P.pz0[i];
        acc[0] = x0 * x0;
        acc[1] = y0 * y0;
        acc[2] = z0 * z0;
        acc[3] = 1.0;
    }
    block_species_reduce(s, acc, n_species, partials + (size_t)blockIdx.x * n_species * 4);
}

template <typename T>
hipError_t launch_p0_sums(hipStream_t st, PartPtrs<T> p, int64_t n_slots, int n_species, double *partials,
                          double *out) {
    if (n_slots <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n_slots + kPushBlock - 1) / kPushBlock);
    hipLaunchKernelGGL(k_p0_sums<T>, dim3(blocks), dim3(kPushBlock), 0, st, p, n_slots, n_species, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_series_reduce(st, partials, (int)blocks, n_species, out, nullptr);
}

// per workgroup, over the particles (padding excluded): max |q2 - 4| and
// max |q3 - 10/3| of the Casimirs q2 = Q^aQ^a = 2 Tr Q^2 and
// q3 = d_abc Q^aQ^bQ^c = 4 Tr Q^3 (the f_abc part of Tr T^aT^bT^c cancels in
// the symmetric contraction), which Eq. (2) conserves
template <typename T>
__global__ void __launch_bounds__(256)
k_casimir(PartPtrs<T> P, int64_t n_slots, double *partials) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double v2 = 0.0, v3 = 0.0;
    if (i < n_slots && P.species[i] >= 0) {
        double q[8], q2 = 0.0;
#pragma unroll
        for (int a = 0; a < 8; a++) {
            q[a] = chunk_ld(P.st, (size_t)P.cap, (size_t)i, kQ + a);
            q2 += q[a] * q[a];
        }
        const M3<double> Qm = herm_from_alg(q);
        const double q3 = 4.0 * re_tr_mul(mul(Qm, Qm), Qm);
        v2 = fabs(q2 - 4.0);
        v3 = fabs(q3 - 10.0 / 3.0);
        if (!isfinite(v2)) v2 = 1e300;
        if (!isfinite(v3)) v3 = 1e300;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v2 = fmax(v2, __shfl_xor(v2, off, 64));
        v3 = fmax(v3, __shfl_xor(v3, off, 64));
    }
    __shared__ double red[2][4];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = v2;
        red[1][threadIdx.x >> 6] = v3;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int k = threadIdx.x;
        partials[2 * blockIdx.x + k] = fmax(fmax(red[k][0], red[k][1]), fmax(red[k][2], red[k][3]));
    }
}

template <typename T>
hipError_t launch_casimir(hipStream_t st, PartPtrs<T> p, int64_t n_slots, double *partials,
                          int *n_blocks_out) {
    unsigned blocks = (unsigned)((n_slots + 255) / 256);
    *n_blocks_out = (int)blocks;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_casimir<T>, dim3(blocks), dim3(256), 0, st, p, n_slots, partials);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256)
k_iota(int32_t *__restrict__ id, int64_t n, int64_t n_valid, int32_t base) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) id[i] = i < n_valid ? base + (int32_t)i : -1;
}

hipError_t launch_iota(hipStream_t st, int32_t *id, int64_t n, int64_t n_valid, int32_t base) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, id, n, n_valid, base);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_push(hipStream_t st, int N, PartPtrs<T> p, int64_t n_slots, FieldPtrs<T> f,
                       const T *F, SpeciesTab<T> tab, int n_species, int n, double dtau, double *partials,
                       const KernelTimer &kt) {
    if (n_slots <= 0) return timer_skip(st, kt);
    unsigned blocks = (unsigned)((n_slots + kPushBlock - 1) / kPushBlock);
    GL_LAUNCH_TIMED(kt, k_push<T>, dim3(blocks), dim3(kPushBlock), 0, st, N, p, n_slots, f, F, tab, n_species, n,
                    (T)dtau, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_push_permuted(hipStream_t st, int N, PartPtrs<T> p, PartPtrs<T> dst, const int32_t *perm,
                                const int32_t *id_src, int32_t *id_dst, int64_t n_slots, FieldPtrs<T> f,
                                const T *F, SpeciesTab<T> tab, int n_species, int n, double dtau,
                                double *partials, const KernelTimer &kt) {
    if (n_slots <= 0) return timer_skip(st, kt);
    unsigned blocks = (unsigned)((n_slots + kPushBlock - 1) / kPushBlock);
    GL_LAUNCH_TIMED(kt, k_push_permuted<T>, dim3(blocks), dim3(kPushBlock), 0, st, N, p, dst, perm, id_src, id_dst,
                    n_slots, f, F, tab, n_species, n, (T)dtau, partials);
    return hipGetLastError();
}

hipError_t launch_series_reduce(hipStream_t st, const double *partials, int n_blocks, int n_species,
                                double *row, const double *sub) {
    hipLaunchKernelGGL(k_series_reduce, dim3(kMaxSpecies), dim3(256), 0, st, partials, n_blocks,
                       n_species, sub, row, (size_t)0);
    return hipGetLastError();
}

hipError_t launch_series_reduce_steps(hipStream_t st, const double *partials, size_t slot_stride, int n_rows,
                                      int n_blocks, int n_species, double *row, const double *sub) {
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_series_reduce, dim3(kMaxSpecies, n_rows), dim3(256), 0, st, partials, n_blocks,
                       n_species, sub, row, slot_stride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_particles_init(hipStream_t st, int N, PartPtrs<T> p, int64_t slot0, int64_t n,
                                 uint64_t seed, int species_id, int kind, double p0) {
    if (n <= 0) return hipSuccess;
    unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_particles_init<T>, dim3(blocks), dim3(256), 0, st, N, p, slot0, n, seed,
                       species_id, kind, p0);
    return hipGetLastError();
}

#define GL_INST(T)                                                                               \
    template hipError_t launch_push<T>(hipStream_t, int, PartPtrs<T>, int64_t, FieldPtrs<T>,      \
                                       const T *, SpeciesTab<T>, int, int, double, double *,     \
                                       const KernelTimer &);                                     \
    template hipError_t launch_push_permuted<T>(hipStream_t, int, PartPtrs<T>, PartPtrs<T>,       \
                                                const int32_t *, const int32_t *, int32_t *,     \
                                                int64_t, FieldPtrs<T>, const T *, SpeciesTab<T>, \
                                                int, int, double, double *, const KernelTimer &); \
    template hipError_t launch_particles_init<T>(hipStream_t, int, PartPtrs<T>, int64_t, int64_t, \
                                                 uint64_t, int, int, double);                    \
    template hipError_t launch_casimir<T>(hipStream_t, PartPtrs<T>, int64_t, double *, int *);             \
    template hipError_t launch_p0_sums<T>(hipStream_t, PartPtrs<T>, int64_t, int, double *, double *);
GL_INST(double)
GL_INST(float)
#undef GL_INST

}  // namespace gl
