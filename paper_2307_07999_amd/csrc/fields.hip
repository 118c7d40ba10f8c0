// fields.hip -- the boost-invariant leapfrog of the classical Yang-Mills
// equations (Eq. (1)) on transverse links, the local-frame site fields the
// particles read, and the field diagnostics.
//
// Lattice Hamiltonian per unit rapidity (a = 1, g absorbed), Milne time tau:
//   H = sum_x [ sum_i Tr E_i^2 / tau + tau Tr pi^2
//               + sum_i Tr (Phi_{+i} - phi)^2 / tau + 2 tau (3 - Re Tr P) ]
// with E_i = tau dA_i/dtau, phi = A_eta, pi = (1/tau) dA_eta/dtau,
// P(x) = U_1(x) U_2(x+1) U_1^dag(x+2) U_2^dag(x) and
// Phi_{+i}(x) = U_i(x) phi(x+i) U_i^dag(x), Phi_{-i}(x) = U_i^dag(x-i) phi(x-i) U_i(x-i).
// One step (E, pi at half steps, U, phi at integer steps):
//   E_1 += dtau { -tau ([P(x)]_X - U_2^dag(x-2)[P(x-2)]_X U_2(x-2)) - (i/tau)[phi, Phi_{+1}] }
//   E_2 += dtau { -tau (U_1^dag(x-1)[P(x-1)]_X U_1(x-1) - [P(x)]_X) - (i/tau)[phi, Phi_{+2}] }
//   pi  += (dtau/tau) sum_i (Phi_{+i} + Phi_{-i} - 2 phi)
//   U_i <- exp(i dtau E_i / tau_{n+1/2}) U_i,   phi += dtau tau_{n+1/2} pi
// This scheme keeps the Gauss law sum_i [E_i(x) - U_i^dag(x-i)E_i(x-i)U_i(x-i)]
// + i[phi, pi] exactly constant.
//
// Kernel design: two lanes per site, one per link direction (the per-site
// work of one lane needs too many registers for more than one wave per SIMD);
// workgroups of 32 x 4 sites.  The links and phi of the tile and a one-site
// halo are staged in LDS with coalesced 16-byte reads of the chunked field
// state, and every neighbour of the stencil is read from there: without the
// tile the step issues ~250 global loads per lane and its waves spend half
// their time waiting on them.  Tiles are numbered so that each XCD owns one
// band of rows (xcd_remap): the neighbour reads of the stencil then hit the
// L2 of the XCD that owns the tile instead of refetching halo lines from
// memory.
#include <algorithm>

#include "fields_dev.hpp"

namespace gl {

constexpr int TX = 32, TY = 8;     // site tiles of the diagnostics
constexpr int SX = 32, SY = 4;     // site tiles of the step: 2 lanes per site

// FP64: two waves per SIMD at the cost of a few spilled registers is faster
// than one wave with everything in registers.
template <typename T>
__global__ void __launch_bounds__(2 * SX * SY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 2 : 4, 8)))
k_field_step(int N, FieldPtrs<T> in, FieldPtrs<T> out, T *__restrict__ F, T tau, T dtau, T tau_h, int reunit) {
    __shared__ LinkTile<T, SX, SY> tile;
    const int tx = (N + SX - 1) / SX;
    const int l = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (l % tx) * SX, y0 = (l / tx) * SY;
    const int lx = threadIdx.x >> 1, ly = threadIdx.y;
    const int tid = threadIdx.x + 2 * SX * threadIdx.y;
    stage_tile(tile, N, in, x0, y0, tid, 2 * SX * SY);
    __syncthreads();
    // every thread takes part (the step synchronises the workgroup); both
    // lanes of a pair are on or off the lattice together
    const bool active = x0 + lx < N && y0 + ly < N;
    field_step_link(tile, N, in, out, F, x0, y0, lx, ly, threadIdx.x & 1, tid, active, tau, dtau, tau_h, reunit);
}

// Static quarks (Sec. 2, Eq. (4)): I_i^a(x) += dtau E_i^a(x, tau_n) from the
// site fields at tau_n (E_x and E_y adding the half stored apart where
// half_stored holds), FP64, and
// per workgroup the sums over its sites of (1/2) sum_a (I_i^a)^2 for
// i = x, y, z with the site count, added in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256)
k_static_accum(int N, const T *__restrict__ F, double *__restrict__ I, double dtau, double *__restrict__ partials) {
    __shared__ double red[4][256];
    const size_t n2 = plane_pitch(N);
    const size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (x < (size_t)N * N) {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 8; a++) {
                double e = (double)chunk_ld(F, n2, x, 8 * i + a);
                if (i < 2 && half_stored(i, (int)(x % N), (int)(x / N)))
                    e += (double)chunk_ld(F, n2, x, 48 + 8 * i + a);
                const double t = pl_ld(I, n2, 8 * i + a, x) + dtau * e;
                pl_st(I, n2, 8 * i + a, x, t);
                s += t * t;
            }
            v[i] = 0.5 * s;
        }
        v[3] = 1.0;
    }
#pragma unroll
    for (int k = 0; k < 4; k++) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < 4; k++) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[(size_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// Lightlike jets (Sec. 2, Eq. (5)): one jet per start site x0, step j since
// its start; it sits in the cell x0 + floor(j dtau + 1/2) along x and feels
// F_x = E_x, F_y = E_y - B_z, F_z = E_z + B_y there (site fields at tau_n),
// transported to its start with W (FP64): I_i += dtau [W F_i W^dag]; when
// this step's drift ends in the next cell, W <- W U_x(cell) with the links of
// tau_n.  Per workgroup: sums of (1/2) sum_a (I_i^a)^2 and the site count.
template <typename T>
__global__ void __launch_bounds__(256)
k_lightlike_accum(int N, const T *__restrict__ F, const T *__restrict__ U, double *__restrict__ W,
                  double *__restrict__ I, int64_t j, double dtau, double *__restrict__ partials) {
    __shared__ double red[4][256];
    const size_t n2 = plane_pitch(N);
    const size_t x0 = (size_t)blockIdx.x * 256 + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (x0 < (size_t)N * N) {
        const int64_t shift = (int64_t)floor((double)j * dtau + 0.5);
        const int ix = (int)(((int64_t)(x0 % N) + shift) % N), iy = (int)(x0 / N);
        const size_t c = (size_t)ix + (size_t)N * iy;
        M3<double> w = load_m(W, n2, x0);
#pragma unroll
        for (int i = 0; i < 3; i++) {
            double f[8], t[8];
#pragma unroll
            for (int a = 0; a < 8; a++) {
                if (i == 0)
                    f[a] = (double)chunk_ld(F, n2, c, a) +
                           (half_stored(0, ix, iy) ? (double)chunk_ld(F, n2, c, 48 + a) : 0.0);
                else if (i == 1)
                    f[a] = ((double)chunk_ld(F, n2, c, 8 + a) +
                            (half_stored(1, ix, iy) ? (double)chunk_ld(F, n2, c, 56 + a) : 0.0)) -
                           (double)chunk_ld(F, n2, c, 40 + a);
                else f[a] = (double)chunk_ld(F, n2, c, 16 + a) + (double)chunk_ld(F, n2, c, 32 + a);
            }
            transport_nd(w, f, t);
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 8; a++) {
                const double q = pl_ld(I, n2, 8 * i + a, x0) + dtau * t[a];
                pl_st(I, n2, 8 * i + a, x0, q);
                s += q * q;
            }
            v[i] = 0.5 * s;
        }
        v[3] = 1.0;
        if ((int64_t)floor((double)(j + 1) * dtau + 0.5) > shift) {
            const M3<T> u = chunk_load_link(U, n2, c, 0);
            M3<double> ud;
#pragma unroll
            for (int r = 0; r < 3; r++)
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    ud.re[r][q] = (double)u.re[r][q];
                    ud.im[r][q] = (double)u.im[r][q];
                }
            store_m(W, n2, x0, mul(w, ud));
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w2 = 128; w2 > 0; w2 >>= 1) {
        if (threadIdx.x < w2)
#pragma unroll
            for (int k = 0; k < 4; k++) red[k][threadIdx.x] += red[k][threadIdx.x + w2];
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[(size_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// Diagnostics per site, reduced per workgroup in FP64:
// [0] max |G^a|, [1] max |E^a|, [2] max |U U^dag - 1|, [3..6] energy terms,
// [7] non-finite count.
constexpr int kDiagVals = 8;

template <typename T>
__global__ void __launch_bounds__(TX *TY)
k_diag(int N, FieldPtrs<T> f, T tau, double *__restrict__ partials) {
    __shared__ double red[kDiagVals][TX * TY];
    int tid = threadIdx.x + TX * threadIdx.y;
    int ix = blockIdx.x * TX + threadIdx.x;
    int iy = blockIdx.y * TY + threadIdx.y;
    double v[kDiagVals] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (ix < N && iy < N) {
        const size_t n2 = (size_t)N * N;
        Nbr nb = neighbours(ix, iy, N);
        M3<T> u1x = chunk_load_link(f.U, n2, nb.x, 0), u2x = chunk_load_link(f.U, n2, nb.x, 1);
        T e1[8], e2[8], e1m[8], e2m[8], ph[8], p[8];
        chunk_load_a(f.E, n2, nb.x, 0, e1);
        chunk_load_a(f.E, n2, nb.x, 8, e2);
        chunk_load_a(f.E, n2, nb.xm1, 0, e1m);
        chunk_load_a(f.E, n2, nb.xm2, 8, e2m);
        chunk_load_a(f.phi, n2, nb.x, 0, ph);
        chunk_load_a(f.pi, n2, nb.x, 0, p);
        M3<T> u1m = chunk_load_link(f.U, n2, nb.xm1, 0), u2m = chunk_load_link(f.U, n2, nb.xm2, 1);
        T t1[8], t2[8];
        transport_dn(u1m, e1m, t1);
        transport_dn(u2m, e2m, t2);
        M3<T> PH = herm_from_alg(ph), PI = herm_from_alg(p);
        M3<T> c = sub(mul(PH, PI), mul(PI, PH));   // [phi, pi]; i[phi,pi] hermitian
        M3<T> ic;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) { ic.re[i][j] = -c.im[i][j]; ic.im[i][j] = c.re[i][j]; }
        T g[8];
        alg_from_herm(ic, g);
        double gmax = 0, emax = 0, et = 0, el = 0, bt = 0;
        int bad = 0;
#pragma unroll
        for (int a = 0; a < 8; a++) {
            double ga = (double)e1[a] - (double)t1[a] + (double)e2[a] - (double)t2[a] + (double)g[a];
            gmax = fmax(gmax, fabs(ga));
            emax = fmax(emax, fmax(fabs((double)e1[a]), fabs((double)e2[a])));
            et += 0.5 * ((double)e1[a] * e1[a] + (double)e2[a] * e2[a]);
            el += 0.5 * (double)p[a] * p[a];
            if (!isfinite((double)e1[a]) || !isfinite((double)e2[a]) || !isfinite((double)ph[a]) ||
                !isfinite((double)p[a]))
                bad++;
        }
        double umax = 0;
        M3<T> uu[2] = {u1x, u2x};
#pragma unroll
        for (int d = 0; d < 2; d++) {
            M3<T> w = mul_nd(uu[d], uu[d]);
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    double dr = (double)w.re[i][j] - (i == j ? 1.0 : 0.0);
                    umax = fmax(umax, fmax(fabs(dr), fabs((double)w.im[i][j])));
                    if (!isfinite((double)uu[d].re[i][j]) || !isfinite((double)uu[d].im[i][j])) bad++;
                }
        }
        // B_T: sum_i Tr(Phi_{+i} - phi)^2
        M3<T> ups[2] = {u1x, u2x};
        size_t xps[2] = {nb.xp1, nb.xp2};
#pragma unroll
        for (int d = 0; d < 2; d++) {
            T v2[8];
            chunk_load_a(f.phi, n2, xps[d], 0, v2);
            M3<T> Pf = mul_nd(mul(ups[d], herm_from_alg(v2)), ups[d]);
            T df[8];
            alg_from_herm(Pf, df);
#pragma unroll
            for (int a = 0; a < 8; a++) {
                double dd = (double)df[a] - (double)ph[a];
                bt += 0.5 * dd * dd;
            }
        }
        M3<T> P = plaq(u1x, chunk_load_link(f.U, n2, nb.xp1, 1), chunk_load_link(f.U, n2, nb.xp2, 0), u2x);
        double bl = 3.0 - ((double)P.re[0][0] + (double)P.re[1][1] + (double)P.re[2][2]);
        v[0] = gmax;
        v[1] = emax;
        v[2] = umax;
        v[3] = et / (double)tau;
        v[4] = el * (double)tau;
        v[5] = bt / (double)tau;
        v[6] = 2.0 * (double)tau * bl;
        v[7] = bad;
    }
#pragma unroll
    for (int k = 0; k < kDiagVals; k++) red[k][tid] = v[k];
    __syncthreads();
    for (int s = TX * TY / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int k = 0; k < kDiagVals; k++) {
                double a = red[k][tid], b = red[k][tid + s];
                red[k][tid] = (k < 3) ? fmax(a, b) : a + b;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        size_t blk = blockIdx.x + (size_t)gridDim.x * blockIdx.y;
#pragma unroll
        for (int k = 0; k < kDiagVals; k++) partials[blk * kDiagVals + k] = red[k][0];
    }
}

// Failure detection: values [0, n) of a flat array, grouped in steps of
// vals_per_step consecutive values (step step0 + i / vals_per_step), are
// tested for NaN and Inf, and a lane holding one lowers *first_bad to its
// step.  Grid-stride; one 16-byte vector of V values per lane and pass.
template <typename V, typename T, int NV>
__global__ void __launch_bounds__(256)
k_check_finite(const T *__restrict__ a, int64_t n, int64_t vals_per_step, int step0, int *first_bad) {
    const int64_t nv = n / NV;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nv; v += stride) {
        const V w = reinterpret_cast<const V *>(a)[v];
        const T *e = reinterpret_cast<const T *>(&w);
        bool bad = false;
#pragma unroll
        for (int k = 0; k < NV; k++) bad |= !isfinite(e[k]);
        if (bad) atomicMin(first_bad, step0 + (int)(v * NV / vals_per_step));
    }
    // a tail shorter than one vector
    const int64_t t = nv * NV + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n && !isfinite(a[t])) atomicMin(first_bad, step0 + (int)(t / vals_per_step));
}

template <typename T>
hipError_t launch_check_finite(hipStream_t st, const T *a, int64_t n, int64_t vals_per_step, int step0,
                               int *first_bad) {
    if (n <= 0) return hipSuccess;
    constexpr int NV = 16 / (int)sizeof(T);
    const int64_t blocks = std::min<int64_t>(2048, std::max<int64_t>(1, (n / NV + 255) / 256));
    if (sizeof(T) == 8)
        hipLaunchKernelGGL((k_check_finite<double2, double, 2>), dim3((unsigned)blocks), dim3(256), 0, st,
                           (const double *)a, n, vals_per_step, step0, first_bad);
    else
        hipLaunchKernelGGL((k_check_finite<float4, float, 4>), dim3((unsigned)blocks), dim3(256), 0, st,
                           (const float *)a, n, vals_per_step, step0, first_bad);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_field_step(hipStream_t st, int N, FieldPtrs<T> in, FieldPtrs<T> out, T *F, double tau,
                             double dtau, int reunit, const KernelTimer &kt) {
    dim3 grid(((N + SX - 1) / SX) * ((N + SY - 1) / SY)), block(2 * SX, SY);
    GL_LAUNCH_TIMED(kt, k_field_step<T>, grid, block, 0, st, N, in, out, F, (T)tau, (T)dtau, (T)(tau + 0.5 * dtau),
                    reunit);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_static_accum(hipStream_t st, int N, const T *F, double *I, double dtau, double *partials,
                               int *n_blocks_out) {
    const int nb = (int)(((size_t)N * N + 255) / 256);
    *n_blocks_out = nb;
    hipLaunchKernelGGL(k_static_accum<T>, dim3(nb), dim3(256), 0, st, N, F, I, dtau, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lightlike_accum(hipStream_t st, int N, const T *F, const T *U, double *W, double *I, int64_t j,
                                  double dtau, double *partials, int *n_blocks_out) {
    const int nb = (int)(((size_t)N * N + 255) / 256);
    *n_blocks_out = nb;
    hipLaunchKernelGGL(k_lightlike_accum<T>, dim3(nb), dim3(256), 0, st, N, F, U, W, I, j, dtau, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diag(hipStream_t st, int N, FieldPtrs<T> f, double tau, double *partials,
                       int *n_blocks_out) {
    dim3 grid((N + TX - 1) / TX, (N + TY - 1) / TY), block(TX, TY);
    *n_blocks_out = (int)(grid.x * grid.y);
    hipLaunchKernelGGL(k_diag<T>, grid, block, 0, st, N, f, (T)tau, partials);
    return hipGetLastError();
}

#define GL_INST(T)                                                                           \
    template hipError_t launch_field_step<T>(hipStream_t, int, FieldPtrs<T>, FieldPtrs<T>, T *,    \
                                             double, double, int, const KernelTimer &);      \
    template hipError_t launch_diag<T>(hipStream_t, int, FieldPtrs<T>, double, double *, int *);     \
    template hipError_t launch_check_finite<T>(hipStream_t, const T *, int64_t, int64_t, int, int *);   \
    template hipError_t launch_static_accum<T>(hipStream_t, int, const T *, double *, double, double *, int *); \
    template hipError_t launch_lightlike_accum<T>(hipStream_t, int, const T *, const T *, double *, double *, \
                                                  int64_t, double, double *, int *);
// the FP64 instantiations come from fields_f64.hip, which includes this file
// and is compiled with its own scheduling flag
#ifdef GL_FIELDS_FP64
GL_INST(double)
#else
GL_INST(float)
#endif
#undef GL_INST

}  // namespace gl
