// init.hip -- MV-model initial conditions of the Glasma (Sec. 1, "Glasma"),
// computed in FP64 on the device:
//   1. Gaussian color charges rho^a per (nucleus, sheet, site) from Philox,
//      packed two colors per complex plane (rho^{2j} + i rho^{2j+1}).
//   2. Poisson solve (-Lap + m^2) Lambda = rho with the 5-point Laplacian,
//      exact in Fourier space: 2-D FFT by LDS-resident mixed-radix (8, 4, 2, 3)
//      Stockham line transforms, several adjacent lines per workgroup; the
//      kernel multiplication sits between the forward and inverse column
//      transforms of one pass.  The kernel is real and even, so the packed
//      pair separates again after the inverse.  Sheets are processed in
//      chunks (charges, transforms and the Wilson-line products of a chunk
//      in one launch each).
//   3. Wilson lines V = prod_s exp(-i Lambda_s), sheet 1 leftmost.
//   4. Matching of the nuclei's pure-gauge links U^n_i(x) = V_n(x) V_n^dag(x+i)
//      to the forward light cone: [(U^A + U^B)(1 + U^dag)]_X = 0 per link by
//      damped Newton with the analytic Jacobian J_ab = -2 Re Tr(T^a W U^dag T^b),
//      started from the SU(3) projection of W (W^dag)^{-1}, W = U^A + U^B.
//   5. pi0(x) = 1/2 sum_i { [(U_i(x) - 1)(U^B_i(x)^dag - U^A_i(x)^dag)]_X
//                         + [(U_i(x-i)^dag - 1)(U^B_i(x-i) - U^A_i(x-i))]_X },
//      and the first half step E^{1/2} = 0, pi^{1/2} = pi0, U^1 = U^0,
//      phi^1 = dtau * tau_{1/2} * pi0.
#include "internal.hpp"
#include "philox.hpp"
#include "su3.hpp"

namespace gl {

// ---- 1. charges ---------------------------------------------------------------
// colours 2j, 2j + 1 of the charge of one sheet at site x: one counter-based
// draw, two normal deviates, scaled by sigma
__device__ __forceinline__ double2 mv_charge_pair(const MvDraw &mv, int sheet, int j, size_t x) {
    U4 w = draw(mv.seed, (uint32_t)x, (uint32_t)(4 * sheet + j), (uint32_t)mv.nucleus);
    double g0, g1;
    box_muller(w, g0, g1);
    return make_double2(mv.sigma * g0, mv.sigma * g1);
}

// sheets sheet0 + blockIdx.y of one nucleus into planes [sheet][4][n2]
__global__ void __launch_bounds__(256)
k_mv_charges(int N, MvDraw mv, double2 *planes) {
    size_t n2 = (size_t)N * N;
    size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (x >= n2) return;
    const int sheet = mv.sheet0 + (int)blockIdx.y;
    double2 *pl = planes + (size_t)blockIdx.y * 4 * n2;
#pragma unroll
    for (int j = 0; j < 4; j++) pl[(size_t)j * n2 + x] = mv_charge_pair(mv, sheet, j, x);
}

__global__ void __launch_bounds__(256)
k_pack(int N, const double *rho, double2 *planes) {
    size_t n2 = (size_t)N * N;
    size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (x >= n2) return;
#pragma unroll
    for (int j = 0; j < 4; j++)
        planes[(size_t)j * n2 + x] = make_double2(rho[(size_t)(2 * j) * n2 + x], rho[(size_t)(2 * j + 1) * n2 + x]);
}

__global__ void __launch_bounds__(256)
k_unpack(int N, const double2 *planes, double *rho) {
    size_t n2 = (size_t)N * N;
    size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (x >= n2) return;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        double2 v = planes[(size_t)j * n2 + x];
        rho[(size_t)(2 * j) * n2 + x] = v.x;
        rho[(size_t)(2 * j + 1) * n2 + x] = v.y;
    }
}

// ---- 2. FFT ------------------------------------------------------------------
constexpr int kFftThreads = 256;
constexpr int kFftMaxN = 1024;
constexpr int kFftElems = 2048;   // complex values per workgroup: C lines of N

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// radix sequence of N: n8 radix-8 stages, then n4 (0 or 1) radix-4, n2 (0
// or 1) radix-2, then n3 radix-3 (N = 2^a 3^b)
struct Radices {
    int n8, n4, n2, n3;
};

__host__ __device__ inline bool radices_of(int N, Radices &rs) {
    rs.n8 = rs.n4 = rs.n2 = rs.n3 = 0;
    int m = N;
    while (m % 8 == 0) { rs.n8++; m /= 8; }
    while (m % 4 == 0) { rs.n4++; m /= 4; }
    while (m % 2 == 0) { rs.n2++; m /= 2; }
    while (m % 3 == 0) { rs.n3++; m /= 3; }
    return m == 1;
}

// lines per workgroup: the largest power of two that divides N, keeps C N
// within kFftElems and is at most 64
static inline int fft_lines_per_group(int N) {
    int C = 1;
    while (C < 64 && N % (2 * C) == 0 && 2 * C * N <= kFftElems) C *= 2;
    return C;
}

// radix-R butterfly of v (twiddled inputs), sign = -1 forward, +1 inverse
template <int R>
__device__ __forceinline__ void butterfly(const double2 *v, double2 *o, int sign) {
    if constexpr (R == 2) {
        o[0] = make_double2(v[0].x + v[1].x, v[0].y + v[1].y);
        o[1] = make_double2(v[0].x - v[1].x, v[0].y - v[1].y);
    } else if constexpr (R == 4) {
        double2 a = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
        double2 b = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
        double2 c = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
        double2 d = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
        double2 di = make_double2(-sign * d.y, sign * d.x);   // sign * i * d
        o[0] = make_double2(a.x + c.x, a.y + c.y);
        o[2] = make_double2(a.x - c.x, a.y - c.y);
        o[1] = make_double2(b.x + di.x, b.y + di.y);
        o[3] = make_double2(b.x - di.x, b.y - di.y);
    } else if constexpr (R == 8) {
        // even and odd halves as radix-4 transforms, joined by
        // t_k = exp(sign i pi k / 4): o[k] = E[k] + t_k O[k], o[k+4] = E[k] - t_k O[k]
        const double h = 0.70710678118654752440;
        const double2 ve[4] = {v[0], v[2], v[4], v[6]}, vo[4] = {v[1], v[3], v[5], v[7]};
        double2 E[4], O[4];
        butterfly<4>(ve, E, sign);
        butterfly<4>(vo, O, sign);
        const double2 t1 = make_double2(h * (O[1].x - sign * O[1].y), h * (O[1].y + sign * O[1].x));
        const double2 t2 = make_double2(-sign * O[2].y, sign * O[2].x);
        const double2 t3 = make_double2(-h * (O[3].x + sign * O[3].y), h * (sign * O[3].x - O[3].y));
        o[0] = make_double2(E[0].x + O[0].x, E[0].y + O[0].y);
        o[4] = make_double2(E[0].x - O[0].x, E[0].y - O[0].y);
        o[1] = make_double2(E[1].x + t1.x, E[1].y + t1.y);
        o[5] = make_double2(E[1].x - t1.x, E[1].y - t1.y);
        o[2] = make_double2(E[2].x + t2.x, E[2].y + t2.y);
        o[6] = make_double2(E[2].x - t2.x, E[2].y - t2.y);
        o[3] = make_double2(E[3].x + t3.x, E[3].y + t3.y);
        o[7] = make_double2(E[3].x - t3.x, E[3].y - t3.y);
    } else {   // R == 3
        const double c3 = -0.5, s3 = 0.86602540378443864676 * sign;
        double2 t = make_double2(v[1].x + v[2].x, v[1].y + v[2].y);
        double2 u = make_double2(v[1].x - v[2].x, v[1].y - v[2].y);
        o[0] = make_double2(v[0].x + t.x, v[0].y + t.y);
        double2 m = make_double2(v[0].x + c3 * t.x, v[0].y + c3 * t.y);
        double2 iu = make_double2(-s3 * u.y, s3 * u.x);   // s3 * i * u
        o[1] = make_double2(m.x + iu.x, m.y + iu.y);
        o[2] = make_double2(m.x - iu.x, m.y - iu.y);
    }
}

// One Stockham stage of radix R on the C lines of N values in buf (in place:
// every thread reads its butterflies into registers, the workgroup
// synchronises, then the results are written).  Twiddle of (r, k) is
// tw[r k N / (Ns R)].
template <int R>
__device__ __forceinline__ void fft_stage(double2 *buf, const double2 *tw, int N, int C, int Ns, int sign) {
    // tw holds exp(-2 pi i j / N); the inverse uses its conjugate
    constexpr int B = (kFftElems / R + kFftThreads - 1) / kFftThreads;   // butterflies per thread
    const int nb = N / R, step = N / (Ns * R), total = C * nb;
    double2 o[B][R];
    int at[B];
#pragma unroll
    for (int b = 0; b < B; b++) {
        const int t = threadIdx.x + b * kFftThreads;
        at[b] = -1;
        if (t < total) {
            const int line = t / nb, j = t % nb, k = j % Ns;
            const double2 *in = buf + line * N;
            double2 v[R];
#pragma unroll
            for (int r = 0; r < R; r++) v[r] = in[j + r * nb];
#pragma unroll
            for (int r = 1; r < R; r++) {
                double2 w = tw[r * k * step];
                if (sign > 0) w.y = -w.y;
                v[r] = cmul(v[r], w);
            }
            butterfly<R>(v, o[b], sign);
            at[b] = line * N + (j / Ns) * Ns * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; b++)
        if (at[b] >= 0)
#pragma unroll
            for (int r = 0; r < R; r++) buf[at[b] + r * Ns] = o[b][r];
    __syncthreads();
}

__device__ __forceinline__ void fft_stages(double2 *buf, const double2 *tw, int N, int C, int sign, Radices rs) {
    int Ns = 1;
    for (int s = 0; s < rs.n8; s++, Ns *= 8) fft_stage<8>(buf, tw, N, C, Ns, sign);
    for (int s = 0; s < rs.n4; s++, Ns *= 4) fft_stage<4>(buf, tw, N, C, Ns, sign);
    for (int s = 0; s < rs.n2; s++, Ns *= 2) fft_stage<2>(buf, tw, N, C, Ns, sign);
    for (int s = 0; s < rs.n3; s++, Ns *= 3) fft_stage<3>(buf, tw, N, C, Ns, sign);
}

// Tables of one solve, filled once: tw[j] = exp(-2 pi i j / N) and
// s2[j] = 4 sin^2(pi j / N), j < N.
__global__ void __launch_bounds__(256)
k_fft_tables(int N, double2 *__restrict__ tw, double *__restrict__ s2) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    double sn, cs;
    sincospi(2.0 * (double)j / (double)N, &sn, &cs);
    tw[j] = make_double2(cs, -sn);
    const double h = sinpi((double)j / (double)N);
    s2[j] = 4.0 * h * h;
}

// In-place transforms of the N x N planes: each workgroup transforms C
// adjacent lines of one plane (rows if cols == 0, columns otherwise), with
// the twiddles exp(-2 pi i j / N) copied from the solve's table into LDS.  Loads
// and stores walk the C lines together, so a column workgroup reads C
// consecutive values of each row.  sign = -1 forward, +1 inverse
// (unnormalised).  MODE kFftPoisson (columns only, after the forward row
// pass): the forward column transform, the multiplication of mode (kx, ky)
// by 1 / (N^2 (4 sin^2(pi kx/N) + 4 sin^2(pi ky/N) + m2)) (zero above
// uv2 > 0) and the inverse column transform, in one pass.  MODE kFftDraw
// (forward rows): the input lines are the MV charges, drawn here instead of
// being written to the planes by a pass of their own and read back.
constexpr int kFftLines = 0, kFftPoisson = 1, kFftDraw = 2;
template <int MODE>
__global__ void __launch_bounds__(kFftThreads)
k_fft_lines(double2 *data, int N, int C, int cols, size_t plane_stride, int groups_per_plane, int sign,
            Radices rs, double m2, double uv2, const double2 *__restrict__ tw_tab, const double *__restrict__ s2_tab,
            MvDraw mv) {
    constexpr bool POISSON = MODE == kFftPoisson;
    // dynamic LDS sized for this N: the lines, then tw[N], then (POISSON) s2[N]
    extern __shared__ double2 lds[];
    double2 *buf = lds, *tw = lds + kFftElems;
    double *s2 = (double *)(tw + N);
    // contiguous runs of groups per XCD: the C-wide column segments of
    // neighbouring groups share cache lines, which then meet in one L2
    const int bid = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int g = bid % groups_per_plane, plane = bid / groups_per_plane;
    double2 *base = data + (size_t)plane * plane_stride;
    const int l0 = g * C;
    for (int j = threadIdx.x; j < N; j += kFftThreads) {
        tw[j] = tw_tab[j];
        if (POISSON) s2[j] = s2_tab[j];
    }
    for (int i = threadIdx.x; i < C * N; i += kFftThreads) {
        const int line = cols ? i % C : i / N, k = cols ? i / C : i % N;
        const size_t addr = cols ? (size_t)k * N + (l0 + line) : (size_t)(l0 + line) * N + k;
        if constexpr (MODE == kFftDraw) buf[line * N + k] = mv_charge_pair(mv, mv.sheet0 + plane / 4, plane % 4, addr);
        else buf[line * N + k] = base[addr];
    }
    __syncthreads();
    if (POISSON) {
        fft_stages(buf, tw, N, C, -1, rs);
        const double nn = (double)N * (double)N;
        for (int i = threadIdx.x; i < C * N; i += kFftThreads) {
            const int line = i / N, k = i % N;   // kx = l0 + line, ky = k
            const double k2 = s2[l0 + line] + s2[k];
            const double gk = (uv2 > 0.0 && k2 > uv2) ? 0.0 : 1.0 / (nn * (k2 + m2));
            buf[i] = make_double2(buf[i].x * gk, buf[i].y * gk);
        }
        __syncthreads();
        fft_stages(buf, tw, N, C, +1, rs);
    } else {
        fft_stages(buf, tw, N, C, sign, rs);
    }
    for (int i = threadIdx.x; i < C * N; i += kFftThreads) {
        const int line = cols ? i % C : i / N, k = cols ? i / C : i % N;
        const size_t addr = cols ? (size_t)k * N + (l0 + line) : (size_t)(l0 + line) * N + k;
        base[addr] = buf[line * N + k];
    }
}

// ---- 3. Wilson lines --------------------------------------------------------
__global__ void __launch_bounds__(256)
k_wilson_init(int N, double *V) {
    size_t n2 = (size_t)N * N;
    size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (x >= n2) return;
    store_m(V, n2, x, m_ident<double>());
}

// V <- V exp(-i Lambda_s) for the n_sheets sheets of planes [sheet][4][n2], in
// sheet order (earlier sheets to the left)
__global__ void __launch_bounds__(256)
k_wilson_accum(int N, const double2 *planes, int n_sheets, double *V) {
    size_t n2 = (size_t)N * N;
    size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (x >= n2) return;
    M3<double> v = load_m(V, n2, x);
    for (int s = 0; s < n_sheets; s++) {
        double lam[8];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            double2 p = planes[((size_t)s * 4 + j) * n2 + x];
            lam[2 * j] = p.x;
            lam[2 * j + 1] = p.y;
        }
        v = mul(v, expi_alg(lam, -1.0));
    }
    store_m(V, n2, x, v);
}

// ---- dipole correlator (calibration of Q_s) -----------------------------------
// Workgroup (b, r): sum over its 256 sites of
// Re Tr V(x) V^dag(x + r e_x) + Re Tr V(x) V^dag(x + r e_y); partials [r][b]
__global__ void __launch_bounds__(256)
k_dipole(int N, const double *__restrict__ V, double *__restrict__ partials) {
    __shared__ double red[256];
    const size_t n2 = (size_t)N * N;
    const size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    double v = 0.0;
    if (x < n2) {
        const int ix = (int)(x % N), iy = (int)(x / N);
        const M3<double> a = load_m(V, n2, x);
        const size_t nb[2] = {(size_t)((ix + r) % N) + (size_t)N * iy, (size_t)ix + (size_t)N * ((iy + r) % N)};
#pragma unroll
        for (int d = 0; d < 2; d++) {
            const M3<double> b = load_m(V, n2, nb[d]);
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) v += a.re[i][j] * b.re[i][j] + a.im[i][j] * b.im[i][j];
        }
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[(size_t)r * gridDim.x + blockIdx.x] = red[0];
}

// D[r] = (sum of the partials of r in a fixed order) / (6 N^2)
__global__ void __launch_bounds__(256)
k_dipole_reduce(int N, const double *__restrict__ partials, int nb, double *__restrict__ D) {
    __shared__ double red[256];
    const int r = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) v += partials[(size_t)r * nb + b];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) D[r] = red[0] / (6.0 * (double)N * (double)N);
}

// ---- 4. matching ------------------------------------------------------------
__device__ inline void cdiv(double ar, double ai, double br, double bi, double &cr, double &ci) {
    double d = br * br + bi * bi;
    cr = (ar * br + ai * bi) / d;
    ci = (ai * br - ar * bi) / d;
}

__device__ inline void det3(const M3<double> &a, double &dr, double &di) {
    auto cm = [](double xr, double xi, double yr, double yi, double &zr, double &zi) {
        zr = xr * yr - xi * yi;
        zi = xr * yi + xi * yr;
    };
    double r = 0, i = 0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        double m1r, m1i, m2r, m2i;
        cm(a.re[1][c1], a.im[1][c1], a.re[2][c2], a.im[2][c2], m1r, m1i);
        cm(a.re[1][c2], a.im[1][c2], a.re[2][c1], a.im[2][c1], m2r, m2i);
        double cofr = m1r - m2r, cofi = m1i - m2i;
        double tr, ti;
        cm(a.re[0][c], a.im[0][c], cofr, cofi, tr, ti);
        r += tr;
        i += ti;
    }
    dr = r;
    di = i;
}

// inverse by cofactors
__device__ inline M3<double> inv3(const M3<double> &a) {
    double dr, di;
    det3(a, dr, di);
    M3<double> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            double pr = a.re[i1][j1] * a.re[i2][j2] - a.im[i1][j1] * a.im[i2][j2];
            double pi = a.re[i1][j1] * a.im[i2][j2] + a.im[i1][j1] * a.re[i2][j2];
            double qr = a.re[i1][j2] * a.re[i2][j1] - a.im[i1][j2] * a.im[i2][j1];
            double qi = a.re[i1][j2] * a.im[i2][j1] + a.im[i1][j2] * a.re[i2][j1];
            double cr, ci;
            cdiv(pr - qr, pi - qi, dr, di, cr, ci);
            r.re[j][i] = cr;
            r.im[j][i] = ci;
        }
    return r;
}

__device__ inline M3<double> dagger(const M3<double> &a) {
    M3<double> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) { r.re[i][j] = a.re[j][i]; r.im[i][j] = -a.im[j][i]; }
    return r;
}

// unitary polar factor by X <- (X + X^{-dag})/2, then principal cube root of det removed
__device__ inline M3<double> su3_project(M3<double> X) {
    for (int it = 0; it < 100; it++) {
        M3<double> Y = add(X, dagger(inv3(X)));
        double ch = 0;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                Y.re[i][j] *= 0.5;
                Y.im[i][j] *= 0.5;
                double a = Y.re[i][j] - X.re[i][j], b = Y.im[i][j] - X.im[i][j];
                ch += a * a + b * b;
            }
        X = Y;
        if (sqrt(ch) < 1e-15) break;
    }
    double dr, di;
    det3(X, dr, di);
    double th = atan2(di, dr) / 3.0;
    double s, c;
    sincos(-th, &s, &c);
    M3<double> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            r.re[i][j] = X.re[i][j] * c - X.im[i][j] * s;
            r.im[i][j] = X.re[i][j] * s + X.im[i][j] * c;
        }
    return r;
}

__device__ inline double match_residual(const M3<double> &W, const M3<double> &U, double *R) {
    M3<double> M = add(W, mul_nd(W, U));   // W (1 + U^dag)
    alg_proj(M, R);
    double m = 0;
#pragma unroll
    for (int a = 0; a < 8; a++) m = fmax(m, fabs(R[a]));
    return m;
}

// Gaussian elimination with partial pivoting, unrolled so that J and b stay
// in registers: each column's largest remaining entry is moved to the pivot
// row by conditional swaps with the rows below it.
__device__ inline bool solve8(double J[8][8], double *b) {
#pragma unroll
    for (int c = 0; c < 8; c++) {
#pragma unroll
        for (int r = c + 1; r < 8; r++) {
            const bool sw = fabs(J[r][c]) > fabs(J[c][c]);
#pragma unroll
            for (int k = c; k < 8; k++) {
                const double t = J[c][k];
                J[c][k] = sw ? J[r][k] : t;
                J[r][k] = sw ? t : J[r][k];
            }
            const double t = b[c];
            b[c] = sw ? b[r] : t;
            b[r] = sw ? t : b[r];
        }
        if (J[c][c] == 0.0) return false;
#pragma unroll
        for (int r = c + 1; r < 8; r++) {
            const double f = J[r][c] / J[c][c];
#pragma unroll
            for (int k = c; k < 8; k++) J[r][k] -= f * J[c][k];
            b[r] -= f * b[c];
        }
    }
#pragma unroll
    for (int i = 7; i >= 0; i--) {
        double s = b[i];
#pragma unroll
        for (int k = i + 1; k < 8; k++) s -= J[i][k] * b[k];
        b[i] = s / J[i][i];
    }
    return true;
}

__device__ inline M3<double> nucleus_link(const double *V, size_t n2, size_t x, size_t xp) {
    return mul_nd(load_m(V, n2, x), load_m(V, n2, xp));
}

// one thread per link (d, x)
__global__ void __launch_bounds__(128)
k_match(int N, const double *VA, const double *VB, double *U0, int *status, int max_iter,
        double tol) {
    size_t n2 = (size_t)N * N;
    size_t t = (size_t)blockIdx.x * 128 + threadIdx.x;
    if (t >= 2 * n2) return;
    int d = (int)(t / n2);
    size_t x = t % n2;
    int ix = (int)(x % N), iy = (int)(x / N);
    size_t xp = d == 0 ? (size_t)(ix + 1 == N ? 0 : ix + 1) + (size_t)N * iy
                       : (size_t)ix + (size_t)N * (iy + 1 == N ? 0 : iy + 1);
    M3<double> W = add(nucleus_link(VA, n2, x, xp), nucleus_link(VB, n2, x, xp));
    M3<double> U = su3_project(mul(W, inv3(dagger(W))));
    double R[8];
    double rn = match_residual(W, U, R);
    int it = 0;
    while (rn >= tol && it < max_iter) {
        M3<double> M = mul_nd(W, U);
        double J[8][8];
        // unrolled: e is a constant unit vector, so M T^b folds to the few
        // non-zero entries of the generator
#pragma unroll
        for (int b = 0; b < 8; b++) {
            double e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            e[b] = 1.0;
            double col[8];
            alg_from_herm(mul(M, herm_from_alg(e)), col);   // 2 Re Tr(T^a M T^b)
            for (int a = 0; a < 8; a++) J[a][b] = -col[a];
        }
        double dl[8];
        for (int a = 0; a < 8; a++) dl[a] = -R[a];
        if (!solve8(J, dl)) break;
        double step = 1.0, rnn = rn, Rn[8];
        M3<double> Un = U;
        for (int h = 0; h < 40; h++) {
            Un = mul(expi_alg(dl, step), U);
            rnn = match_residual(W, Un, Rn);
            if (rnn < rn) break;
            step *= 0.5;
        }
        U = Un;
        for (int a = 0; a < 8; a++) R[a] = Rn[a];
        rn = rnn;
        it++;
    }
    store_m(U0 + (size_t)d * 18 * n2, n2, x, U);
    if (!(rn < tol)) atomicOr(status, 1);
}

// ---- 5. pi0 -------------------------------------------------------------------
__global__ void __launch_bounds__(128)
k_pi0(int N, const double *VA, const double *VB, const double *U0, double *pi0) {
    size_t n2 = (size_t)N * N;
    size_t x = (size_t)blockIdx.x * 128 + threadIdx.x;
    if (x >= n2) return;
    int ix = (int)(x % N), iy = (int)(x / N);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int d = 0; d < 2; d++) {
        int pxi = d == 0 ? (ix + 1 == N ? 0 : ix + 1) : ix, pyi = d == 0 ? iy : (iy + 1 == N ? 0 : iy + 1);
        int mxi = d == 0 ? (ix == 0 ? N - 1 : ix - 1) : ix, myi = d == 0 ? iy : (iy == 0 ? N - 1 : iy - 1);
        size_t xp = (size_t)pxi + (size_t)N * pyi, xm = (size_t)mxi + (size_t)N * myi;
        M3<double> one = m_ident<double>();
        {
            M3<double> u = load_m(U0 + (size_t)d * 18 * n2, n2, x);
            M3<double> ua = nucleus_link(VA, n2, x, xp), ub = nucleus_link(VB, n2, x, xp);
            M3<double> m = mul(sub(u, one), sub(dagger(ub), dagger(ua)));
            double v[8];
            alg_proj(m, v);
            for (int a = 0; a < 8; a++) acc[a] += v[a];
        }
        {
            M3<double> u = load_m(U0 + (size_t)d * 18 * n2, n2, xm);
            M3<double> ua = nucleus_link(VA, n2, xm, x), ub = nucleus_link(VB, n2, xm, x);
            M3<double> m = mul(sub(dagger(u), one), sub(ub, ua));
            double v[8];
            alg_proj(m, v);
            for (int a = 0; a < 8; a++) acc[a] += v[a];
        }
    }
    for (int a = 0; a < 8; a++) pi0[(size_t)a * n2 + x] = 0.5 * acc[a];
}

template <typename T>
__global__ void __launch_bounds__(256)
k_first_half_step(int N, const double *U0, const double *pi0, FieldPtrs<T> out, double dtau) {
    size_t n2 = (size_t)N * N;
    size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (x >= n2) return;
    // the field state is stored in chunked planes, written here in whole
    // chunks; it keeps the first two rows of each link
    constexpr int NV = 16 / (int)sizeof(T);
    for (int d = 0; d < 2; d++) {
        T v[kLinkVals];
        for (int c = 0; c < kLinkVals; c++) v[c] = (T)U0[(size_t)(18 * d + c) * n2 + x];
        for (int c = 0; c < kLinkVals; c += NV) chunk_st16(out.U, n2, x, kLinkVals * d + c, v + c);
    }
    const T zero[NV] = {};
    for (int c = 0; c < 16; c += NV) chunk_st16(out.E, n2, x, c, zero);
    const double th = 0.5 * dtau;
    T pv[8], fv[8];
    for (int a = 0; a < 8; a++) {
        double p = pi0[(size_t)a * n2 + x];
        pv[a] = (T)p;
        fv[a] = (T)(dtau * th * p);
    }
    for (int a = 0; a < 8; a += NV) {
        chunk_st16(out.pi, n2, x, a, pv + a);
        chunk_st16(out.phi, n2, x, a, fv + a);
    }
}

// ---- launchers ----------------------------------------------------------------
static inline unsigned blocks_for(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_mv_charges(hipStream_t st, int N, double sigma, uint64_t seed, int nucleus,
                             int sheet0, int n_sheets, double2 *planes) {
    const MvDraw mv{sigma, seed, nucleus, sheet0};
    hipLaunchKernelGGL(k_mv_charges, dim3(blocks_for((size_t)N * N, 256), n_sheets), dim3(256), 0, st, N, mv,
                       planes);
    return hipGetLastError();
}

hipError_t launch_charges_to_planes(hipStream_t st, int N, const double *rho, double2 *planes) {
    hipLaunchKernelGGL(k_pack, dim3(blocks_for((size_t)N * N, 256)), dim3(256), 0, st, N, rho, planes);
    return hipGetLastError();
}

hipError_t launch_planes_to_charges(hipStream_t st, int N, const double2 *planes, double *rho) {
    hipLaunchKernelGGL(k_unpack, dim3(blocks_for((size_t)N * N, 256)), dim3(256), 0, st, N, planes, rho);
    return hipGetLastError();
}

hipError_t launch_fft_tables(hipStream_t st, int N, double2 *tab) {
    if (N > kFftMaxN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fft_tables, dim3((N + 255) / 256), dim3(256), 0, st, N, tab, (double *)(tab + kFftMaxN));
    return hipGetLastError();
}

// Poisson solve of n_sheets x 4 planes: forward row transforms, the fused
// column pass (forward, kernel, inverse) and inverse row transforms; tab
// holds the tables of launch_fft_tables for this N.  With draw, the forward
// row pass draws the MV charges itself (the planes' input is not read).
hipError_t launch_poisson(hipStream_t st, int N, double m2, double uv2, double2 *planes, int n_sheets,
                          const double2 *tab, const MvDraw *draw) {
    Radices rs;
    if (N > kFftMaxN || !radices_of(N, rs)) return hipErrorInvalidValue;
    const size_t n2 = (size_t)N * N;
    const int C = fft_lines_per_group(N), groups = N / C, n_planes = 4 * n_sheets;
    const double *s2 = (const double *)(tab + kFftMaxN);
    const size_t lds_lines = (kFftElems + (size_t)N) * sizeof(double2), lds_poisson = lds_lines + N * sizeof(double);
    const MvDraw mv = draw ? *draw : MvDraw{0.0, 0, 0, 0};
    if (draw)
        hipLaunchKernelGGL(k_fft_lines<kFftDraw>, dim3(n_planes * groups), dim3(kFftThreads), lds_lines, st, planes,
                           N, C, 0, n2, groups, -1, rs, m2, uv2, tab, s2, mv);
    else
        hipLaunchKernelGGL(k_fft_lines<kFftLines>, dim3(n_planes * groups), dim3(kFftThreads), lds_lines, st, planes,
                           N, C, 0, n2, groups, -1, rs, m2, uv2, tab, s2, mv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fft_lines<kFftPoisson>, dim3(n_planes * groups), dim3(kFftThreads), lds_poisson, st,
                       planes, N, C, 1, n2, groups, -1, rs, m2, uv2, tab, s2, mv);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fft_lines<kFftLines>, dim3(n_planes * groups), dim3(kFftThreads), lds_lines, st, planes,
                       N, C, 0, n2, groups, +1, rs, m2, uv2, tab, s2, mv);
    return hipGetLastError();
}

hipError_t launch_dipole(hipStream_t st, int N, const double *V, int rmax, double *partials, double *D) {
    const int nb = (int)blocks_for((size_t)N * N, 256);
    hipLaunchKernelGGL(k_dipole, dim3(nb, rmax + 1), dim3(256), 0, st, N, V, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dipole_reduce, dim3(rmax + 1), dim3(256), 0, st, N, (const double *)partials, nb, D);
    return hipGetLastError();
}

hipError_t launch_wilson_init(hipStream_t st, int N, double *V) {
    hipLaunchKernelGGL(k_wilson_init, dim3(blocks_for((size_t)N * N, 256)), dim3(256), 0, st, N, V);
    return hipGetLastError();
}

hipError_t launch_wilson_accum(hipStream_t st, int N, const double2 *planes, int n_sheets, double *V) {
    hipLaunchKernelGGL(k_wilson_accum, dim3(blocks_for((size_t)N * N, 256)), dim3(256), 0, st, N,
                       planes, n_sheets, V);
    return hipGetLastError();
}

hipError_t launch_match_pi0(hipStream_t st, int N, const double *VA, const double *VB, double *U0,
                           double *pi0, int *status, int max_iter, double tol) {
    size_t n2 = (size_t)N * N;
    hipLaunchKernelGGL(k_match, dim3(blocks_for(2 * n2, 128)), dim3(128), 0, st, N, VA, VB, U0, status,
                       max_iter, tol);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pi0, dim3(blocks_for(n2, 128)), dim3(128), 0, st, N, VA, VB, U0, pi0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_first_half_step(hipStream_t st, int N, const double *U0, const double *pi0,
                                  FieldPtrs<T> out, double dtau) {
    hipLaunchKernelGGL(k_first_half_step<T>, dim3(blocks_for((size_t)N * N, 256)), dim3(256), 0, st, N,
                       U0, pi0, out, dtau);
    return hipGetLastError();
}

template hipError_t launch_first_half_step<double>(hipStream_t, int, const double *, const double *,
                                                   FieldPtrs<double>, double);
template hipError_t launch_first_half_step<float>(hipStream_t, int, const double *, const double *,
                                                  FieldPtrs<float>, double);

}  // namespace gl
