// glasma_oracle.cpp -- TEST INFRASTRUCTURE ONLY (see glasma_oracle.h).
//
// A plain FP64 reading of the method of Avramescu et al. (Hard Probes 2023):
// MV color sources (Sec. 1, "Glasma"), the boost-invariant classical
// Yang-Mills evolution of Eq. (1) on gauge links and plaquettes, Wong's
// equations Eq. (2) solved with link-built particle Wilson lines (Sec. 1,
// "Probes in Glasma"), and the momentum broadening behind Eq. (3) (Sec. 2).
// Every discretisation detail the paper leaves open is fixed by one reading,
// stated next to the code that implements it.  Nothing here is blocked,
// fused or vectorised; it is meant to be checked by eye.

#include "glasma_oracle.h"

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

typedef std::complex<double> cd;
const cd IU(0.0, 1.0);

struct Mat {
    cd m[3][3];
};

Mat zero() {
    Mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.m[i][j] = 0.0;
    return r;
}

Mat ident() {
    Mat r = zero();
    for (int i = 0; i < 3; i++) r.m[i][i] = 1.0;
    return r;
}

Mat mul(const Mat &a, const Mat &b) {
    Mat r = zero();
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++) r.m[i][j] += a.m[i][k] * b.m[k][j];
    return r;
}

Mat add(const Mat &a, const Mat &b) {
    Mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.m[i][j] = a.m[i][j] + b.m[i][j];
    return r;
}

Mat sub(const Mat &a, const Mat &b) {
    Mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.m[i][j] = a.m[i][j] - b.m[i][j];
    return r;
}

Mat scale(cd s, const Mat &a) {
    Mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.m[i][j] = s * a.m[i][j];
    return r;
}

Mat dag(const Mat &a) {
    Mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.m[i][j] = std::conj(a.m[j][i]);
    return r;
}

cd trace(const Mat &a) { return a.m[0][0] + a.m[1][1] + a.m[2][2]; }

double frob(const Mat &a) {
    double s = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) s += std::norm(a.m[i][j]);
    return std::sqrt(s);
}

Mat load(const double *p) {
    Mat r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.m[i][j] = cd(p[2 * (3 * i + j)], p[2 * (3 * i + j) + 1]);
    return r;
}

void store(const Mat &a, double *p) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            p[2 * (3 * i + j)] = a.m[i][j].real();
            p[2 * (3 * i + j) + 1] = a.m[i][j].imag();
        }
}

// SU(3) generators T^a = lambda^a / 2 from the Gell-Mann matrices; these are
// the "T^a" of the color charge Q = Q^a T^a (Sec. 1, "Probes in Glasma").
const Mat &gen(int a) {
    static Mat T[8];
    static bool ready = false;
    if (!ready) {
        for (int k = 0; k < 8; k++) T[k] = zero();
        const double h = 0.5;
        T[0].m[0][1] = h;             T[0].m[1][0] = h;
        T[1].m[0][1] = -IU * h;       T[1].m[1][0] = IU * h;
        T[2].m[0][0] = h;             T[2].m[1][1] = -h;
        T[3].m[0][2] = h;             T[3].m[2][0] = h;
        T[4].m[0][2] = -IU * h;       T[4].m[2][0] = IU * h;
        T[5].m[1][2] = h;             T[5].m[2][1] = h;
        T[6].m[1][2] = -IU * h;       T[6].m[2][1] = IU * h;
        const double s3 = 1.0 / std::sqrt(3.0);
        T[7].m[0][0] = h * s3;        T[7].m[1][1] = h * s3;   T[7].m[2][2] = -2.0 * h * s3;
        ready = true;
    }
    return T[a];
}

// X = x^a T^a
Mat alg(const double *x) {
    Mat r = zero();
    for (int a = 0; a < 8; a++) r = add(r, scale(x[a], gen(a)));
    return r;
}

// Components of a hermitian matrix, X^a = 2 Tr(T^a X).
void herm_comps(const Mat &X, double *x) {
    for (int a = 0; a < 8; a++) x[a] = 2.0 * std::real(trace(mul(gen(a), X)));
}

// Components of the projection [M]_X = (M - M^dag)/(2i) - (trace)/3:
// 2 Tr(T^a [M]_X) = 2 Im Tr(T^a M) because the generators are traceless.
void proj_comps(const Mat &M, double *x) {
    for (int a = 0; a < 8; a++) x[a] = 2.0 * std::imag(trace(mul(gen(a), M)));
}

Mat proj_mat(const Mat &M) {
    double x[8];
    proj_comps(M, x);
    return alg(x);
}

// Matrix exponential by its power series, with scaling and squaring.
Mat expm(const Mat &A) {
    double nrm = frob(A);
    int s = 0;
    while (nrm > 0.25) {
        nrm *= 0.5;
        s++;
    }
    Mat B = scale(std::ldexp(1.0, -s), A);
    Mat sum = ident(), term = ident();
    for (int k = 1; k < 60; k++) {
        term = scale(1.0 / k, mul(term, B));
        sum = add(sum, term);
        if (frob(term) < 1e-22) break;
    }
    for (int k = 0; k < s; k++) sum = mul(sum, sum);
    return sum;
}

// exp(i x^a T^a)
Mat expi(const double *x) { return expm(scale(IU, alg(x))); }

// ---- lattice indexing ------------------------------------------------------
inline int site(int N, int ix, int iy) {
    ix %= N;
    if (ix < 0) ix += N;
    iy %= N;
    if (iy < 0) iy += N;
    return ix + N * iy;
}
// neighbour of x shifted by s in direction d (0 = x, 1 = y)
inline int shift(int N, int x, int d, int s) {
    int ix = x % N, iy = x / N;
    if (d == 0) ix += s; else iy += s;
    return site(N, ix, iy);
}

struct Field {
    int N;
    const double *U, *phi;
    Mat link(int d, int x) const { return load(U + ((size_t)d * N * N + x) * 18); }
    Mat ph(int x) const { return alg(phi + (size_t)x * 8); }
};

// Plaquette P(x) = U_1(x) U_2(x+1) U_1^dag(x+2) U_2^dag(x): the elementary
// closed loop of the link/plaquette discretisation (Sec. 1, "Glasma").
Mat plaquette(const Field &f, int x) {
    int N = f.N;
    return mul(mul(f.link(0, x), f.link(1, shift(N, x, 0, 1))),
               mul(dag(f.link(0, shift(N, x, 1, 1))), dag(f.link(1, x))));
}

// phi(x+i) parallel-transported to x: U_i(x) phi(x+i) U_i^dag(x)
Mat phi_fwd(const Field &f, int x, int d) {
    Mat U = f.link(d, x);
    return mul(mul(U, f.ph(shift(f.N, x, d, 1))), dag(U));
}

// phi(x-i) parallel-transported to x: U_i^dag(x-i) phi(x-i) U_i(x-i)
Mat phi_bwd(const Field &f, int x, int d) {
    int xm = shift(f.N, x, d, -1);
    Mat U = f.link(d, xm);
    return mul(mul(dag(U), f.ph(xm)), U);
}

// Reading of Eq. (1) on the boost-invariant lattice (Milne time, A_tau = 0):
// fields E_i = tau dA_i/dtau, phi = A_eta, pi = (1/tau) dA_eta/dtau, with
// Hamiltonian per unit rapidity
//   H = sum_x [ (1/tau) sum_i Tr E_i^2 + tau Tr pi^2
//              + (1/tau) sum_i Tr (Phi_{+i} - phi)^2 + 2 tau (3 - Re Tr P) ].
// The forces below are -dH/d(link) (left derivative) and -dH/dphi.
void site_forces(const Field &f, double tau, int x, double *FE1, double *FE2,
                 double *Fpi) {
    int N = f.N;
    int xm1 = shift(N, x, 0, -1), xm2 = shift(N, x, 1, -1);
    Mat Px = proj_mat(plaquette(f, x));
    Mat P1 = proj_mat(plaquette(f, xm1));
    Mat P2 = proj_mat(plaquette(f, xm2));
    Mat U1m = f.link(0, xm1), U2m = f.link(1, xm2);
    Mat P1t = mul(mul(dag(U1m), P1), U1m);   // P(x-1) carried to x
    Mat P2t = mul(mul(dag(U2m), P2), U2m);   // P(x-2) carried to x
    Mat ph = f.ph(x);
    Mat Pf1 = phi_fwd(f, x, 0), Pf2 = phi_fwd(f, x, 1);
    Mat Pb1 = phi_bwd(f, x, 0), Pb2 = phi_bwd(f, x, 1);
    // E_1: -tau([P(x)] - [P(x-2)]) - (i/tau)[phi, Phi_{+1}]
    Mat c1 = scale(-IU / tau, sub(mul(ph, Pf1), mul(Pf1, ph)));
    Mat c2 = scale(-IU / tau, sub(mul(ph, Pf2), mul(Pf2, ph)));
    Mat f1 = add(scale(-tau, sub(Px, P2t)), c1);
    Mat f2 = add(scale(-tau, sub(P1t, Px)), c2);
    herm_comps(f1, FE1);
    herm_comps(f2, FE2);
    Mat lap = sub(add(add(Pf1, Pb1), add(Pf2, Pb2)), scale(4.0, ph));
    herm_comps(scale(1.0 / tau, lap), Fpi);
}

// Local-frame site fields at tau_n used by the particles (NGP interpolation;
// the paper only says "colored particle-in-cell", Sec. 1).  E is the time
// average of the two half-step values, averaged over the two links that meet
// at the site; B_z from the clover of the four plaquettes touching x.
// Ebar[d][0] is the time-averaged E_d at x, Ebar[d][1] at x - d; pibar at x.
void site_fields(const Field &f, double tau, int x, const double Ebar[2][2][8],
                 const double *pibar, double *F) {
    int N = f.N;
    Mat Es[2];
    for (int d = 0; d < 2; d++) {
        Mat Um = f.link(d, shift(N, x, d, -1));
        Es[d] = scale(0.5, add(alg(Ebar[d][0]), mul(mul(dag(Um), alg(Ebar[d][1])), Um)));
    }
    Mat Dphi[2];
    for (int d = 0; d < 2; d++) Dphi[d] = scale(0.5, sub(phi_fwd(f, x, d), phi_bwd(f, x, d)));
    // clover: P(x), P(x-1), P(x-2), P(x-1-2), each carried to x
    int xm1 = shift(N, x, 0, -1), xm2 = shift(N, x, 1, -1), xm12 = shift(N, xm1, 1, -1);
    Mat C = proj_mat(plaquette(f, x));
    Mat U1 = f.link(0, xm1);
    C = add(C, mul(mul(dag(U1), proj_mat(plaquette(f, xm1))), U1));
    Mat U2 = f.link(1, xm2);
    C = add(C, mul(mul(dag(U2), proj_mat(plaquette(f, xm2))), U2));
    Mat W = mul(f.link(0, xm12), f.link(1, xm2));   // path x-1-2 -> x-2 -> x
    C = add(C, mul(mul(dag(W), proj_mat(plaquette(f, xm12))), W));
    C = scale(0.25, C);
    double *Ex = F, *Ey = F + 8, *Ez = F + 16, *Bx = F + 24, *By = F + 32, *Bz = F + 40;
    herm_comps(scale(1.0 / tau, Es[0]), Ex);
    herm_comps(scale(1.0 / tau, Es[1]), Ey);
    for (int a = 0; a < 8; a++) Ez[a] = pibar[a];
    herm_comps(scale(-1.0 / tau, Dphi[1]), Bx);
    herm_comps(scale(1.0 / tau, Dphi[0]), By);
    herm_comps(scale(-1.0, C), Bz);
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ---------------------
void philox(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4]) {
    uint32_t k0 = key[0], k1 = key[1];
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int r = 0; r < 10; r++) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// uniform (2k+1) 2^-53 with k the top 52 bits of the 64-bit word (hi:lo)
double u53(uint32_t lo, uint32_t hi) {
    uint64_t v = ((uint64_t)hi << 32) | (uint64_t)lo;
    uint64_t k = ((v >> 12) << 1) | 1u;
    return std::ldexp((double)k, -53);
}

void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t out[4]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {c0, c1, c2, 0u};
    philox(key, ctr, out);
}

// Box-Muller: the two uniforms of one draw give two standard normals.
void gauss2(const uint32_t w[4], double *g0, double *g1) {
    double u1 = u53(w[0], w[1]), u2 = u53(w[2], w[3]);
    double r = std::sqrt(-2.0 * std::log(u1));
    const double twopi = 6.283185307179586476925286766559;
    *g0 = r * std::cos(twopi * u2);
    *g1 = r * std::sin(twopi * u2);
}

// ---- FFT: plain recursive decimation in time, radix 2 and 3 ---------------
void dft_rec(const cd *in, int stride, int n, cd *out, int sign) {
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int r = (n % 2 == 0) ? 2 : ((n % 3 == 0) ? 3 : n);
    int m = n / r;
    const double pi = 3.141592653589793238462643383279;
    if (r == n) {   // no radix left: direct sum
        for (int k = 0; k < n; k++) {
            cd s = 0.0;
            for (int j = 0; j < n; j++) s += in[(size_t)j * stride] * std::polar(1.0, sign * 2.0 * pi * (double)((long)j * k % n) / n);
            out[k] = s;
        }
        return;
    }
    std::vector<cd> sub_out((size_t)n);
    for (int j = 0; j < r; j++) dft_rec(in + (size_t)j * stride, stride * r, m, sub_out.data() + (size_t)j * m, sign);
    for (int k = 0; k < m; k++)
        for (int q = 0; q < r; q++) {
            int kk = k + q * m;
            cd s = 0.0;
            for (int j = 0; j < r; j++) s += sub_out[(size_t)j * m + k] * std::polar(1.0, sign * 2.0 * pi * (double)((long)j * kk % n) / n);
            out[kk] = s;
        }
}

// 2-D DFT of an N x N complex plane (rows then columns), sign -1 forward
void fft2(int N, std::vector<cd> &a, int sign) {
    std::vector<cd> line(N), res(N);
    for (int y = 0; y < N; y++) {
        for (int x = 0; x < N; x++) line[x] = a[(size_t)x + (size_t)N * y];
        dft_rec(line.data(), 1, N, res.data(), sign);
        for (int x = 0; x < N; x++) a[(size_t)x + (size_t)N * y] = res[x];
    }
    for (int x = 0; x < N; x++) {
        for (int y = 0; y < N; y++) line[y] = a[(size_t)x + (size_t)N * y];
        dft_rec(line.data(), 1, N, res.data(), sign);
        for (int y = 0; y < N; y++) a[(size_t)x + (size_t)N * y] = res[y];
    }
}

// Reading of the MV-model Poisson step: (-Lap + m^2) Lambda = rho with the
// 5-point lattice Laplacian, solved exactly in Fourier space
// (denominator 4 sin^2(pi kx/N) + 4 sin^2(pi ky/N) + m^2).  An optional UV
// regulator removes the modes whose lattice momentum squared exceeds uv2
// (uv2 <= 0: no cut).
void poisson(int N, double m2, double uv2, const double *src, size_t src_stride, double *out,
             size_t out_stride) {
    std::vector<cd> a((size_t)N * N);
    for (size_t x = 0; x < (size_t)N * N; x++) a[x] = src[x * src_stride];
    fft2(N, a, -1);
    const double pi = 3.141592653589793238462643383279;
    for (int ky = 0; ky < N; ky++)
        for (int kx = 0; kx < N; kx++) {
            double sx = std::sin(pi * kx / N), sy = std::sin(pi * ky / N);
            double k2 = 4.0 * sx * sx + 4.0 * sy * sy;
            if (uv2 > 0.0 && k2 > uv2) a[(size_t)kx + (size_t)N * ky] = 0.0;
            else a[(size_t)kx + (size_t)N * ky] /= (k2 + m2);
        }
    fft2(N, a, +1);
    double inv = 1.0 / ((double)N * N);
    for (size_t x = 0; x < (size_t)N * N; x++) out[x * out_stride] = a[x].real() * inv;
}

// solve J d = b for 8x8 by Gaussian elimination with partial pivoting
bool solve8(double J[8][8], double b[8], double d[8]) {
    double A[8][9];
    for (int i = 0; i < 8; i++) {
        for (int j = 0; j < 8; j++) A[i][j] = J[i][j];
        A[i][8] = b[i];
    }
    for (int c = 0; c < 8; c++) {
        int piv = c;
        for (int r = c + 1; r < 8; r++)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0) return false;
        if (piv != c)
            for (int j = 0; j < 9; j++) std::swap(A[c][j], A[piv][j]);
        for (int r = c + 1; r < 8; r++) {
            double fct = A[r][c] / A[c][c];
            for (int j = c; j < 9; j++) A[r][j] -= fct * A[c][j];
        }
    }
    for (int i = 7; i >= 0; i--) {
        double s = A[i][8];
        for (int j = i + 1; j < 8; j++) s -= A[i][j] * d[j];
        d[i] = s / A[i][i];
    }
    return true;
}

cd det3(const Mat &a) {
    return a.m[0][0] * (a.m[1][1] * a.m[2][2] - a.m[1][2] * a.m[2][1])
         - a.m[0][1] * (a.m[1][0] * a.m[2][2] - a.m[1][2] * a.m[2][0])
         + a.m[0][2] * (a.m[1][0] * a.m[2][1] - a.m[1][1] * a.m[2][0]);
}

// inverse by cofactors
Mat inv3(const Mat &a) {
    Mat c;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            c.m[j][i] = a.m[i1][j1] * a.m[i2][j2] - a.m[i1][j2] * a.m[i2][j1];
        }
    return scale(1.0 / det3(a), c);
}

// SU(3) projection: unitary polar factor of M (the closest unitary matrix),
// found by the iteration X <- (X + X^{-dag})/2, then its determinant phase
// removed with the principal cube root.
Mat su3_project(const Mat &M) {
    Mat X = M;
    for (int it = 0; it < 100; it++) {
        Mat Y = scale(0.5, add(X, dag(inv3(X))));
        double ch = frob(sub(Y, X));
        X = Y;
        if (ch < 1e-15) break;
    }
    double th = std::arg(det3(X));
    return scale(std::polar(1.0, -th / 3.0), X);
}

// residual of the matching condition [(UA + UB)(1 + U^dag)]_X
void match_residual(const Mat &W, const Mat &U, double *R) {
    proj_comps(mul(W, add(ident(), dag(U))), R);
}

double maxabs8(const double *v) {
    double m = 0.0;
    for (int a = 0; a < 8; a++) m = std::fmax(m, std::fabs(v[a]));
    return m;
}

}  // namespace

// ============================================================================
extern "C" {

void orc_generator(int a, double *T18) { store(gen(a), T18); }

double orc_dsym(int a, int b, int c) {
    Mat ab = add(mul(gen(a), gen(b)), mul(gen(b), gen(a)));
    return 2.0 * std::real(trace(mul(ab, gen(c))));
}

void orc_expi(const double *x8, double *U18) { store(expi(x8), U18); }

void orc_expm(const double *A18, double *out18) { store(expm(load(A18)), out18); }

void orc_proj(const double *M18, double *x8) { proj_comps(load(M18), x8); }

void orc_philox(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4]) {
    philox(key, ctr, out);
}

double orc_u53(uint32_t lo, uint32_t hi) { return u53(lo, hi); }

// MV color charges (Sec. 1, "Glasma"): independent Gaussian rho^a per site,
// sheet and nucleus.  Draw layout: counter (site, 4*sheet + j, nucleus, 0),
// j = 0..3, each draw giving colors 2j and 2j+1 through Box-Muller.
void orc_mv_charges(int N, double sigma, uint64_t seed, int nucleus, int sheet,
                    double *rho) {
    for (int x = 0; x < N * N; x++)
        for (int j = 0; j < 4; j++) {
            uint32_t w[4];
            draw(seed, (uint32_t)x, (uint32_t)(4 * sheet + j), (uint32_t)nucleus, w);
            double g0, g1;
            gauss2(w, &g0, &g1);
            rho[(size_t)x * 8 + 2 * j] = sigma * g0;
            rho[(size_t)x * 8 + 2 * j + 1] = sigma * g1;
        }
}

int orc_fft(int n, double *data, int sign) {
    if (n < 1) return -1;
    std::vector<cd> in(n), out(n);
    for (int k = 0; k < n; k++) in[k] = cd(data[2 * k], data[2 * k + 1]);
    dft_rec(in.data(), 1, n, out.data(), sign);
    for (int k = 0; k < n; k++) {
        data[2 * k] = out[k].real();
        data[2 * k + 1] = out[k].imag();
    }
    return 0;
}

int orc_poisson(int N, double m2, const double *src, double *out) {
    if (N < 1 || m2 <= 0.0) return -1;
    poisson(N, m2, 0.0, src, 1, out, 1);
    return 0;
}

int orc_poisson_uv(int N, double m2, double uv2, const double *src, double *out) {
    if (N < 1 || m2 <= 0.0) return -1;
    poisson(N, m2, uv2, src, 1, out, 1);
    return 0;
}

// Path-ordered Wilson line of one nucleus, V = exp(-i L_1) ... exp(-i L_Ns),
// sheet 1 leftmost, where L_s solves the Poisson equation for sheet s.
int orc_wilson_line(int N, double sigma, double m2, int n_sheets, uint64_t seed,
                    int nucleus, double *V) {
    return orc_wilson_line_uv(N, sigma, m2, 0.0, n_sheets, seed, nucleus, V);
}

int orc_wilson_line_uv(int N, double sigma, double m2, double uv2, int n_sheets, uint64_t seed,
                       int nucleus, double *V) {
    if (N < 1 || n_sheets < 1 || m2 <= 0.0) return -1;
    size_t N2 = (size_t)N * N;
    std::vector<Mat> v(N2, ident());
    std::vector<double> rho(N2 * 8), lam(N2 * 8);
    for (int s = 0; s < n_sheets; s++) {
        orc_mv_charges(N, sigma, seed, nucleus, s, rho.data());
        for (int a = 0; a < 8; a++) poisson(N, m2, uv2, rho.data() + a, 8, lam.data() + a, 8);
        for (size_t x = 0; x < N2; x++) {
            double ml[8];
            for (int a = 0; a < 8; a++) ml[a] = -lam[x * 8 + a];
            v[x] = mul(v[x], expi(ml));
        }
    }
    for (size_t x = 0; x < N2; x++) store(v[x], V + x * 18);
    return 0;
}

void orc_nucleus_links(int N, const double *V, double *Un) {
    size_t N2 = (size_t)N * N;
    for (int d = 0; d < 2; d++)
        for (int x = 0; x < N * N; x++) {
            Mat a = load(V + (size_t)x * 18);
            Mat b = load(V + (size_t)shift(N, x, d, 1) * 18);
            store(mul(a, dag(b)), Un + ((size_t)d * N2 + x) * 18);
        }
}

// Matching of the two nuclei's pure-gauge links to the forward light cone
// (Sec. 1, "Glasma": fields produced after the collision).  The paper does not
// print the lattice condition; the reading used is
// [(UA + UB)(1 + U^dag)]_X = 0 solved by damped Newton with a central-difference
// Jacobian, started from the SU(3) projection of W (W^dag)^{-1}, W = UA + UB
// (the exact solution when both nuclei lie in one SU(2) subgroup).
int orc_match_link(const double *UA18, const double *UB18, double *U18, double tol,
                   int max_iter, double *res_out) {
    Mat UA = load(UA18), UB = load(UB18);
    Mat W = add(UA, UB);
    Mat U = su3_project(mul(W, inv3(dag(W))));
    double R[8];
    match_residual(W, U, R);
    double rn = maxabs8(R);
    int it = 0;
    const double eps = 1e-6;
    while (rn >= tol && it < max_iter) {
        double J[8][8];
        for (int b = 0; b < 8; b++) {
            double e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            e[b] = eps;
            double Rp[8], Rm[8];
            match_residual(W, mul(expi(e), U), Rp);
            e[b] = -eps;
            match_residual(W, mul(expi(e), U), Rm);
            for (int a = 0; a < 8; a++) J[a][b] = (Rp[a] - Rm[a]) / (2.0 * eps);
        }
        double mR[8], d[8];
        for (int a = 0; a < 8; a++) mR[a] = -R[a];
        if (!solve8(J, mR, d)) break;
        double step = 1.0;
        Mat Un;
        double Rn[8], rnn = 0.0;
        for (int h = 0; h < 40; h++) {
            double ds[8];
            for (int a = 0; a < 8; a++) ds[a] = step * d[a];
            Un = mul(expi(ds), U);
            match_residual(W, Un, Rn);
            rnn = maxabs8(Rn);
            if (rnn < rn) break;
            step *= 0.5;
        }
        U = Un;
        for (int a = 0; a < 8; a++) R[a] = Rn[a];
        rn = rnn;
        it++;
    }
    store(U, U18);
    if (res_out) *res_out = rn;
    return rn < tol ? it : -3;
}

// Initial longitudinal field (reading; the paper gives no formula):
// pi0(x) = 1/2 sum_i { [(U_i(x) - 1)(UB_i(x)^dag - UA_i(x)^dag)]_X
//                    + [(U_i(x-i)^dag - 1)(UB_i(x-i) - UA_i(x-i))]_X }.
void orc_pi0(int N, const double *U, const double *UA, const double *UB, double *pi0) {
    size_t N2 = (size_t)N * N;
    for (int x = 0; x < N * N; x++) {
        Mat acc = zero();
        for (int d = 0; d < 2; d++) {
            int xm = shift(N, x, d, -1);
            Mat u = load(U + ((size_t)d * N2 + x) * 18);
            Mat ua = load(UA + ((size_t)d * N2 + x) * 18);
            Mat ub = load(UB + ((size_t)d * N2 + x) * 18);
            acc = add(acc, proj_mat(mul(sub(u, ident()), sub(dag(ub), dag(ua)))));
            Mat um = load(U + ((size_t)d * N2 + xm) * 18);
            Mat uam = load(UA + ((size_t)d * N2 + xm) * 18);
            Mat ubm = load(UB + ((size_t)d * N2 + xm) * 18);
            acc = add(acc, proj_mat(mul(sub(dag(um), ident()), sub(ubm, uam))));
        }
        herm_comps(scale(0.5, acc), pi0 + (size_t)x * 8);
    }
}

// Whole initial condition.  At tau = 0 the transverse electric field and phi
// vanish; the first half step gives E^{1/2} = 0, pi^{1/2} = pi0 and
// U^1 = U^0, phi^1 = dtau * tau_{1/2} * pi0 (the tau = 0 forces vanish).
int orc_init_glasma(int N, double sigma, double m2, int n_sheets, uint64_t seed,
                    double dtau, double *U, double *E, double *phi, double *pi,
                    double *max_res_out) {
    return orc_init_glasma_uv(N, sigma, m2, 0.0, n_sheets, seed, dtau, U, E, phi, pi, max_res_out);
}

int orc_init_glasma_uv(int N, double sigma, double m2, double uv2, int n_sheets, uint64_t seed,
                       double dtau, double *U, double *E, double *phi, double *pi,
                       double *max_res_out) {
    size_t N2 = (size_t)N * N;
    std::vector<double> VA(N2 * 18), VB(N2 * 18), UA(2 * N2 * 18), UB(2 * N2 * 18);
    int rc = orc_wilson_line_uv(N, sigma, m2, uv2, n_sheets, seed, 0, VA.data());
    if (rc) return rc;
    rc = orc_wilson_line_uv(N, sigma, m2, uv2, n_sheets, seed, 1, VB.data());
    if (rc) return rc;
    orc_nucleus_links(N, VA.data(), UA.data());
    orc_nucleus_links(N, VB.data(), UB.data());
    double worst = 0.0;
    int status = 0;
    for (size_t l = 0; l < 2 * N2; l++) {
        double res;
        int it = orc_match_link(UA.data() + l * 18, UB.data() + l * 18, U + l * 18, 1e-13, 100, &res);
        if (it < 0) status = -3;
        worst = std::fmax(worst, res);
    }
    if (max_res_out) *max_res_out = worst;
    std::vector<double> p0(N2 * 8);
    orc_pi0(N, U, UA.data(), UB.data(), p0.data());
    double th = 0.5 * dtau;
    for (size_t k = 0; k < 2 * N2 * 8; k++) E[k] = 0.0;
    for (size_t k = 0; k < N2 * 8; k++) {
        pi[k] = p0[k];
        phi[k] = dtau * th * p0[k];
    }
    return status;
}

void orc_forces(int N, double tau, const double *U, const double *phi, double *FE,
                double *Fpi) {
    Field f{N, U, phi};
    size_t N2 = (size_t)N * N;
    for (int x = 0; x < N * N; x++)
        site_forces(f, tau, x, FE + (size_t)x * 8, FE + (N2 + x) * 8, Fpi + (size_t)x * 8);
}

// One leapfrog step of the reading of Eq. (1):
//   E^{n+1/2} = E^{n-1/2} + dtau F_E(U^n, phi^n; tau_n)
//   pi^{n+1/2} = pi^{n-1/2} + dtau F_pi(U^n, phi^n; tau_n)
//   U^{n+1} = exp(i dtau E^{n+1/2} / tau_{n+1/2}) U^n
//   phi^{n+1} = phi^n + dtau tau_{n+1/2} pi^{n+1/2}
void orc_field_step(int N, int n, double dtau, double *U, double *E, double *phi,
                    double *pi, double *F) {
    size_t N2 = (size_t)N * N;
    double tau = n * dtau, th = (n + 0.5) * dtau;
    std::vector<double> FE(2 * N2 * 8), Fpi(N2 * 8);
    orc_forces(N, tau, U, phi, FE.data(), Fpi.data());
    std::vector<double> Eo(E, E + 2 * N2 * 8), pio(pi, pi + N2 * 8);
    for (size_t k = 0; k < 2 * N2 * 8; k++) E[k] = Eo[k] + dtau * FE[k];
    for (size_t k = 0; k < N2 * 8; k++) pi[k] = pio[k] + dtau * Fpi[k];
    if (F) {
        Field f{N, U, phi};
        for (int x = 0; x < N * N; x++) {
            double Ebar[2][2][8], pibar[8];
            for (int d = 0; d < 2; d++) {
                int xs[2] = {x, shift(N, x, d, -1)};
                for (int w = 0; w < 2; w++)
                    for (int a = 0; a < 8; a++) {
                        size_t k = ((size_t)d * N2 + xs[w]) * 8 + a;
                        Ebar[d][w][a] = 0.5 * (Eo[k] + E[k]);
                    }
            }
            for (int a = 0; a < 8; a++) pibar[a] = 0.5 * (pio[(size_t)x * 8 + a] + pi[(size_t)x * 8 + a]);
            site_fields(f, tau, x, Ebar, pibar, F + (size_t)x * 48);
        }
    }
    for (int d = 0; d < 2; d++)
        for (size_t x = 0; x < N2; x++) {
            double a[8];
            for (int c = 0; c < 8; c++) a[c] = dtau / th * E[(d * N2 + x) * 8 + c];
            Mat u = load(U + (d * N2 + x) * 18);
            store(mul(expi(a), u), U + (d * N2 + x) * 18);
        }
    for (size_t k = 0; k < N2 * 8; k++) phi[k] += dtau * th * pi[k];
}

void orc_field_step_sites(int N, int n, double dtau, const double *U, const double *E,
                          const double *phi, const double *pi, int ns, const int *sites,
                          double *U_new, double *E_new, double *phi_new, double *pi_new,
                          double *F) {
    size_t N2 = (size_t)N * N;
    double tau = n * dtau, th = (n + 0.5) * dtau;
    Field f{N, U, phi};
    // the site-field average needs E^{n+1/2} at x-1 and x-2 as well
    for (int k = 0; k < ns; k++) {
        int x = sites[k];
        int nb[3] = {x, shift(N, x, 0, -1), shift(N, x, 1, -1)};
        double En[2][3][8];   // [dir][which site][comp]
        double pin[8];
        for (int s = 0; s < 3; s++) {
            double FE1[8], FE2[8], Fpi[8];
            site_forces(f, tau, nb[s], FE1, FE2, Fpi);
            for (int a = 0; a < 8; a++) {
                En[0][s][a] = E[((size_t)nb[s]) * 8 + a] + dtau * FE1[a];
                En[1][s][a] = E[(N2 + nb[s]) * 8 + a] + dtau * FE2[a];
                if (s == 0) pin[a] = pi[(size_t)x * 8 + a] + dtau * Fpi[a];
            }
        }
        if (F) {
            double Ebar[2][2][8], pibar[8];
            for (int d = 0; d < 2; d++)
                for (int a = 0; a < 8; a++) {
                    Ebar[d][0][a] = 0.5 * (E[((size_t)d * N2 + x) * 8 + a] + En[d][0][a]);
                    Ebar[d][1][a] = 0.5 * (E[((size_t)d * N2 + nb[1 + d]) * 8 + a] + En[d][1 + d][a]);
                }
            for (int a = 0; a < 8; a++) pibar[a] = 0.5 * (pi[(size_t)x * 8 + a] + pin[a]);
            site_fields(f, tau, x, Ebar, pibar, F + (size_t)k * 48);
        }
        for (int d = 0; d < 2; d++) {
            double a8[8];
            for (int a = 0; a < 8; a++) {
                E_new[((size_t)k * 2 + d) * 8 + a] = En[d][0][a];
                a8[a] = dtau / th * En[d][0][a];
            }
            store(mul(expi(a8), f.link(d, x)), U_new + ((size_t)k * 2 + d) * 18);
        }
        for (int a = 0; a < 8; a++) {
            pi_new[(size_t)k * 8 + a] = pin[a];
            phi_new[(size_t)k * 8 + a] = phi[(size_t)x * 8 + a] + dtau * th * pin[a];
        }
    }
}

void orc_energy(int N, double tau, const double *U, const double *E, const double *phi,
                const double *pi, double out[4]) {
    Field f{N, U, phi};
    size_t N2 = (size_t)N * N;
    double eT = 0, eL = 0, bT = 0, bL = 0;
    for (int x = 0; x < N * N; x++) {
        for (int d = 0; d < 2; d++) {
            Mat e = alg(E + (d * N2 + x) * 8);
            eT += std::real(trace(mul(e, e))) / tau;
            Mat dp = sub(phi_fwd(f, x, d), f.ph(x));
            bT += std::real(trace(mul(dp, dp))) / tau;
        }
        Mat p = alg(pi + (size_t)x * 8);
        eL += tau * std::real(trace(mul(p, p)));
        bL += 2.0 * tau * (3.0 - std::real(trace(plaquette(f, x))));
    }
    out[0] = eT; out[1] = eL; out[2] = bT; out[3] = bL;
}

// Gauss law G(x) = sum_i [E_i(x) - U_i^dag(x-i) E_i(x-i) U_i(x-i)] + i[phi, pi]
void orc_gauss(int N, const double *U, const double *E, const double *phi,
               const double *pi, double *G) {
    Field f{N, U, phi};
    size_t N2 = (size_t)N * N;
    for (int x = 0; x < N * N; x++) {
        Mat g = zero();
        for (int d = 0; d < 2; d++) {
            int xm = shift(N, x, d, -1);
            Mat Um = f.link(d, xm);
            g = add(g, sub(alg(E + (d * N2 + x) * 8), mul(mul(dag(Um), alg(E + (d * N2 + xm) * 8)), Um)));
        }
        Mat ph = f.ph(x), p = alg(pi + (size_t)x * 8);
        g = add(g, scale(IU, sub(mul(ph, p), mul(p, ph))));
        herm_comps(g, G + (size_t)x * 8);
    }
}

// Particle initialisation (Sec. 1 "Probes in Glasma" and Sec. 2 toy model):
// uniform transverse position, eta = 0, color charge Q = U Q0 U^dag with U
// Haar-distributed (QR of a complex Gaussian matrix, Mezzadri 2007) and Q0
// diagonal with q2 = Q^aQ^a = 4, q3 = d_abc Q^aQ^bQ^c = 10/3 (the stated
// moments <Q^aQ^b> = delta^ab/2, <Q^aQ^bQ^c> = d^abc/4).
// Draw layout for particle i of species s: counter (i, j, 2 + s, 0), j = 0
// position, j = 1 azimuth, j = 2..10 the nine Gaussian pairs of the matrix.
void orc_particles_init(int N, uint64_t seed, int species_id, int kind, double p0,
                        int np, int *cell, double *off, double *eta, double *p,
                        double *Q, double *p0v) {
    // roots of lambda^3 - lambda - 5/18 = 0 by bisection on three brackets
    double q0[3];
    double brk[3][2] = {{1.0, 1.5}, {-0.5, 0.0}, {-1.0, -0.5}};
    for (int r = 0; r < 3; r++) {
        double lo = brk[r][0], hi = brk[r][1];
        auto fpoly = [](double l) { return l * l * l - l - 5.0 / 18.0; };
        for (int it = 0; it < 200; it++) {
            double mid = 0.5 * (lo + hi);
            if ((fpoly(lo) < 0) == (fpoly(mid) < 0)) lo = mid; else hi = mid;
        }
        q0[r] = 0.5 * (lo + hi);
    }
    Mat Q0 = zero();
    for (int r = 0; r < 3; r++) Q0.m[r][r] = q0[r];
    const double twopi = 6.283185307179586476925286766559;
    for (int i = 0; i < np; i++) {
        uint32_t w[4];
        uint32_t stream = (uint32_t)(2 + species_id);
        draw(seed, (uint32_t)i, 0u, stream, w);
        double X = u53(w[0], w[1]) * N, Y = u53(w[2], w[3]) * N;
        double fx = std::floor(X + 0.5), fy = std::floor(Y + 0.5);
        cell[2 * i] = ((int)fx) % N;
        cell[2 * i + 1] = ((int)fy) % N;
        off[2 * i] = X - fx;
        off[2 * i + 1] = Y - fy;
        eta[i] = 0.0;
        draw(seed, (uint32_t)i, 1u, stream, w);
        double phiaz = twopi * u53(w[0], w[1]);
        double px, py;
        if (kind == 0) {
            px = p0 * std::cos(phiaz);
            py = p0 * std::sin(phiaz);
        } else {
            px = p0;
            py = 0.0;
        }
        p[3 * i] = px; p[3 * i + 1] = py; p[3 * i + 2] = 0.0;
        p0v[3 * i] = px; p0v[3 * i + 1] = py; p0v[3 * i + 2] = 0.0;
        Mat Z;
        for (int k = 0; k < 9; k++) {
            draw(seed, (uint32_t)i, (uint32_t)(2 + k), stream, w);
            double g0, g1;
            gauss2(w, &g0, &g1);
            Z.m[k / 3][k % 3] = cd(g0, g1);
        }
        // Gram-Schmidt on the columns of Z (R then has a positive diagonal)
        Mat Uh = zero();
        for (int c = 0; c < 3; c++) {
            cd v[3] = {Z.m[0][c], Z.m[1][c], Z.m[2][c]};
            for (int pcol = 0; pcol < c; pcol++) {
                cd dot = 0.0;
                for (int r = 0; r < 3; r++) dot += std::conj(Uh.m[r][pcol]) * Z.m[r][c];
                for (int r = 0; r < 3; r++) v[r] -= dot * Uh.m[r][pcol];
            }
            double nr = std::sqrt(std::norm(v[0]) + std::norm(v[1]) + std::norm(v[2]));
            for (int r = 0; r < 3; r++) Uh.m[r][c] = v[r] / nr;
        }
        herm_comps(mul(mul(Uh, Q0), dag(Uh)), Q + (size_t)8 * i);
    }
}

// One step of Wong's equations, Eq. (2), for the particles (reading: Boris
// push of dp/dtau = Q^a (E^a + v x B^a) in the local frame, with the
// longitudinal momentum kept as P_eta = tau^2 p^eta so that the Milne
// connection term is exact; color rotated by the link-built Wilson line of
// the path, which conserves the Casimirs as the paper requires).
void orc_particle_step(int N, int n, double dtau, const double *U, const double *phi,
                       const double *F, int np, int *cell, double *off, double *eta,
                       double *p, double *Q, const double *p0v, const int *species,
                       int nspecies, const double *mass, const int *nform,
                       double *series) {
    Field f{N, U, phi};
    double tau = n * dtau, th = (n + 0.5) * dtau;
    for (int i = 0; i < np; i++) {
        int s = species[i];
        if (s < 0 || s >= nspecies || n < nform[s]) continue;
        double m = mass[s];
        int x = site(N, cell[2 * i], cell[2 * i + 1]);
        const double *Fx = F + (size_t)x * 48;
        double e[3], b[3];
        for (int k = 0; k < 3; k++) {
            e[k] = 0.0;
            b[k] = 0.0;
            for (int a = 0; a < 8; a++) {
                e[k] += Q[8 * i + a] * Fx[8 * k + a];
                b[k] += Q[8 * i + a] * Fx[8 * (3 + k) + a];
            }
        }
        // Boris kick at tau_n
        double pl[3] = {p[3 * i], p[3 * i + 1], p[3 * i + 2] / tau};
        double pm[3];
        for (int k = 0; k < 3; k++) pm[k] = pl[k] + 0.5 * dtau * e[k];
        double g = std::sqrt(m * m + pm[0] * pm[0] + pm[1] * pm[1] + pm[2] * pm[2]);
        double t[3];
        for (int k = 0; k < 3; k++) t[k] = b[k] * dtau / (2.0 * g);
        double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
        double sv[3];
        for (int k = 0; k < 3; k++) sv[k] = 2.0 * t[k] / (1.0 + t2);
        double pp[3] = {pm[0] + (pm[1] * t[2] - pm[2] * t[1]),
                        pm[1] + (pm[2] * t[0] - pm[0] * t[2]),
                        pm[2] + (pm[0] * t[1] - pm[1] * t[0])};
        double pq[3] = {pm[0] + (pp[1] * sv[2] - pp[2] * sv[1]),
                        pm[1] + (pp[2] * sv[0] - pp[0] * sv[2]),
                        pm[2] + (pp[0] * sv[1] - pp[1] * sv[0])};
        for (int k = 0; k < 3; k++) pl[k] = pq[k] + 0.5 * dtau * e[k];
        p[3 * i] = pl[0];
        p[3 * i + 1] = pl[1];
        p[3 * i + 2] = tau * pl[2];
        // drift to tau_{n+1} with velocities at tau_{n+1/2}
        double Peta = p[3 * i + 2];
        double pzh = Peta / th;
        double ptau = std::sqrt(m * m + pl[0] * pl[0] + pl[1] * pl[1] + pzh * pzh);
        double eta_old = eta[i];
        off[2 * i] += dtau * pl[0] / ptau;
        off[2 * i + 1] += dtau * pl[1] / ptau;
        double deta = dtau * Peta / (th * th * ptau);
        eta[i] = eta_old + deta;
        // color rotation along eta with the old cell's phi: Q <- W Q W^dag
        Mat Qm = alg(Q + (size_t)8 * i);
        double pa[8];
        for (int a = 0; a < 8; a++) pa[a] = -phi[(size_t)x * 8 + a] * deta;
        Mat W = expi(pa);
        Qm = mul(mul(W, Qm), dag(W));
        // cell crossings, x first then y, color carried by the crossed link
        for (int d = 0; d < 2; d++) {
            int c = site(N, cell[0 + 2 * i], cell[1 + 2 * i]);
            if (off[2 * i + d] >= 0.5) {
                Mat Ul = f.link(d, c);
                Qm = mul(mul(dag(Ul), Qm), Ul);
                off[2 * i + d] -= 1.0;
                cell[2 * i + d] = (cell[2 * i + d] + 1) % N;
            } else if (off[2 * i + d] < -0.5) {
                int cm = shift(N, c, d, -1);
                Mat Ul = f.link(d, cm);
                Qm = mul(mul(Ul, Qm), dag(Ul));
                off[2 * i + d] += 1.0;
                cell[2 * i + d] = (cell[2 * i + d] + N - 1) % N;
            }
        }
        herm_comps(Qm, Q + (size_t)8 * i);
        // broadening at tau_{n+1/2}: delta p_i^2 = p_i^2 - p_i^2(tau_form)
        double etab = 0.5 * (eta_old + eta[i]);
        double pzlab = ptau * std::sinh(etab) + pzh * std::cosh(etab);
        series[4 * s + 0] += pl[0] * pl[0] - p0v[3 * i] * p0v[3 * i];
        series[4 * s + 1] += pl[1] * pl[1] - p0v[3 * i + 1] * p0v[3 * i + 1];
        series[4 * s + 2] += pzlab * pzlab - p0v[3 * i + 2] * p0v[3 * i + 2];
        series[4 * s + 3] += 1.0;
    }
}

int orc_run(int N, double sigma, double m2, int n_sheets, uint64_t seed, double dtau,
            int n_steps, int nspecies, const int *kind, const double *mass,
            const double *p0, const int *nform, const int *np, double *U, double *E,
            double *phi, double *pi, int *cell, double *off, double *eta, double *p,
            double *Q, double *p0v, int *species, double *series_out) {
    double res;
    int rc = orc_init_glasma(N, sigma, m2, n_sheets, seed, dtau, U, E, phi, pi, &res);
    if (rc) return rc;
    int total = 0;
    for (int s = 0; s < nspecies; s++) {
        orc_particles_init(N, seed, s, kind[s], p0[s], np[s], cell + 2 * total, off + 2 * total,
                           eta + total, p + 3 * total, Q + 8 * (size_t)total, p0v + 3 * total);
        for (int i = 0; i < np[s]; i++) species[total + i] = s;
        total += np[s];
    }
    size_t N2 = (size_t)N * N;
    std::vector<double> F(N2 * 48), Uold(2 * N2 * 18), phiold(N2 * 8);
    for (int k = 0; k < n_steps; k++) {
        int n = 1 + k;
        std::memcpy(Uold.data(), U, sizeof(double) * 2 * N2 * 18);
        std::memcpy(phiold.data(), phi, sizeof(double) * N2 * 8);
        orc_field_step(N, n, dtau, U, E, phi, pi, F.data());
        double *row = series_out + (size_t)k * nspecies * 4;
        for (int j = 0; j < nspecies * 4; j++) row[j] = 0.0;
        orc_particle_step(N, n, dtau, Uold.data(), phiold.data(), F.data(), total, cell, off,
                          eta, p, Q, p0v, species, nspecies, mass, nform, row);
    }
    return 0;
}

}  // extern "C"
