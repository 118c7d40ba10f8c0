// su3.hpp -- register-resident SU(3) arithmetic for gfx950 kernels.
//
// Matrices are 3x3 complex held as separate real and imaginary 3x3 arrays so
// that every entry is its own register; all loops are unrolled.  Algebra
// elements X = X^a T^a (T^a = lambda^a/2) travel as 8 reals.  T is float or
// double; the same code serves both precisions.
#pragma once
#include <hip/hip_runtime.h>

namespace gl {

template <typename T>
struct M3 {
    T re[3][3];
    T im[3][3];
};

template <typename T>
__device__ __forceinline__ M3<T> m_zero() {
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) { r.re[i][j] = T(0); r.im[i][j] = T(0); }
    return r;
}

template <typename T>
__device__ __forceinline__ M3<T> m_ident() {
    M3<T> r = m_zero<T>();
    r.re[0][0] = r.re[1][1] = r.re[2][2] = T(1);
    return r;
}

// A B
template <typename T>
__device__ __forceinline__ M3<T> mul(const M3<T> &a, const M3<T> &b) {
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            T sr = T(0), si = T(0);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                sr = fma(a.re[i][k], b.re[k][j], sr);
                sr = fma(-a.im[i][k], b.im[k][j], sr);
                si = fma(a.re[i][k], b.im[k][j], si);
                si = fma(a.im[i][k], b.re[k][j], si);
            }
            r.re[i][j] = sr;
            r.im[i][j] = si;
        }
    return r;
}

// A B^dag
template <typename T>
__device__ __forceinline__ M3<T> mul_nd(const M3<T> &a, const M3<T> &b) {
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            T sr = T(0), si = T(0);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                // a[i][k] * conj(b[j][k])
                sr = fma(a.re[i][k], b.re[j][k], sr);
                sr = fma(a.im[i][k], b.im[j][k], sr);
                si = fma(a.im[i][k], b.re[j][k], si);
                si = fma(-a.re[i][k], b.im[j][k], si);
            }
            r.re[i][j] = sr;
            r.im[i][j] = si;
        }
    return r;
}

// A^dag B
template <typename T>
__device__ __forceinline__ M3<T> mul_dn(const M3<T> &a, const M3<T> &b) {
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            T sr = T(0), si = T(0);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                // conj(a[k][i]) * b[k][j]
                sr = fma(a.re[k][i], b.re[k][j], sr);
                sr = fma(a.im[k][i], b.im[k][j], sr);
                si = fma(a.re[k][i], b.im[k][j], si);
                si = fma(-a.im[k][i], b.re[k][j], si);
            }
            r.re[i][j] = sr;
            r.im[i][j] = si;
        }
    return r;
}

template <typename T>
__device__ __forceinline__ M3<T> add(const M3<T> &a, const M3<T> &b) {
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            r.re[i][j] = a.re[i][j] + b.re[i][j];
            r.im[i][j] = a.im[i][j] + b.im[i][j];
        }
    return r;
}

template <typename T>
__device__ __forceinline__ M3<T> sub(const M3<T> &a, const M3<T> &b) {
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            r.re[i][j] = a.re[i][j] - b.re[i][j];
            r.im[i][j] = a.im[i][j] - b.im[i][j];
        }
    return r;
}

// ---- algebra <-> matrix -----------------------------------------------------
// Hermitian X = x^a T^a written out from the Gell-Mann matrices.
template <typename T>
__device__ __forceinline__ M3<T> herm_from_alg(const T *x) {
    const T h = T(0.5);
    const T s3 = T(0.57735026918962576451);   // 1/sqrt(3)
    M3<T> r;
    r.re[0][0] = h * (x[2] + s3 * x[7]);
    r.re[1][1] = h * (-x[2] + s3 * x[7]);
    r.re[2][2] = -s3 * x[7];
    r.im[0][0] = r.im[1][1] = r.im[2][2] = T(0);
    r.re[0][1] = h * x[0];  r.im[0][1] = -h * x[1];
    r.re[1][0] = h * x[0];  r.im[1][0] = h * x[1];
    r.re[0][2] = h * x[3];  r.im[0][2] = -h * x[4];
    r.re[2][0] = h * x[3];  r.im[2][0] = h * x[4];
    r.re[1][2] = h * x[5];  r.im[1][2] = -h * x[6];
    r.re[2][1] = h * x[5];  r.im[2][1] = h * x[6];
    return r;
}

// x^a = 2 Re Tr(T^a H) of a hermitian H (only its hermitian part counts).
template <typename T>
__device__ __forceinline__ void alg_from_herm(const M3<T> &H, T *x) {
    const T s3 = T(0.57735026918962576451);
    x[0] = H.re[0][1] + H.re[1][0];
    x[1] = H.im[1][0] - H.im[0][1];
    x[2] = H.re[0][0] - H.re[1][1];
    x[3] = H.re[0][2] + H.re[2][0];
    x[4] = H.im[2][0] - H.im[0][2];
    x[5] = H.re[1][2] + H.re[2][1];
    x[6] = H.im[2][1] - H.im[1][2];
    x[7] = s3 * (H.re[0][0] + H.re[1][1] - T(2) * H.re[2][2]);
}

// Components of [M]_X = (M - M^dag)/(2i) - trace/3:  x^a = 2 Im Tr(T^a M).
template <typename T>
__device__ __forceinline__ void alg_proj(const M3<T> &M, T *x) {
    const T s3 = T(0.57735026918962576451);
    x[0] = M.im[0][1] + M.im[1][0];
    x[1] = M.re[0][1] - M.re[1][0];
    x[2] = M.im[0][0] - M.im[1][1];
    x[3] = M.im[0][2] + M.im[2][0];
    x[4] = M.re[0][2] - M.re[2][0];
    x[5] = M.im[1][2] + M.im[2][1];
    x[6] = M.re[1][2] - M.re[2][1];
    x[7] = s3 * (M.im[0][0] + M.im[1][1] - T(2) * M.im[2][2]);
}

// Tr(A B) real part for hermitian A, B
template <typename T>
__device__ __forceinline__ T re_tr_mul(const M3<T> &a, const M3<T> &b) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) s += a.re[i][k] * b.re[k][i] - a.im[i][k] * b.im[k][i];
    return s;
}

// ---- hermitian results computed from their upper triangle -------------------
// A product known to be hermitian only needs its entries (i, j), i < j, and
// the real parts of its diagonal; these give the algebra components exactly
// as alg_from_herm does for a hermitian matrix.
template <typename T>
__device__ __forceinline__ void alg_from_upper(const T d[3], const T ur[3], const T ui[3], T *x) {
    // ur/ui: entries (0,1), (0,2), (1,2)
    const T s3 = T(0.57735026918962576451);
    x[0] = T(2) * ur[0];
    x[1] = T(-2) * ui[0];
    x[2] = d[0] - d[1];
    x[3] = T(2) * ur[1];
    x[4] = T(-2) * ui[1];
    x[5] = T(2) * ur[2];
    x[6] = T(-2) * ui[2];
    x[7] = s3 * (d[0] + d[1] - T(2) * d[2]);
}

// algebra components of the hermitian U^dag W (W = X U with X hermitian)
template <typename T>
__device__ __forceinline__ void alg_herm_dn(const M3<T> &U, const M3<T> &W, T *x) {
    T d[3], ur[3], ui[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        T s = T(0);
#pragma unroll
        for (int k = 0; k < 3; k++) s = fma(U.re[k][i], W.re[k][i], fma(U.im[k][i], W.im[k][i], s));
        d[i] = s;
    }
    constexpr int I[3] = {0, 0, 1}, J[3] = {1, 2, 2};
#pragma unroll
    for (int e = 0; e < 3; e++) {
        T sr = T(0), si = T(0);
#pragma unroll
        for (int k = 0; k < 3; k++) {   // conj(U_ki) W_kj
            sr = fma(U.re[k][I[e]], W.re[k][J[e]], fma(U.im[k][I[e]], W.im[k][J[e]], sr));
            si = fma(U.re[k][I[e]], W.im[k][J[e]], fma(-U.im[k][I[e]], W.re[k][J[e]], si));
        }
        ur[e] = sr;
        ui[e] = si;
    }
    alg_from_upper(d, ur, ui, x);
}

// algebra components of the hermitian W U^dag (W = U X with X hermitian)
template <typename T>
__device__ __forceinline__ void alg_herm_nd(const M3<T> &W, const M3<T> &U, T *x) {
    T d[3], ur[3], ui[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        T s = T(0);
#pragma unroll
        for (int k = 0; k < 3; k++) s = fma(W.re[i][k], U.re[i][k], fma(W.im[i][k], U.im[i][k], s));
        d[i] = s;
    }
    constexpr int I[3] = {0, 0, 1}, J[3] = {1, 2, 2};
#pragma unroll
    for (int e = 0; e < 3; e++) {
        T sr = T(0), si = T(0);
#pragma unroll
        for (int k = 0; k < 3; k++) {   // W_ik conj(U_jk)
            sr = fma(W.re[I[e]][k], U.re[J[e]][k], fma(W.im[I[e]][k], U.im[J[e]][k], sr));
            si = fma(W.im[I[e]][k], U.re[J[e]][k], fma(-W.re[I[e]][k], U.im[J[e]][k], si));
        }
        ur[e] = sr;
        ui[e] = si;
    }
    alg_from_upper(d, ur, ui, x);
}

// x^c = sum_ab f_abc a^a b^b: the components of -i[A, B] for A = a^a T^a and
// B = b^b T^b, from the SU(3) structure constants ([T^a, T^b] = i f_abc T^c;
// f_123 = 1, f_147 = f_246 = f_257 = f_345 = 1/2, f_156 = f_367 = -1/2,
// f_458 = f_678 = sqrt(3)/2, written here 0-based).
template <typename T>
__device__ __forceinline__ void alg_comm(const T *a, const T *b, T *c) {
    const T h = T(0.5), r3 = T(0.86602540378443864676);
#pragma unroll
    for (int k = 0; k < 8; k++) c[k] = T(0);
    auto term = [&](int i, int j, int k, T f) {   // every cyclic order of one f_ijk
        c[k] = fma(f, a[i] * b[j] - a[j] * b[i], c[k]);
        c[i] = fma(f, a[j] * b[k] - a[k] * b[j], c[i]);
        c[j] = fma(f, a[k] * b[i] - a[i] * b[k], c[j]);
    };
    term(0, 1, 2, T(1));
    term(0, 3, 6, h);
    term(0, 4, 5, -h);
    term(1, 3, 5, h);
    term(1, 4, 6, h);
    term(2, 3, 4, h);
    term(2, 5, 6, -h);
    term(3, 4, 7, r3);
    term(5, 6, 7, r3);
}

// Q^2 of a hermitian Q from its upper triangle (the lower one by conjugation)
template <typename T>
__device__ __forceinline__ M3<T> herm_square(const M3<T> &Q) {
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = i; j < 3; j++) {
            T sr = T(0), si = T(0);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                sr = fma(Q.re[i][k], Q.re[k][j], fma(-Q.im[i][k], Q.im[k][j], sr));
                si = fma(Q.re[i][k], Q.im[k][j], fma(Q.im[i][k], Q.re[k][j], si));
            }
            r.re[i][j] = sr;
            r.im[i][j] = i == j ? T(0) : si;
            if (i != j) {
                r.re[j][i] = sr;
                r.im[j][i] = -si;
            }
        }
    return r;
}

// ---- exponential of i Q for hermitian traceless Q ---------------------------
// Cayley-Hamilton form exp(iQ) = f0 + f1 Q + f2 Q^2.  For c1 = Tr(Q^2)/2 up
// to 0.12 (spectral norm |Q| <= sqrt(4 c1 / 3) <= 0.4) the f_j are the power
// series sum_k (iQ)^k / k! with Q^k = a_k + b_k Q + c_k Q^2 reduced by
// Q^3 = c1 Q + c0 (c0 = det Q): a' = c0 c, b' = a + c1 c, c' = b.  Truncated
// after K terms its error is below |Q|^(K+1) e^|Q| / (K+1)!: 8e-19 for
// K = 14 (double), 1e-9 for K = 8 (float).  Larger Q take the closed form of
// C. Morningstar and M. Peardon, Phys. Rev. D 69 (2004) 054501, Sec. III.
template <typename T>
__device__ __forceinline__ M3<T> expi_herm(const M3<T> &Q) {
    M3<T> Q2 = herm_square(Q);
    T c1 = T(0.5) * (Q2.re[0][0] + Q2.re[1][1] + Q2.re[2][2]);
    // det of hermitian traceless Q = Tr(Q^3)/3
    T c0 = re_tr_mul(Q, Q2) * T(1.0 / 3.0);
    T f0r, f0i, f1r, f1i, f2r, f2i;
    if (c1 <= T(0.12)) {
        constexpr int K = sizeof(T) == 8 ? 14 : 8;
        T A = T(1), B = T(0), C = T(0);   // a_k / k!, b_k / k!, c_k / k!
        f0r = f0i = f1r = f1i = f2r = f2i = T(0);
#pragma unroll
        for (int k = 0; k <= K; k++) {
            switch (k & 3) {   // i^k
                case 0: f0r += A; f1r += B; f2r += C; break;
                case 1: f0i += A; f1i += B; f2i += C; break;
                case 2: f0r -= A; f1r -= B; f2r -= C; break;
                default: f0i -= A; f1i -= B; f2i -= C; break;
            }
            const T r = T(1) / T(k + 1);
            const T An = c0 * C * r, Bn = fma(c1, C, A) * r;
            C = B * r;
            A = An;
            B = Bn;
        }
    } else {
        bool neg = c0 < T(0);
        T c0a = neg ? -c0 : c0;
        T c1o3 = c1 * T(1.0 / 3.0);
        T sq = sqrt(c1o3);
        T c0max = T(2) * c1o3 * sq;
        T ratio = c0a / c0max;
        ratio = ratio > T(1) ? T(1) : ratio;
        T theta = acos(ratio);
        T u = sq * cos(theta * T(1.0 / 3.0));
        T w = sqrt(c1) * sin(theta * T(1.0 / 3.0));
        T u2 = u * u, w2 = w * w;
        T xi0;
        if (w < T(0.05)) xi0 = T(1) - w2 * T(1.0 / 6.0) * (T(1) - w2 * T(1.0 / 20.0) * (T(1) - w2 * T(1.0 / 42.0)));
        else xi0 = sin(w) / w;
        T cw = cos(w);
        T c2u = cos(T(2) * u), s2u = sin(T(2) * u);
        T cu = cos(u), su = sin(u);   // e^{-iu} = cu - i su
        // h0 = (u^2 - w^2) e^{2iu} + e^{-iu} [8u^2 cos w + 2iu(3u^2 + w^2) xi0]
        T a_r = T(8) * u2 * cw, a_i = T(2) * u * (T(3) * u2 + w2) * xi0;
        T h0r = (u2 - w2) * c2u + (cu * a_r + su * a_i);
        T h0i = (u2 - w2) * s2u + (cu * a_i - su * a_r);
        // h1 = 2u e^{2iu} - e^{-iu} [2u cos w - i(3u^2 - w^2) xi0]
        T b_r = T(2) * u * cw, b_i = -(T(3) * u2 - w2) * xi0;
        T h1r = T(2) * u * c2u - (cu * b_r + su * b_i);
        T h1i = T(2) * u * s2u - (cu * b_i - su * b_r);
        // h2 = e^{2iu} - e^{-iu} [cos w + 3iu xi0]
        T d_r = cw, d_i = T(3) * u * xi0;
        T h2r = c2u - (cu * d_r + su * d_i);
        T h2i = s2u - (cu * d_i - su * d_r);
        T inv = T(1) / (T(9) * u2 - w2);
        f0r = h0r * inv; f0i = h0i * inv;
        f1r = h1r * inv; f1i = h1i * inv;
        f2r = h2r * inv; f2i = h2i * inv;
        if (neg) {   // f_j(-c0) = (-1)^j conj(f_j(c0))
            f0i = -f0i;
            f1r = -f1r;
            f2i = -f2i;
        }
    }
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            // f1 Q + f2 Q^2 with Q, Q^2 hermitian (complex entries)
            T qr = Q.re[i][j], qi = Q.im[i][j], pr = Q2.re[i][j], pi = Q2.im[i][j];
            T rr = f1r * qr - f1i * qi + f2r * pr - f2i * pi;
            T ri = f1r * qi + f1i * qr + f2r * pi + f2i * pr;
            if (i == j) { rr += f0r; ri += f0i; }
            r.re[i][j] = rr;
            r.im[i][j] = ri;
        }
    return r;
}

// exp(i s x^a T^a)
template <typename T>
__device__ __forceinline__ M3<T> expi_alg(const T *x, T s) {
    T y[8];
#pragma unroll
    for (int a = 0; a < 8; a++) y[a] = s * x[a];
    return expi_herm(herm_from_alg(y));
}

// Gram-Schmidt on rows 0 and 1, row 2 = conj(r0 x r1): nearest-by-construction SU(3)
template <typename T>
__device__ __forceinline__ M3<T> reunitarize(const M3<T> &m) {
    M3<T> r;
    T n0 = T(0);
#pragma unroll
    for (int k = 0; k < 3; k++) n0 += m.re[0][k] * m.re[0][k] + m.im[0][k] * m.im[0][k];
    T in0 = T(1) / sqrt(n0);
#pragma unroll
    for (int k = 0; k < 3; k++) { r.re[0][k] = m.re[0][k] * in0; r.im[0][k] = m.im[0][k] * in0; }
    // <r0, m1> = sum conj(r0_k) m1_k
    T dr = T(0), di = T(0);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        dr += r.re[0][k] * m.re[1][k] + r.im[0][k] * m.im[1][k];
        di += r.re[0][k] * m.im[1][k] - r.im[0][k] * m.re[1][k];
    }
    T v_r[3], v_i[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        v_r[k] = m.re[1][k] - (dr * r.re[0][k] - di * r.im[0][k]);
        v_i[k] = m.im[1][k] - (dr * r.im[0][k] + di * r.re[0][k]);
    }
    T n1 = v_r[0] * v_r[0] + v_i[0] * v_i[0] + v_r[1] * v_r[1] + v_i[1] * v_i[1] + v_r[2] * v_r[2] + v_i[2] * v_i[2];
    T in1 = T(1) / sqrt(n1);
#pragma unroll
    for (int k = 0; k < 3; k++) { r.re[1][k] = v_r[k] * in1; r.im[1][k] = v_i[k] * in1; }
    // row2 = conj(r0 x r1)
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int a = (k + 1) % 3, b = (k + 2) % 3;
        T cr = r.re[0][a] * r.re[1][b] - r.im[0][a] * r.im[1][b] - (r.re[0][b] * r.re[1][a] - r.im[0][b] * r.im[1][a]);
        T ci = r.re[0][a] * r.im[1][b] + r.im[0][a] * r.re[1][b] - (r.re[0][b] * r.im[1][a] + r.im[0][b] * r.re[1][a]);
        r.re[2][k] = cr;
        r.im[2][k] = -ci;
    }
    return r;
}

// Products with a hermitian X = x^a T^a as herm_from_alg builds it, whose
// diagonal is real: the terms with its (zero) imaginary diagonal are left out,
// and the others are summed in the order of mul.  Without fast-math the
// compiler keeps an FMA by a zero, so mul would spend 18 of its 108 FMAs on
// them.
template <typename T>
__device__ __forceinline__ M3<T> mul_herm_u(const M3<T> &X, const M3<T> &b) {   // X b
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            T sr = T(0), si = T(0);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                sr = fma(X.re[i][k], b.re[k][j], sr);
                if (k != i) sr = fma(-X.im[i][k], b.im[k][j], sr);
                si = fma(X.re[i][k], b.im[k][j], si);
                if (k != i) si = fma(X.im[i][k], b.re[k][j], si);
            }
            r.re[i][j] = sr;
            r.im[i][j] = si;
        }
    return r;
}
template <typename T>
__device__ __forceinline__ M3<T> mul_u_herm(const M3<T> &a, const M3<T> &X) {   // a X
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            T sr = T(0), si = T(0);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                sr = fma(a.re[i][k], X.re[k][j], sr);
                if (k != j) sr = fma(-a.im[i][k], X.im[k][j], sr);
                if (k != j) si = fma(a.re[i][k], X.im[k][j], si);
                si = fma(a.im[i][k], X.re[k][j], si);
            }
            r.re[i][j] = sr;
            r.im[i][j] = si;
        }
    return r;
}

// U^dag X U and U X U^dag of the hermitian X = x^a T^a, returned as algebra
// components.  HERM = false takes the general product (the same sums, with
// the zero terms): in the FP32 field step the shorter product changed the
// register allocation into more spills (batch FP32 field kernel 1 -> 8 dwords,
// 64-event batch 0.920 -> 0.930 s), so that kernel keeps it.
template <bool HERM = true, typename T>
__device__ __forceinline__ void transport_dn(const M3<T> &U, const T *x, T *out) {
    if constexpr (HERM) alg_herm_dn(U, mul_herm_u(herm_from_alg(x), U), out);
    else alg_herm_dn(U, mul(herm_from_alg(x), U), out);
}
template <bool HERM = true, typename T>
__device__ __forceinline__ void transport_nd(const M3<T> &U, const T *x, T *out) {
    if constexpr (HERM) alg_herm_nd(mul_u_herm(U, herm_from_alg(x)), U, out);
    else alg_herm_nd(mul(U, herm_from_alg(x)), U, out);
}

// ---- lane exchanges within a wave (DPP, no LDS traffic) -------------------
// dpp_ctrl codes: quad_perm(1,0,3,2) swaps lanes 2k and 2k+1, quad_perm(2,3,0,1)
// swaps pairs within a quad, row_half_mirror reverses 8 lanes, row_mirror 16.
constexpr int kDppSwap1 = 0xB1, kDppSwap2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    typedef int i32x2 __attribute__((ext_vector_type(2)));
    i32x2 h = __builtin_bit_cast(i32x2, v);
    h.x = __builtin_amdgcn_update_dpp(0, h.x, CTRL, 0xF, 0xF, false);
    h.y = __builtin_amdgcn_update_dpp(0, h.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, h);
}

// Sum over the 16 lanes of each row of the wave; every lane of a row gets
// the same total (each step adds two partial sums that are equal as a pair).
template <typename T>
__device__ __forceinline__ T row_sum(T v) {
    v += dpp<kDppSwap1>(v);
    v += dpp<kDppSwap2>(v);
    v += dpp<kDppHalfMirror>(v);
    v += dpp<kDppMirror>(v);
    return v;
}

// ---- structure-of-arrays loads/stores ---------------------------------------
// Arrays are read and written through buffer resources: the array base lives
// in scalar registers, the lane's byte offset is one 32-bit vector register
// and the plane offset a scalar, so the many plane accesses of a site cost no
// per-lane 64-bit address arithmetic.  Lattice planes hold at most 2^20 sites,
// and the particle capacity is capped so that the widest particle array (the
// record, in chunk planes over all slots) stays below 2^31 bytes, so every
// byte offset fits in 32 bits.  Offsets x may include a whole number of planes (a lane-dependent
// choice of planes).
constexpr int kBufConfig = 0x00020000;   // raw 32-bit data, gfx9-family layout
constexpr int kLinkVals = 12;            // stored values of a link (its first two rows)
// cache-policy operand of a buffer access: the non-temporal hint, for data
// read or written once per kernel and not again until much other traffic
// has passed (it then leaves the caches to data that is reused).
// stream_policy(ST) is the policy of such streamed arrays: the hint when
// the kernels' working set overflows the 256 MB last-level cache (ST), none
// when it fits.  A single FP64 event (field state, site fields, particles:
// over 400 MB per step at 512^2) overflows it: streaming the particle
// records and most of the new field state (E, phi, pi; the links, which the
// next step stages with their halo, stay cached) keeps the gathered site
// fields cached (push 113 -> 94 us).  A single FP32 event fits, and the hint
// only sends the next kernel's inputs to HBM (step 89 -> 100 us).  A batch
// of events overflows it in either precision (FP32 64-event batch 986 ->
// 969 ms).  kStreamed<T> is the single-event choice.
constexpr int kNonTemporal = 2;
constexpr int stream_policy(bool streamed) { return streamed ? kNonTemporal : 0; }
template <typename T>
constexpr bool kStreamed = sizeof(T) == 8;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, 0x7FFFFFFF, kBufConfig);
}
__device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ __forceinline__ double bld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
__device__ __forceinline__ int32_t bld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, int32_t) {
    return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
}
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, vo, so, 0);
}
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, double v) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, 0);
}
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, int32_t v) {
    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)v, r, vo, so, 0);
}

// element x of plane k of the array at p (planes n2 elements apart)
template <typename T>
__device__ __forceinline__ T pl_ld(const T *p, size_t n2, int k, size_t x) {
    return bld(buf(p), (uint32_t)(x * sizeof(T)), (uint32_t)((size_t)k * n2 * sizeof(T)), T());
}
template <typename T>
__device__ __forceinline__ void pl_st(T *p, size_t n2, int k, size_t x, T v) {
    bst(buf(p), (uint32_t)(x * sizeof(T)), (uint32_t)((size_t)k * n2 * sizeof(T)), v);
}
// element x of a single array
template <typename T>
__device__ __forceinline__ T el_ld(const T *p, size_t x) {
    return bld(buf(p), (uint32_t)(x * sizeof(T)), 0u, T());
}
template <typename T>
__device__ __forceinline__ void el_st(T *p, size_t x, T v) {
    bst(buf(p), (uint32_t)(x * sizeof(T)), 0u, v);
}
// element x of a 32-bit integer array with the cache policy CP
template <int CP>
__device__ __forceinline__ int32_t el_ld_i32(const int32_t *p, size_t x) {
    return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(buf(p), (uint32_t)(x * 4), 0u, CP);
}
template <int CP>
__device__ __forceinline__ void el_st_i32(int32_t *p, size_t x, int32_t v) {
    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)v, buf(p), (uint32_t)(x * 4), 0u, CP);
}

// Chunked planes: values are grouped in 16-byte chunks of NV = 16 /
// sizeof(T) consecutive values k; chunk plane k / NV holds the chunks of
// all n2 sites in site order, so value k of site x sits at element
// ((k / NV) n2 + x) NV + k mod NV.  One lane reads or writes a chunk in one
// 16-byte access, and lanes of neighbouring sites touch neighbouring chunks.
template <typename T>
__device__ __forceinline__ T chunk_ld(const T *p, size_t n2, size_t x, int k) {
    constexpr int NV = 16 / (int)sizeof(T);
    return bld(buf(p), (uint32_t)(x * 16 + (k % NV) * sizeof(T)), (uint32_t)((size_t)(k / NV) * n2 * 16), T());
}
template <int CP = 0, typename T>
__device__ __forceinline__ void chunk_ld16(const T *p, size_t n2, size_t x, int k, T *out) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    struct V { T v[16 / sizeof(T)]; };
    constexpr int NV = 16 / (int)sizeof(T);
    const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(buf(p), (uint32_t)(x * 16),
                                                          (uint32_t)((size_t)(k / NV) * n2 * 16), CP);
    const V r = __builtin_bit_cast(V, w);
#pragma unroll
    for (int i = 0; i < NV; i++) out[i] = r.v[i];
}
// A store of more than 8 bytes needs one wait state before a vector
// instruction may overwrite its data registers.  The compiler inserts it only
// for buffer stores without a scalar offset register, and on gfx950 the
// hazard is also there with one: the data of a 16-byte store was overwritten
// by the next instruction in a few lanes.  Every 16-byte store therefore puts
// its whole offset in the vector offset and passes a constant zero soffset.
template <int CP = 0, typename T>
__device__ __forceinline__ void chunk_st16(T *p, size_t n2, size_t x, int k, const T *in) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    struct V { T v[16 / sizeof(T)]; };
    constexpr int NV = 16 / (int)sizeof(T);
    V r;
#pragma unroll
    for (int i = 0; i < NV; i++) r.v[i] = in[i];
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, r), buf(p),
                                           (uint32_t)((x + (size_t)(k / NV) * n2) * 16), 0u, CP);
}


template <typename T>
__device__ __forceinline__ void chunk_st(T *p, size_t n2, size_t x, int k, T v) {
    constexpr int NV = 16 / (int)sizeof(T);
    bst(buf(p), (uint32_t)(x * 16 + (k % NV) * sizeof(T)), (uint32_t)((size_t)(k / NV) * n2 * 16), v);
}

// Accesses whose value index differs between the lanes of a wave (the two
// lanes of a site own different link directions): the whole offset goes
// into the per-lane offset, so the access stays one instruction (a
// lane-dependent scalar offset would be split into a loop over its values).
template <typename T>
__device__ __forceinline__ uint32_t chunk_off(size_t n2, size_t x, int k) {
    constexpr int NV = 16 / (int)sizeof(T);
    return (uint32_t)((x + (size_t)(k / NV) * n2) * 16 + (size_t)(k % NV) * sizeof(T));
}
template <int CP = 0, typename T>
__device__ __forceinline__ void chunk_ld16_l(const T *p, size_t n2, size_t x, int k, T *out) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    struct V { T v[16 / sizeof(T)]; };
    const V r = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(buf(p), chunk_off<T>(n2, x, k), 0u, CP));
#pragma unroll
    for (int i = 0; i < (int)(16 / sizeof(T)); i++) out[i] = r.v[i];
}
template <int CP = 0, typename T>
__device__ __forceinline__ void chunk_st16_l(T *p, size_t n2, size_t x, int k, const T *in) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    struct V { T v[16 / sizeof(T)]; };
    V r;
#pragma unroll
    for (int i = 0; i < (int)(16 / sizeof(T)); i++) r.v[i] = in[i];
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, r), buf(p), chunk_off<T>(n2, x, k), 0u, CP);
}
// n values k0.. (k0 and n multiples of 16 / sizeof(T)), lane-dependent k0
template <int n, int CP = 0, typename T>
__device__ __forceinline__ void chunk_load_n_l(const T *p, size_t n2, size_t x, int k0, T *v) {
#pragma unroll
    for (int k = 0; k < n; k += 16 / (int)sizeof(T)) chunk_ld16_l<CP>(p, n2, x, k0 + k, v + k);
}
template <int n, int CP = 0, typename T>
__device__ __forceinline__ void chunk_store_n_l(T *p, size_t n2, size_t x, int k0, const T *v) {
#pragma unroll
    for (int k = 0; k < n; k += 16 / (int)sizeof(T)) chunk_st16_l<CP>(p, n2, x, k0 + k, v + k);
}
// the stored rows of link d + 1 of site x (values 12d .. 12d + 11) from the
// first 12 of the link's 18 values v, d lane-dependent
template <int CP = 0, typename T>
__device__ __forceinline__ void chunk_store_link_l(T *p, size_t n2, size_t x, int d, const T *v) {
    chunk_store_n_l<kLinkVals, CP>(p, n2, x, kLinkVals * d, v);
}

// A link plane set: 18 planes of n2 values, entry (i,j) real at plane 2(3i+j).
template <typename T>
__device__ __forceinline__ M3<T> load_m(const T *__restrict__ base, size_t n2, size_t x) {
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            r.re[i][j] = pl_ld(base, n2, 2 * (3 * i + j), x);
            r.im[i][j] = pl_ld(base, n2, 2 * (3 * i + j) + 1, x);
        }
    return r;
}

template <typename T>
__device__ __forceinline__ void store_m(T *__restrict__ base, size_t n2, size_t x, const M3<T> &m) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            pl_st(base, n2, 2 * (3 * i + j), x, m.re[i][j]);
            pl_st(base, n2, 2 * (3 * i + j) + 1, x, m.im[i][j]);
        }
}

// Links in the field state hold their first two rows, kLinkVals = 12 values
// (entry (i,j) real at 2(3i+j), imaginary next to it, i = 0, 1): for SU(3)
// the third row is the complex conjugate of the cross product of the first
// two (its cofactors), rebuilt where a link is read.  Link d + 1 of a site
// is the values 12d .. 12d + 11 of its record (three chunks in FP32, six in
// FP64).

// row 2 of m from rows 0 and 1: conj(r0 x r1)
template <typename T>
__device__ __forceinline__ void third_row(M3<T> &m) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        const T cr = m.re[0][a] * m.re[1][b] - m.im[0][a] * m.im[1][b] -
                     (m.re[0][b] * m.re[1][a] - m.im[0][b] * m.im[1][a]);
        const T ci = m.re[0][a] * m.im[1][b] + m.im[0][a] * m.re[1][b] -
                     (m.re[0][b] * m.im[1][a] + m.im[0][b] * m.re[1][a]);
        m.re[2][k] = cr;
        m.im[2][k] = -ci;
    }
}

// the link from its two stored rows v[0..11]
template <typename T>
__device__ __forceinline__ M3<T> link_from_rows(const T *v) {
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            r.re[i][j] = v[2 * (3 * i + j)];
            r.im[i][j] = v[2 * (3 * i + j) + 1];
        }
    third_row(r);
    return r;
}

// link d + 1 of site x (d the same for all lanes)
template <typename T>
__device__ __forceinline__ M3<T> chunk_load_link(const T *__restrict__ p, size_t n2, size_t x, int d) {
    T v[kLinkVals];
#pragma unroll
    for (int k = 0; k < kLinkVals; k += 16 / (int)sizeof(T)) chunk_ld16(p, n2, x, kLinkVals * d + k, v + k);
    return link_from_rows(v);
}

// an algebra vector: the 8 values k0..k0+7 (k0 a multiple of 16 / sizeof(T),
// the same for all lanes)
template <typename T>
__device__ __forceinline__ void chunk_load_a(const T *__restrict__ p, size_t n2, size_t x, int k0, T *v) {
#pragma unroll
    for (int a = 0; a < 8; a += 16 / (int)sizeof(T)) chunk_ld16(p, n2, x, k0 + a, v + a);
}

}  // namespace gl
