// mlp.hip -- the learned surrogate: a fully connected network
// (n_in -> width x depth -> n_out, SiLU) with BF16 weights and activations,
// FP32 accumulation on the matrix cores, FP32 master weights and Adam.  It
// maps (Q_s, quark mass, initial p_T, formation time, tau) to the broadening
// observables the solver produces; the solver generates its training data and
// measures its error (paper_2307_07999_amd/surrogate.py).
//
// Dense products use v_mfma_f32_16x16x16_bf16: a 64 x 64 output tile per
// 256-thread workgroup, each wave a 32 x 32 quarter as 2 x 2 MFMA blocks,
// operands staged through LDS in 16-deep K slices.  Operand layout of one
// 16x16x16 MFMA for lane l: A row l%16, k = 4(l/16)..+3; B column l%16,
// k = 4(l/16)..+3; result column l%16, rows 4(l/16)..+3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "../../include/glasma.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16;

__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even
__device__ __forceinline__ bf16 f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}

constexpr int BM = 64, BN = 64, BK = 16;

// C[M x N] = sum_k A(m, k) B(k, n) (+ bias[n]); A(m,k) = TA ? A[k*lda+m] : A[m*lda+k],
// B(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n].  Writes C (FP32) if non-null and
// act(C) as BF16 to H if non-null (act: 0 identity, 1 SiLU).
template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
k_gemm(const bf16 *__restrict__ A, int lda, const bf16 *__restrict__ B, int ldb, int M, int N, int K,
       const float *__restrict__ bias, float *__restrict__ C, int ldc, bf16 *__restrict__ H, int ldh, int act) {
    __shared__ bf16 sA[BM][BK];
    __shared__ bf16 sB[BN][BK];   // transposed: sB[n][k]
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += BK) {
        // A tile 64 x 16
#pragma unroll
        for (int q = 0; q < 4; q++) {
            int r, c;
            if (!TA) { r = t >> 2; c = (t & 3) * 4 + q; }
            else { c = t >> 4; r = (t & 15) * 4 + q; }
            int m = m0 + r, k = k0 + c;
            bf16 v = 0;
            if (m < M && k < K) v = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
            sA[r][c] = v;
        }
        // B tile 16 x 64 stored as sB[n][k]
#pragma unroll
        for (int q = 0; q < 4; q++) {
            int r, c;   // r: k within tile, c: n within tile
            if (!TB) { r = t >> 4; c = (t & 15) * 4 + q; }
            else { c = t >> 2; r = (t & 3) * 4 + q; }
            int k = k0 + r, n = n0 + c;
            bf16 v = 0;
            if (k < K && n < N) v = TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
            sB[c][r] = v;
        }
        __syncthreads();
        const int kk = 4 * (lane >> 4), li = lane & 15;
#pragma unroll
        for (int i = 0; i < 2; i++) {
            bf16x4 a;
#pragma unroll
            for (int j = 0; j < 4; j++) a[j] = (short)sA[wm + 16 * i + li][kk + j];
#pragma unroll
            for (int j2 = 0; j2 < 2; j2++) {
                bf16x4 b;
#pragma unroll
                for (int j = 0; j < 4; j++) b[j] = (short)sB[wn + 16 * j2 + li][kk + j];
                acc[i][j2] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[i][j2], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    const int col = lane & 15, rb = 4 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j2 = 0; j2 < 2; j2++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                int m = m0 + wm + 16 * i + rb + j, n = n0 + wn + 16 * j2 + col;
                if (m < M && n < N) {
                    float v = acc[i][j2][j] + (bias ? bias[n] : 0.f);
                    if (C) C[(size_t)m * ldc + n] = v;
                    if (H) {
                        float h = act == 1 ? v / (1.f + __expf(-v)) : v;
                        H[(size_t)m * ldh + n] = f2bf(h);
                    }
                }
            }
}

// gather a batch by permutation, scale inputs to [-1, 1] (BF16) and standardise
// targets; target c is first divided by X[col]^pw[c] when col >= 0
__global__ void __launch_bounds__(256)
k_prep(const float *__restrict__ X, const float *__restrict__ Y, const int32_t *__restrict__ idx, int64_t off,
       int B, int nin, int nout, const float *__restrict__ sc, int pcol, bf16 *__restrict__ Xb,
       float *__restrict__ Yb) {
    int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= B) return;
    int64_t s = idx ? idx[off + r] : off + r;
    for (int c = 0; c < nin; c++) {
        float lo = sc[c], hi = sc[nin + c];
        Xb[(size_t)r * nin + c] = f2bf(2.f * (X[s * nin + c] - lo) / (hi - lo) - 1.f);
    }
    if (Y)
        for (int c = 0; c < nout; c++) {
            float mu = sc[2 * nin + c], sd = sc[2 * nin + nout + c];
            float y = Y[s * nout + c];
            if (pcol >= 0) y /= powf(X[s * nin + pcol], sc[2 * nin + 2 * nout + c]);
            Yb[(size_t)r * nout + c] = (y - mu) / sd;
        }
}

// dZ = 2 (Z - Y) / (B nout); loss partial per workgroup
__global__ void __launch_bounds__(256)
k_loss(const float *__restrict__ Z, const float *__restrict__ Y, int count, float scale, float *__restrict__ dZ,
       bf16 *__restrict__ dZb, float *__restrict__ loss_acc) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < count; i += 256) {
        float d = Z[i] - Y[i];
        s += d * d;
        float g = 2.f * d * scale;
        dZ[i] = g;
        dZb[i] = f2bf(g);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss_acc += red[0] * scale;
}

// dZ = dH * SiLU'(Z)
__global__ void __launch_bounds__(256)
k_silu_back(const float *__restrict__ dH, const float *__restrict__ Z, int64_t count, float *__restrict__ dZ,
            bf16 *__restrict__ dZb) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    float z = Z[i], sg = 1.f / (1.f + __expf(-z));
    float g = dH[i] * sg * (1.f + z * (1.f - sg));
    dZ[i] = g;
    dZb[i] = f2bf(g);
}

// db[n] = sum_m dZ[m][n], fixed order
__global__ void __launch_bounds__(256)
k_colsum(const float *__restrict__ dZ, int M, int N, float *__restrict__ db) {
    __shared__ float red[256];
    int n = blockIdx.x;
    float s = 0.f;
    for (int m = threadIdx.x; m < M; m += 256) s += dZ[(size_t)m * N + n];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[n] = red[0];
}

__global__ void __launch_bounds__(256)
k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v, int64_t n,
       float lr, float b1, float b2, float c1, float c2, float eps) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void __launch_bounds__(256)
k_to_bf16(const float *__restrict__ w, int64_t n, bf16 *__restrict__ o) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) o[i] = f2bf(w[i]);
}

// outputs back to physical units: undo the standardisation and the input power
__global__ void __launch_bounds__(256)
k_unscale(const float *__restrict__ Z, int B, int nout, const float *__restrict__ sc_out,
          const float *__restrict__ X, int nin, int pcol, float *__restrict__ Y) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= B * nout) return;
    int c = i % nout, r = i / nout;
    float y = Z[i] * sc_out[nout + c] + sc_out[c];
    if (pcol >= 0) y *= powf(X[(size_t)r * nin + pcol], sc_out[2 * nout + c]);
    Y[i] = y;
}

__global__ void k_zero1(float *p) {
    if (threadIdx.x == 0) *p = 0.f;
}

thread_local std::string g_mlp_err;

gl_status mfail(gl_status s, const std::string &m) {
    g_mlp_err = m;
    return s;
}

#define MHIP(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return mfail(GL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline size_t al(size_t v) { return (v + 255) & ~(size_t)255; }
inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

struct gl_mlp {
    gl_mlp_desc d;
    hipStream_t st;
    char *ws;
    int L;                                      // linear layers = depth + 1
    std::vector<int> din, dout;                 // per layer
    std::vector<int64_t> woff, boff;            // offsets in the flat parameter vector
    int64_t n_params, n_w;                      // all parameters, weights only
    // device buffers
    float *P, *G, *Mo, *Vo;                     // master params, grads, Adam moments
    bf16 *Wb;                                   // BF16 weights, per layer at woff
    float *sc;                                  // scaling: in_lo, in_hi, out_mean, out_std
    bf16 *Xb;                                   // [max_batch][n_in]
    float *Yb;                                  // [max_batch][n_out]
    std::vector<float *> Z;                     // pre-activations per layer [max_batch][dout]
    std::vector<bf16 *> Hb;                     // BF16 activations per layer
    float *dZ, *dH;                             // FP32 scratch [max_batch][width_max]
    bf16 *dZb;
    float *loss;                                // 1 float
    int32_t *perm;                              // [max_samples]
    int64_t max_samples;
    int64_t adam_t = 0;
    int pcol = -1;                              // input column of the output power, -1: none
    // trust region of gl_surrogate_query: the training box, and the held-out
    // error per (class of the discrete column) x (bin of the binned column)
    bool trust = false;
    std::vector<float> t_lo, t_hi, t_classes, t_edges, t_err;
    int t_class_col = -1, t_bin_col = -1;
    float t_class_tol = 0.f, t_err_max = 0.f;
};

namespace {

struct MlpSizes {
    size_t total;
};

gl_status mlp_layout(const gl_mlp_desc *d, int64_t max_samples, gl_mlp *m, size_t *total) {
    if (!d || d->n_in < 1 || d->n_out < 1 || d->width < 1 || d->depth < 1 || d->max_batch < 1)
        return mfail(GL_EINVAL, "bad MLP description");
    if (max_samples < 0) return mfail(GL_EINVAL, "max_samples must be >= 0");
    int L = d->depth + 1;
    std::vector<int> din(L), dout(L);
    for (int l = 0; l < L; l++) {
        din[l] = l == 0 ? d->n_in : d->width;
        dout[l] = l == L - 1 ? d->n_out : d->width;
    }
    int64_t np = 0, nw = 0;
    std::vector<int64_t> woff(L), boff(L);
    for (int l = 0; l < L; l++) {
        woff[l] = np;
        np += (int64_t)din[l] * dout[l];
        nw += (int64_t)din[l] * dout[l];
    }
    for (int l = 0; l < L; l++) {
        boff[l] = np;
        np += dout[l];
    }
    const int64_t B = d->max_batch;
    const int wmax = std::max(d->width, std::max(d->n_in, d->n_out));
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off = al(off + b);
        return o;
    };
    size_t oP = take(np * 4), oG = take(np * 4), oM = take(np * 4), oV = take(np * 4), oW = take(nw * 2);
    size_t osc = take((2 * d->n_in + 3 * d->n_out) * 4), oX = take(B * d->n_in * 2), oY = take(B * d->n_out * 4);
    std::vector<size_t> oZ(L), oH(L);
    for (int l = 0; l < L; l++) {
        oZ[l] = take(B * dout[l] * 4);
        oH[l] = take(B * dout[l] * 2);
    }
    size_t odZ = take(B * wmax * 4), odH = take(B * wmax * 4), odZb = take(B * wmax * 2), oloss = take(4);
    size_t operm = take(std::max<int64_t>(1, max_samples) * 4);
    *total = off;
    if (m) {
        char *w = m->ws;
        m->d = *d;
        m->L = L;
        m->din = din;
        m->dout = dout;
        m->woff = woff;
        m->boff = boff;
        m->n_params = np;
        m->n_w = nw;
        m->P = (float *)(w + oP);
        m->G = (float *)(w + oG);
        m->Mo = (float *)(w + oM);
        m->Vo = (float *)(w + oV);
        m->Wb = (bf16 *)(w + oW);
        m->sc = (float *)(w + osc);
        m->Xb = (bf16 *)(w + oX);
        m->Yb = (float *)(w + oY);
        m->Z.resize(L);
        m->Hb.resize(L);
        for (int l = 0; l < L; l++) {
            m->Z[l] = (float *)(w + oZ[l]);
            m->Hb[l] = (bf16 *)(w + oH[l]);
        }
        m->dZ = (float *)(w + odZ);
        m->dH = (float *)(w + odH);
        m->dZb = (bf16 *)(w + odZb);
        m->loss = (float *)(w + oloss);
        m->perm = (int32_t *)(w + operm);
        m->max_samples = max_samples;
    }
    return GL_OK;
}

template <bool TA, bool TB>
hipError_t gemm(hipStream_t st, const bf16 *A, int lda, const bf16 *B, int ldb, int M, int N, int K, const float *bias,
                float *C, int ldc, bf16 *H, int ldh, int act) {
    dim3 grid(nb(N, BN), nb(M, BM));
    hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, bias, C, ldc, H, ldh, act);
    return hipGetLastError();
}

// forward on the staged batch Xb of B rows
gl_status forward(gl_mlp *m, int B) {
    const bf16 *in = m->Xb;
    for (int l = 0; l < m->L; l++) {
        bool last = l == m->L - 1;
        MHIP((gemm<false, true>(m->st, in, m->din[l], m->Wb + m->woff[l], m->din[l], B, m->dout[l], m->din[l],
                                m->P + m->boff[l], m->Z[l], m->dout[l], last ? nullptr : m->Hb[l], m->dout[l], 1)));
        in = m->Hb[l];
    }
    return GL_OK;
}

// backward from the loss on the staged targets; gradients into G
gl_status backward(gl_mlp *m, int B) {
    const int L = m->L;
    const int no = m->d.n_out;
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, m->st, m->Z[L - 1], m->Yb, B * no, 1.f / (float)(B * no),
                       m->dZ, m->dZb, m->loss);
    MHIP(hipGetLastError());
    for (int l = L - 1; l >= 0; l--) {
        const int di = m->din[l], dd = m->dout[l];
        const bf16 *Hprev = l == 0 ? m->Xb : m->Hb[l - 1];
        // dW[o][i] = sum_b dZ[b][o] Hprev[b][i]
        MHIP((gemm<true, false>(m->st, m->dZb, dd, Hprev, di, dd, di, B, nullptr, m->G + m->woff[l], di, nullptr, 0,
                                0)));
        hipLaunchKernelGGL(k_colsum, dim3(dd), dim3(256), 0, m->st, m->dZ, B, dd, m->G + m->boff[l]);
        MHIP(hipGetLastError());
        if (l > 0) {
            // dH[b][i] = sum_o dZ[b][o] W[o][i]
            MHIP((gemm<false, false>(m->st, m->dZb, dd, m->Wb + m->woff[l], di, B, di, dd, nullptr, m->dH, di,
                                     nullptr, 0, 0)));
            hipLaunchKernelGGL(k_silu_back, dim3(nb((int64_t)B * di, 256)), dim3(256), 0, m->st, m->dH, m->Z[l - 1],
                               (int64_t)B * di, m->dZ, m->dZb);
            MHIP(hipGetLastError());
        }
    }
    return GL_OK;
}

gl_status sync_weights(gl_mlp *m) {
    hipLaunchKernelGGL(k_to_bf16, dim3(nb(m->n_w, 256)), dim3(256), 0, m->st, m->P, m->n_w, m->Wb);
    MHIP(hipGetLastError());
    return GL_OK;
}

}  // namespace

extern "C" {

const char *gl_mlp_last_error(void) { return g_mlp_err.c_str(); }

gl_status gl_mlp_required_bytes(const gl_mlp_desc *d, int64_t max_samples, size_t *bytes) {
    if (!bytes) return mfail(GL_EINVAL, "null output");
    return mlp_layout(d, max_samples, nullptr, bytes);
}

gl_status gl_mlp_create(const gl_mlp_desc *d, int64_t max_samples, void *ws, size_t bytes, void *stream, uint64_t seed,
                        gl_mlp **out) {
    if (!out) return mfail(GL_EINVAL, "null output");
    *out = nullptr;
    size_t need = 0;
    gl_status s = mlp_layout(d, max_samples, nullptr, &need);
    if (s) return s;
    if (!ws || ((uintptr_t)ws & 255)) return mfail(GL_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < need) return mfail(GL_ENOMEM, "workspace smaller than gl_mlp_required_bytes()");
    gl_mlp *m = new (std::nothrow) gl_mlp();
    if (!m) return mfail(GL_ENOMEM, "host allocation failed");
    m->ws = (char *)ws;
    m->st = (hipStream_t)stream;
    mlp_layout(d, max_samples, m, &need);
    // He-uniform weights, zero biases (host draw from a seeded Mersenne twister)
    std::vector<float> p(m->n_params, 0.f);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < m->L; l++) {
        float bound = std::sqrt(6.f / (float)m->din[l]) * (l == m->L - 1 ? 0.1f : 1.f);
        std::uniform_real_distribution<float> u(-bound, bound);
        for (int64_t k = 0; k < (int64_t)m->din[l] * m->dout[l]; k++) p[m->woff[l] + k] = u(rng);
    }
    std::vector<float> sc(2 * d->n_in + 3 * d->n_out, 0.f);
    for (int c = 0; c < d->n_in; c++) {
        sc[c] = -1.f;
        sc[d->n_in + c] = 1.f;
    }
    for (int c = 0; c < d->n_out; c++) {
        sc[2 * d->n_in + c] = 0.f;
        sc[2 * d->n_in + d->n_out + c] = 1.f;
    }
    auto bad = [&](const char *w) {
        delete m;
        return mfail(GL_EDEVICE, w);
    };
    if (hipMemcpyAsync(m->P, p.data(), p.size() * 4, hipMemcpyHostToDevice, m->st) != hipSuccess ||
        hipMemcpyAsync(m->sc, sc.data(), sc.size() * 4, hipMemcpyHostToDevice, m->st) != hipSuccess ||
        hipMemsetAsync(m->Mo, 0, m->n_params * 4, m->st) != hipSuccess ||
        hipMemsetAsync(m->Vo, 0, m->n_params * 4, m->st) != hipSuccess)
        return bad("upload failed");
    if (sync_weights(m) || hipStreamSynchronize(m->st) != hipSuccess) return bad("init failed");
    *out = m;
    return GL_OK;
}

void gl_mlp_destroy(gl_mlp *m) { delete m; }

gl_status gl_mlp_set_scaling(gl_mlp *m, const float *in_lo, const float *in_hi, const float *out_mean,
                             const float *out_std) {
    if (!m || !in_lo || !in_hi || !out_mean || !out_std) return mfail(GL_EINVAL, "null argument");
    const int ni = m->d.n_in, no = m->d.n_out;
    std::vector<float> sc(2 * ni + 2 * no);
    for (int c = 0; c < ni; c++) {
        if (!(in_hi[c] > in_lo[c])) return mfail(GL_EINVAL, "in_hi must exceed in_lo");
        sc[c] = in_lo[c];
        sc[ni + c] = in_hi[c];
    }
    for (int c = 0; c < no; c++) {
        if (!(out_std[c] > 0)) return mfail(GL_EINVAL, "out_std must be > 0");
        sc[2 * ni + c] = out_mean[c];
        sc[2 * ni + no + c] = out_std[c];
    }
    MHIP(hipMemcpyAsync(m->sc, sc.data(), sc.size() * 4, hipMemcpyHostToDevice, m->st));
    MHIP(hipStreamSynchronize(m->st));
    return GL_OK;
}

gl_status gl_mlp_set_output_power(gl_mlp *m, int32_t col, const float *powers) {
    if (!m) return mfail(GL_EINVAL, "null argument");
    if (col >= m->d.n_in || (col >= 0 && !powers)) return mfail(GL_EINVAL, "bad column or powers");
    m->pcol = col < 0 ? -1 : col;
    if (col >= 0) {
        MHIP(hipMemcpyAsync(m->sc + 2 * m->d.n_in + 2 * m->d.n_out, powers, m->d.n_out * 4, hipMemcpyHostToDevice,
                            m->st));
        MHIP(hipStreamSynchronize(m->st));
    }
    return GL_OK;
}

gl_status gl_mlp_train(gl_mlp *m, const float *X, const float *Y, int64_t n, int32_t epochs, int32_t batch, float lr,
                       uint64_t seed, float *loss_per_epoch) {
    if (!m || !X || !Y) return mfail(GL_EINVAL, "null argument");
    if (n < 1 || n > m->max_samples || batch < 1 || batch > m->d.max_batch || epochs < 0)
        return mfail(GL_EINVAL, "bad sizes (n <= max_samples, batch <= max_batch)");
    std::mt19937_64 rng(seed);
    std::vector<int32_t> perm(n);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const int64_t nbat = n / batch;   // whole batches only
    if (nbat < 1) return mfail(GL_EINVAL, "fewer samples than one batch");
    for (int ep = 0; ep < epochs; ep++) {
        for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
        for (int64_t i = n - 1; i > 0; i--) std::swap(perm[i], perm[(int64_t)(rng() % (uint64_t)(i + 1))]);
        MHIP(hipMemcpyAsync(m->perm, perm.data(), n * 4, hipMemcpyHostToDevice, m->st));
        hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, m->st, m->loss);
        for (int64_t bi = 0; bi < nbat; bi++) {
            hipLaunchKernelGGL(k_prep, dim3(nb(batch, 256)), dim3(256), 0, m->st, X, Y, m->perm, bi * batch, batch,
                               m->d.n_in, m->d.n_out, m->sc, m->pcol, m->Xb, m->Yb);
            MHIP(hipGetLastError());
            gl_status s = forward(m, batch);
            if (s) return s;
            s = backward(m, batch);
            if (s) return s;
            m->adam_t++;
            float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
            hipLaunchKernelGGL(k_adam, dim3(nb(m->n_params, 256)), dim3(256), 0, m->st, m->P, m->G, m->Mo, m->Vo,
                               m->n_params, lr, b1, b2, c1, c2, eps);
            MHIP(hipGetLastError());
            s = sync_weights(m);
            if (s) return s;
        }
        if (loss_per_epoch) {
            float l = 0;
            MHIP(hipMemcpyAsync(&l, m->loss, 4, hipMemcpyDeviceToHost, m->st));
            MHIP(hipStreamSynchronize(m->st));
            loss_per_epoch[ep] = l / (float)nbat;
        }
    }
    MHIP(hipStreamSynchronize(m->st));
    return GL_OK;
}

gl_status gl_mlp_infer(gl_mlp *m, const float *X, float *Y, int64_t n) {
    if (!m || !X || !Y) return mfail(GL_EINVAL, "null argument");
    if (n < 0) return mfail(GL_EINVAL, "n must be >= 0");
    const int B = m->d.max_batch;
    for (int64_t off = 0; off < n; off += B) {
        int b = (int)std::min<int64_t>(B, n - off);
        hipLaunchKernelGGL(k_prep, dim3(nb(b, 256)), dim3(256), 0, m->st, X, (const float *)nullptr,
                           (const int32_t *)nullptr, off, b, m->d.n_in, m->d.n_out, m->sc, m->pcol, m->Xb,
                           (float *)nullptr);
        MHIP(hipGetLastError());
        gl_status s = forward(m, b);
        if (s) return s;
        hipLaunchKernelGGL(k_unscale, dim3(nb((int64_t)b * m->d.n_out, 256)), dim3(256), 0, m->st, m->Z[m->L - 1], b,
                           m->d.n_out, m->sc + 2 * m->d.n_in, X + off * m->d.n_in, m->d.n_in, m->pcol,
                           Y + off * m->d.n_out);
        MHIP(hipGetLastError());
    }
    return GL_OK;
}

}  // extern "C"

// ---- inference without allocation ---------------------------------------------
// gl_mlp_infer_noalloc stages its rows in a fixed device array of this file
// instead of the model's workspace: the scaled inputs (BF16), two BF16
// activation buffers used in turn by the hidden layers, and the last layer's
// FP32 output, for as many rows per pass as fit.  Each device holds its own
// copy of the array until the process ends; calls on one device share it.
constexpr size_t kInferScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char infer_scratch[kInferScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kScratchDevices] = {};   // device address of infer_scratch, per device

// the address of this device's copy of the array, looked up once per device
// with that device current (the symbol's name is a host-side stand-in)
gl_status infer_scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kScratchDevices) return mfail(GL_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(infer_scratch));
        if (e != hipSuccess || !p)
            return mfail(GL_EDEVICE, std::string("hipGetSymbolAddress(infer_scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return GL_OK;
}

// rows per pass that fit the array: inputs n_in BF16, two activation
// buffers of width BF16, outputs n_out FP32 per row, each buffer 256-aligned
int64_t infer_rows_per_pass(const gl_mlp *m) {
    const int64_t per_row = 2 * (int64_t)m->d.n_in + 2 * 2 * (int64_t)m->d.width + 4 * (int64_t)m->d.n_out;
    const int64_t rows = ((int64_t)kInferScratchBytes - 4 * 256) / per_row;
    return rows / 64 * 64;
}

}  // namespace

extern "C" {

gl_status gl_mlp_infer_noalloc(gl_mlp *m, const float *X, float *Y, int64_t n) {
    if (!m || !X || !Y) return mfail(GL_EINVAL, "null argument");
    if (n < 0) return mfail(GL_EINVAL, "n must be >= 0");
    const int64_t R = infer_rows_per_pass(m);
    if (R < 64)
        return mfail(GL_EINVAL, "network too wide for the inference scratch of " +
                                    std::to_string(kInferScratchBytes) + " bytes: 64 rows of inputs, two activation "
                                    "buffers and outputs must fit (width <= " +
                                    std::to_string(((int64_t)kInferScratchBytes - 1024) / 64 / 4 - 2) + " or so)");
    if (n == 0) return GL_OK;
    // the device of the model's stream must be current: the scratch address
    // is taken per device
    int dev = -1;
    MHIP(hipGetDevice(&dev));
    hipDevice_t sdev = dev;
    if (m->st) MHIP(hipStreamGetDevice(m->st, &sdev));
    if (sdev != dev) return mfail(GL_EINVAL, "the device of the model's stream is not the current device");
    void *base = nullptr;
    if (gl_status s = infer_scratch_address(dev, &base)) return s;
    char *sp = (char *)base;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        char *p = sp + off;
        off = al(off + bytes);
        return p;
    };
    bf16 *Xb = (bf16 *)carve((size_t)R * m->d.n_in * 2);
    bf16 *Hs[2] = {(bf16 *)carve((size_t)R * m->d.width * 2), (bf16 *)carve((size_t)R * m->d.width * 2)};
    float *Z = (float *)carve((size_t)R * m->d.n_out * 4);
    if (off > kInferScratchBytes) return mfail(GL_EINVAL, "inference scratch layout exceeds the array");
    for (int64_t r0 = 0; r0 < n; r0 += R) {
        const int b = (int)std::min<int64_t>(R, n - r0);
        hipLaunchKernelGGL(k_prep, dim3(nb(b, 256)), dim3(256), 0, m->st, X, (const float *)nullptr,
                           (const int32_t *)nullptr, r0, b, m->d.n_in, m->d.n_out, m->sc, m->pcol, Xb,
                           (float *)nullptr);
        MHIP(hipGetLastError());
        const bf16 *in = Xb;
        for (int l = 0; l < m->L; l++) {
            const bool last = l == m->L - 1;
            MHIP((gemm<false, true>(m->st, in, m->din[l], m->Wb + m->woff[l], m->din[l], b, m->dout[l], m->din[l],
                                    m->P + m->boff[l], last ? Z : nullptr, m->dout[l], last ? nullptr : Hs[l & 1],
                                    m->dout[l], 1)));
            in = Hs[l & 1];
        }
        hipLaunchKernelGGL(k_unscale, dim3(nb((int64_t)b * m->d.n_out, 256)), dim3(256), 0, m->st, Z, b, m->d.n_out,
                           m->sc + 2 * m->d.n_in, X + r0 * m->d.n_in, m->d.n_in, m->pcol, Y + r0 * m->d.n_out);
        MHIP(hipGetLastError());
    }
    return GL_OK;
}

gl_status gl_mlp_set_trust(gl_mlp *m, const float *lo, const float *hi, int32_t class_col, int32_t n_classes,
                           const float *classes, float class_tol, int32_t bin_col, int32_t n_bins,
                           const float *bin_edges, const float *err, float err_max) {
    if (!m || !lo || !hi) return mfail(GL_EINVAL, "null argument");
    const int ni = m->d.n_in;
    if (class_col < 0 || class_col >= ni || bin_col < 0 || bin_col >= ni || n_classes < 1 || n_bins < 1 || !classes ||
        !bin_edges || !err || !(class_tol >= 0) || !(err_max >= 0))
        return mfail(GL_EINVAL, "bad trust table (columns, counts, tolerances)");
    for (int c = 0; c < ni; c++)
        if (!(hi[c] >= lo[c])) return mfail(GL_EINVAL, "box hi must be >= lo");
    for (int b = 0; b < n_bins; b++)
        if (!(bin_edges[b + 1] > bin_edges[b])) return mfail(GL_EINVAL, "bin edges must increase");
    m->t_lo.assign(lo, lo + ni);
    m->t_hi.assign(hi, hi + ni);
    m->t_classes.assign(classes, classes + n_classes);
    m->t_edges.assign(bin_edges, bin_edges + n_bins + 1);
    m->t_err.assign(err, err + (size_t)n_classes * n_bins);
    m->t_class_col = class_col;
    m->t_bin_col = bin_col;
    m->t_class_tol = class_tol;
    m->t_err_max = err_max;
    m->trust = true;
    return GL_OK;
}

gl_status gl_surrogate_query(gl_mlp *m, const float *X, int64_t n, float *Y, int32_t *verdict) {
    if (!m || !X || !verdict || (n > 0 && !Y)) return mfail(GL_EINVAL, "null argument");
    if (n < 0) return mfail(GL_EINVAL, "n must be >= 0");
    if (!m->trust) return mfail(GL_ESTATE, "no trust table: call gl_mlp_set_trust after training");
    const int ni = m->d.n_in, no = m->d.n_out;
    // the decision, row by row on the host: inside the box, of a known
    // class, in a cell whose calibrated held-out error is small enough
    *verdict = GL_SURROGATE_NETWORK;
    for (int64_t r = 0; r < n && *verdict == GL_SURROGATE_NETWORK; r++) {
        const float *x = X + r * ni;
        for (int c = 0; c < ni; c++)
            if (!(x[c] >= m->t_lo[c] && x[c] <= m->t_hi[c])) *verdict = GL_SURROGATE_OUTSIDE_DOMAIN;
        if (*verdict != GL_SURROGATE_NETWORK) break;
        int cls = -1;
        for (size_t k = 0; k < m->t_classes.size(); k++)
            if (std::fabs(x[m->t_class_col] - m->t_classes[k]) <= m->t_class_tol) cls = (int)k;
        if (cls < 0) {
            *verdict = GL_SURROGATE_OUTSIDE_DOMAIN;
            break;
        }
        const int nb = (int)m->t_edges.size() - 1;
        const float v = x[m->t_bin_col];
        int bin = -1;
        for (int b = 0; b < nb; b++)
            if (v >= m->t_edges[b] && (v < m->t_edges[b + 1] || (b == nb - 1 && v <= m->t_edges[b + 1]))) bin = b;
        if (bin < 0) {
            *verdict = GL_SURROGATE_OUTSIDE_DOMAIN;
            break;
        }
        const float e = m->t_err[(size_t)cls * nb + bin];
        if (!(e <= m->t_err_max)) *verdict = GL_SURROGATE_UNTRUSTED;
    }
    if (*verdict != GL_SURROGATE_NETWORK || n == 0) return GL_OK;
    // inference: the rows staged in the model's FP32 scratch (dZ holds
    // max_batch x max(width, n_in, n_out) floats), outputs in dH
    const int64_t wmax = std::max(m->d.width, std::max(m->d.n_in, m->d.n_out));
    const int64_t per = std::max<int64_t>(1, std::min<int64_t>(m->d.max_batch, (int64_t)m->d.max_batch * wmax / ni));
    const int64_t rows = std::min<int64_t>(per, (int64_t)m->d.max_batch * wmax / no);
    for (int64_t r0 = 0; r0 < n; r0 += rows) {
        const int64_t b = std::min<int64_t>(rows, n - r0);
        MHIP(hipMemcpyAsync(m->dZ, X + r0 * ni, (size_t)b * ni * 4, hipMemcpyHostToDevice, m->st));
        gl_status s = gl_mlp_infer(m, m->dZ, m->dH, b);
        if (s) return s;
        MHIP(hipMemcpyAsync(Y + r0 * no, m->dH, (size_t)b * no * 4, hipMemcpyDeviceToHost, m->st));
    }
    MHIP(hipStreamSynchronize(m->st));
    return GL_OK;
}

gl_status gl_mlp_grads(gl_mlp *m, const float *X, const float *Y, int32_t n, float *grads, float *loss) {
    if (!m || !X || !Y || !grads) return mfail(GL_EINVAL, "null argument");
    if (n < 1 || n > m->d.max_batch) return mfail(GL_EINVAL, "n must be in [1, max_batch]");
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, m->st, m->loss);
    hipLaunchKernelGGL(k_prep, dim3(nb(n, 256)), dim3(256), 0, m->st, X, Y, (const int32_t *)nullptr, (int64_t)0, n,
                       m->d.n_in, m->d.n_out, m->sc, m->pcol, m->Xb, m->Yb);
    MHIP(hipGetLastError());
    gl_status s = forward(m, n);
    if (s) return s;
    s = backward(m, n);
    if (s) return s;
    MHIP(hipMemcpyAsync(grads, m->G, m->n_params * 4, hipMemcpyDeviceToHost, m->st));
    if (loss) MHIP(hipMemcpyAsync(loss, m->loss, 4, hipMemcpyDeviceToHost, m->st));
    MHIP(hipStreamSynchronize(m->st));
    return GL_OK;
}

gl_status gl_mlp_params(gl_mlp *m, float *get, const float *set, int64_t *n_params) {
    if (!m) return mfail(GL_EINVAL, "null argument");
    if (n_params) *n_params = m->n_params;
    if (set) {
        MHIP(hipMemcpyAsync(m->P, set, m->n_params * 4, hipMemcpyHostToDevice, m->st));
        gl_status s = sync_weights(m);
        if (s) return s;
    }
    if (get) MHIP(hipMemcpyAsync(get, m->P, m->n_params * 4, hipMemcpyDeviceToHost, m->st));
    MHIP(hipStreamSynchronize(m->st));
    return GL_OK;
}

}  // extern "C"
