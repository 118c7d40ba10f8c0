// push_dev.hpp -- per-particle device function of the push of Wong's
// equations and the per-species workgroup reduction, shared by the
// single-event and the batched kernels.  The scheme is described in
// particles.hip.
#pragma once
#include "internal.hpp"
#include "su3.hpp"

namespace gl {

// One particle step: the particle in slot i of P is written to slot j of W
// (the same slot of the same arrays, or its sorted position in the other
// buffer; with MOVE, also a particle that is not pushed).  Returns the
// species of an active particle (-1 otherwise) and in acc its squared
// momenta p_x^2, p_y^2, p_z^2 (lab frame) at tau_{n+1/2} and a count of 1;
// the series reduction subtracts the species' sums of the squared momenta at
// formation.  A wave makes up to six dependent trips to memory: the particle
// state (all of it, before the activity test), the site fields and phi of its
// cell in three groups, and the link of each crossing; each trip holds few
// registers, which buys the occupancy that hides the latency of the others.
template <typename T, bool MOVE = false, bool ST = kStreamed<T>>
__device__ __forceinline__ int push_particle(int N, const PartPtrs<T> &P, int64_t i, const PartPtrs<T> &W, int64_t j,
                                             const FieldPtrs<T> &f, const T *__restrict__ F,
                                             const SpeciesTab<T> &tab, int n, T dtau, double *acc) {
    const size_t n2 = plane_pitch(N);
    acc[0] = acc[1] = acc[2] = acc[3] = 0.0;
    constexpr int CP = stream_policy(ST);   // the particle arrays are streamed (ST)
    const int s = el_ld_i32<CP>(P.species, i);
    int cx = el_ld_i32<CP>(P.cx, i), cy = el_ld_i32<CP>(P.cy, i);
    // the state record in 16-byte loads
    T r[kPartRec<T>];
#pragma unroll
    for (int k = 0; k < kPartRec<T>; k += 16 / (int)sizeof(T)) chunk_ld16<CP>(P.st, (size_t)P.cap, (size_t)i, k, r + k);
    T q[8];
#pragma unroll
    for (int a = 0; a < 8; a++) q[a] = r[kQ + a];
    T pl[3] = {r[kPx], r[kPy], r[kPeta]};
    T ox = r[kOx], oy = r[kOy];
    const T eta_old = r[kEta];
    const bool active = s >= 0 && n >= tab.nform[s];
    if (active) {
        const T tau = dtau * (T)n, th = dtau * ((T)n + T(0.5));
        const T m = tab.mass[s];
        const size_t x = (size_t)cx + (size_t)N * cy;
        // the cell's site-field record, in 16-byte loads: the six fields,
        // and the second half of E_x or E_y where it is stored apart (zero
        // elsewhere).  Where the working set overflows the last-level cache
        // (ST: single FP64 events, batches) those halves are loaded only
        // where they are stored, which spares a fifth of the gathered lines;
        // a single FP32 event, whose site fields stay cached, loads them
        // everywhere and selects, without the divergent branch (push 43.3
        // against 41.9 us).  The record is contracted with Q in three groups
        // (E_x, E_y, then E_z, B and phi), each loaded just before its sums,
        // so that at most a third of it is live: the FP32 push then fits 79
        // VGPRs, six waves per SIMD (FP32 push 42.8 -> 41.4 us, FP64 73.2 ->
        // 71.3 us, FP32 64-event batch 0.937 -> 0.921 s)
        constexpr int NV = 16 / (int)sizeof(T);
        T e[3], b[3], ph[8];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            // E_x or E_y and its second half where it is stored apart
            T re[8], rh[8];
#pragma unroll
            for (int j = 0; j < 8; j += NV) chunk_ld16(F, n2, x, 8 * k + j, re + j);
            const bool stored = half_stored(k, cx, cy);
            if constexpr (ST) {
                if (stored) {
#pragma unroll
                    for (int j = 0; j < 8; j += NV) chunk_ld16(F, n2, x, 48 + 8 * k + j, rh + j);
                } else {
#pragma unroll
                    for (int j = 0; j < 8; j++) rh[j] = T(0);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 8; j += NV) chunk_ld16(F, n2, x, 48 + 8 * k + j, rh + j);
#pragma unroll
                for (int j = 0; j < 8; j++) rh[j] = stored ? rh[j] : T(0);
            }
            T se = T(0);
#pragma unroll
            for (int a = 0; a < 8; a++) se = fma(q[a], re[a] + rh[a], se);
            e[k] = se;
            __builtin_amdgcn_sched_barrier(0);
        }
        {
            // E_z (slots 16..23), B_x, B_y, B_z (24..47) and phi
            T rb[32];
#pragma unroll
            for (int j = 0; j < 32; j += NV) chunk_ld16(F, n2, x, 16 + j, rb + j);
            chunk_load_a(f.phi, n2, x, 0, ph);
            T se = T(0);
#pragma unroll
            for (int a = 0; a < 8; a++) se = fma(q[a], rb[a], se);
            e[2] = se;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                T sb = T(0);
#pragma unroll
                for (int a = 0; a < 8; a++) sb = fma(q[a], rb[8 + 8 * k + a], sb);
                b[k] = sb;
            }
        }
        // Boris kick at tau_n
        pl[2] /= tau;
        T pm[3];
#pragma unroll
        for (int k = 0; k < 3; k++) pm[k] = pl[k] + T(0.5) * dtau * e[k];
        T g = sqrt(m * m + pm[0] * pm[0] + pm[1] * pm[1] + pm[2] * pm[2]);
        T h = dtau / (T(2) * g);
        T t[3] = {b[0] * h, b[1] * h, b[2] * h};
        T t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
        T sf = T(2) / (T(1) + t2);
        T sv[3] = {sf * t[0], sf * t[1], sf * t[2]};
        T pp[3] = {pm[0] + (pm[1] * t[2] - pm[2] * t[1]), pm[1] + (pm[2] * t[0] - pm[0] * t[2]),
                   pm[2] + (pm[0] * t[1] - pm[1] * t[0])};
        T pq[3] = {pm[0] + (pp[1] * sv[2] - pp[2] * sv[1]), pm[1] + (pp[2] * sv[0] - pp[0] * sv[2]),
                   pm[2] + (pp[0] * sv[1] - pp[1] * sv[0])};
#pragma unroll
        for (int k = 0; k < 3; k++) pl[k] = pq[k] + T(0.5) * dtau * e[k];
        const T peta = tau * pl[2];
        // drift
        const T pzh = peta / th;
        const T ptau = sqrt(m * m + pl[0] * pl[0] + pl[1] * pl[1] + pzh * pzh);
        ox += dtau * pl[0] / ptau;
        oy += dtau * pl[1] / ptau;
        const T deta = dtau * peta / (th * th * ptau);
        const T eta_new = eta_old + deta;
        // cells crossed, x first then y
        const int sx = ox >= T(0.5) ? 1 : (ox < T(-0.5) ? -1 : 0);
        const int sy = oy >= T(0.5) ? 1 : (oy < T(-0.5) ? -1 : 0);
        const int cxm = cx == 0 ? N - 1 : cx - 1, cym = cy == 0 ? N - 1 : cy - 1;
        const int cx1 = sx > 0 ? (cx + 1 == N ? 0 : cx + 1) : (sx < 0 ? cxm : cx);
        const int cy1 = sy > 0 ? (cy + 1 == N ? 0 : cy + 1) : (sy < 0 ? cym : cy);
        // colour rotation along eta with phi^n at the old cell: Q <- W Q W^dag
        transport_nd(expi_alg(ph, -deta), q, q);
        // crossings: Q <- U^dag Q U forward, U Q U^dag backward.  Each link is
        // loaded when its transport is due (the scheduling barriers keep the
        // compiler from hoisting the loads): holding both links through the
        // exponential took the FP64 push to 214 VGPRs and two waves per SIMD;
        // loaded one after the other it fits 168 VGPRs and three waves, and
        // the extra trip to memory costs less than the lost occupancy (FP64
        // push 83.1 -> 74.0 us at 512^2 with 7e5 particles)
        __builtin_amdgcn_sched_barrier(0);
        if (sx != 0) {
            const M3<T> ux = chunk_load_link(f.U, n2, (size_t)(sx > 0 ? cx : cxm) + (size_t)N * cy, 0);
            if (sx > 0) transport_dn(ux, q, q);
            else transport_nd(ux, q, q);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (sy != 0) {
            const M3<T> uy = chunk_load_link(f.U, n2, (size_t)cx1 + (size_t)N * (sy > 0 ? cy : cym), 1);
            if (sy > 0) transport_dn(uy, q, q);
            else transport_nd(uy, q, q);
        }
        ox -= (T)sx;
        oy -= (T)sy;
        el_st_i32<CP>(W.cx, j, cx1);
        el_st_i32<CP>(W.cy, j, cy1);
        r[kOx] = ox;
        r[kOy] = oy;
        r[kEta] = eta_new;
        r[kPx] = pl[0];
        r[kPy] = pl[1];
        r[kPeta] = peta;
#pragma unroll
        for (int a = 0; a < 8; a++) r[kQ + a] = q[a];
#pragma unroll
        for (int k = 0; k < kPartRec<T>; k += 16 / (int)sizeof(T)) chunk_st16<CP>(W.st, (size_t)W.cap, (size_t)j, k, r + k);
        // broadening at tau_{n+1/2}, accumulated in FP64
        const double etab = 0.5 * ((double)eta_old + (double)eta_new);
        // sinh and cosh from one expm1 (exact-to-rounding for small rapidities)
        const double em = expm1(etab), ie = 1.0 / (em + 1.0);
        const double sh = 0.5 * em * (em + 2.0) * ie, ch = 1.0 + 0.5 * em * em * ie;
        const double pzlab = (double)ptau * sh + (double)pzh * ch;
        acc[0] = (double)pl[0] * pl[0];
        acc[1] = (double)pl[1] * pl[1];
        acc[2] = pzlab * pzlab;
        acc[3] = 1.0;
    } else if (MOVE) {
        el_st_i32<CP>(W.cx, j, cx);
        el_st_i32<CP>(W.cy, j, cy);
#pragma unroll
        for (int k = 0; k < kPartRec<T>; k += 16 / (int)sizeof(T)) chunk_st16<CP>(W.st, (size_t)W.cap, (size_t)j, k, r + k);
    }
    return active ? s : -1;
}

// Per-species workgroup reduction of kPushBlock threads (particles of
// several species share a workgroup once they are sorted by cell).  Every
// thread writes its species and four terms to LDS; then work item (g, c)
// sums term c % 4 of species c / 4 over the 32 particles of segment g in
// particle order, and thread c adds the segments in order -- a fixed order,
// so the partial sums are deterministic.  Writes out[sp * 4 + k].
__device__ __forceinline__ void block_species_reduce(int s, const double *acc, int n_species,
                                                     double *__restrict__ out) {
    constexpr int kSeg = 8, kLen = kPushBlock / kSeg;
    __shared__ double val[4][kPushBlock];
    __shared__ int spc[kPushBlock];
    __shared__ double part[kSeg][kMaxSpecies * 4];
    const int t = threadIdx.x;
    spc[t] = s;
#pragma unroll
    for (int k = 0; k < 4; k++) val[k][t] = acc[k];
    __syncthreads();
    const int ncol = n_species * 4;
    for (int w = t; w < kSeg * ncol; w += kPushBlock) {
        const int g = w / ncol, c = w % ncol, sp = c >> 2, k = c & 3;
        double sum = 0.0;
#pragma unroll 8
        for (int i = g * kLen; i < (g + 1) * kLen; i++) sum += spc[i] == sp ? val[k][i] : 0.0;
        part[g][c] = sum;
    }
    __syncthreads();
    if (t < ncol) {
        double sum = 0.0;
#pragma unroll
        for (int g = 0; g < kSeg; g++) sum += part[g][t];
        out[t] = sum;
    }
}

}  // namespace gl
