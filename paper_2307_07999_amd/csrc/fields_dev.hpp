// fields_dev.hpp -- per-site device functions of the leapfrog step and of the
// local-frame site fields, shared by the single-event and the batched kernels.
// The scheme is described in fields.hip, the site-field reading at
// field_step_link.
#pragma once
#include "internal.hpp"
#include "su3.hpp"

namespace gl {

// The field step's transports use the hermitian-aware products in FP64; in
// FP32 only the staple's and the clover corner's, which come before the
// scalar couplings, where registers are free (FP32 field step 38.0 -> 37.3
// us at 512^2; taken everywhere, FP32 spills one more dword and loses it).
template <typename T>
constexpr bool kHermFS = sizeof(T) == 8;
constexpr bool kHermPlaq = true;
// FP64: E_i(x) and the pi half are loaded before the scalar couplings and
// arrive while those are computed (the step waited on them: 79.6 -> 74.5 us
// at 512^2).  FP32 loads them where they are used: held over the couplings
// its registers would spill (38.4 -> 41.9 us).
template <typename T>
constexpr bool kEarlyEP = sizeof(T) == 8;

// values slot..slot+7 of the site-field record of site x
template <typename T>
__device__ __forceinline__ void store_rec(T *__restrict__ F, size_t n2, size_t x, int slot, const T *v) {
    chunk_store_n_l<8>(F, n2, x, slot, v);
}

struct Nbr {
    size_t x, xp1, xm1, xp2, xm2, xp1m2, xm1p2, xm1m2;
};

__device__ __forceinline__ Nbr neighbours(int ix, int iy, int N) {
    int ixp = ix + 1 == N ? 0 : ix + 1, ixm = ix == 0 ? N - 1 : ix - 1;
    int iyp = iy + 1 == N ? 0 : iy + 1, iym = iy == 0 ? N - 1 : iy - 1;
    Nbr n;
    n.x = (size_t)ix + (size_t)N * iy;
    n.xp1 = (size_t)ixp + (size_t)N * iy;
    n.xm1 = (size_t)ixm + (size_t)N * iy;
    n.xp2 = (size_t)ix + (size_t)N * iyp;
    n.xm2 = (size_t)ix + (size_t)N * iym;
    n.xp1m2 = (size_t)ixp + (size_t)N * iym;
    n.xm1p2 = (size_t)ixm + (size_t)N * iyp;
    n.xm1m2 = (size_t)ixm + (size_t)N * iym;
    return n;
}

// P(x) = U_1(x) U_2(x+1) U_1^dag(x+2) U_2^dag(x)
template <typename T>
__device__ __forceinline__ M3<T> plaq(const M3<T> &u1x, const M3<T> &u2xp1, const M3<T> &u1xp2,
                                      const M3<T> &u2x) {
    return mul_nd(mul_nd(mul(u1x, u2xp1), u1xp2), u2x);
}

// Exchange with the partner lane of a site's lane pair (lanes 2s and 2s+1).
template <typename T>
__device__ __forceinline__ T pair_swap(T v) {
    return dpp<kDppSwap1>(v);
}
template <typename T>
__device__ __forceinline__ M3<T> pair_swap(const M3<T> &m) {
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            r.re[i][j] = pair_swap(m.re[i][j]);
            r.im[i][j] = pair_swap(m.im[i][j]);
        }
    return r;
}

// Components 4h..4h+3 of an algebra vector v into a record slot (the two
// lanes of a site store one half each).
template <typename T>
__device__ __forceinline__ void store_half(T *__restrict__ F, size_t n2, size_t x, int slot, const T *v, int h) {
    constexpr int NV = 16 / sizeof(T);
    T w[4];
#pragma unroll
    for (int k = 0; k < 4; k++) w[k] = h ? v[4 + k] : v[k];
#pragma unroll
    for (int k = 0; k < 4; k += NV) chunk_st16_l(F, n2, x, slot + 4 * h + k, w + k);
}

// Links of a block of SX x SY sites and a one-site halo, staged in LDS;
// region site (rx, ry) is the lattice site (x0 - 1 + rx, y0 - 1 + ry) mod N.
// Chunk-major like the field state: the values of a site are held in
// 16-byte chunks (NV = 16 / sizeof(T) values), chunk c of all region sites
// contiguous, so a lane reads a link with 16-byte LDS accesses.  Per site:
// U_1 in chunks [0, LC), U_2 in [LC, 2 LC); a link is its 18 values (entry
// (i,j) real at 2(3i+j), imaginary next to it), padded in FP32 to 5 whole
// chunks.  The tile also holds the plaquette algebra [P(x)]_X of the region
// sites (rx, ry), rx <= SX, ry <= SY (the block and its lower and left halo),
// computed once per step and read by the staples and the clover of the
// neighbouring sites.
template <typename T, int SX, int SY>
struct LinkTile {
    static constexpr int NV = 16 / (int)sizeof(T);
    static constexpr int LC = (18 + NV - 1) / NV;      // chunks per link
    static constexpr int NC = 2 * LC;                  // chunks per site
    static constexpr int RX = SX + 2, RY = SY + 2, R = RX * RY;
    static constexpr int PX = SX + 1, PN = PX * (SY + 1);   // plaquette-algebra region
    struct alignas(16) Chunk {
        T v[NV];
    };
    Chunk c[NC * R];
    Chunk pa[(8 / NV) * PN];
    // link d (0: U_1, 1: U_2) of region site r
    __device__ __forceinline__ M3<T> m(int d, int r) const {
        T v[LC * NV];
        const Chunk *p = c + (size_t)(LC * d) * R + r;
#pragma unroll
        for (int j = 0; j < 18 / NV; j++) {
            const Chunk w = p[j * R];
#pragma unroll
            for (int k = 0; k < NV; k++) v[j * NV + k] = w.v[k];
        }
        if constexpr (18 % NV != 0) {   // FP32: values 16 and 17 in the first half of the fifth chunk
            typedef T T2 __attribute__((ext_vector_type(2)));
            const T2 h = *reinterpret_cast<const T2 *>(&p[(18 / NV) * R]);
            v[16] = h.x;
            v[17] = h.y;
        }
        M3<T> u;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                u.re[i][j] = v[2 * (3 * i + j)];
                u.im[i][j] = v[2 * (3 * i + j) + 1];
            }
        return u;
    }
    // index of region site (rx, ry) in the plaquette-algebra region
    static __device__ __forceinline__ int pidx(int rx, int ry) { return rx + PX * ry; }
    __device__ __forceinline__ void plaq(int p, T *out) const {
#pragma unroll
        for (int j = 0; j < 8 / NV; j++) {
            const Chunk w = pa[j * PN + p];
#pragma unroll
            for (int k = 0; k < NV; k++) out[j * NV + k] = w.v[k];
        }
    }
    __device__ __forceinline__ void put_plaq(int p, const T *v) {
#pragma unroll
        for (int j = 0; j < 8 / NV; j++) {
            Chunk w;
#pragma unroll
            for (int k = 0; k < NV; k++) w.v[k] = v[j * NV + k];
            pa[j * PN + p] = w;
        }
    }
};

// All threads of the workgroup copy the tile's links from the state; the
// caller synchronises the workgroup before the tile is read.
template <typename T, int SX, int SY>
__device__ __forceinline__ void stage_tile(LinkTile<T, SX, SY> &t, int N, const FieldPtrs<T> &in, int x0, int y0,
                                           int tid, int nthreads) {
    using Tl = LinkTile<T, SX, SY>;
    using Chunk = typename Tl::Chunk;
    constexpr int NV = Tl::NV, LC = Tl::LC, R = Tl::R;
    const size_t n2 = plane_pitch(N);
    for (int r = tid; r < R; r += nthreads) {
        int gx = (x0 - 1 + r % Tl::RX) % N, gy = (y0 - 1 + r / Tl::RX) % N;
        gx += gx < 0 ? N : 0;
        gy += gy < 0 ? N : 0;
        const size_t site = (size_t)gx + (size_t)N * gy;
        // the stored rows of the site's two links, in 16-byte loads; each
        // link is completed with its third row once here
        T s[2 * kLinkVals], u[36];
#pragma unroll
        for (int k = 0; k < 2 * kLinkVals; k += NV) chunk_ld16(in.U, n2, site, k, s + k);
#pragma unroll
        for (int d = 0; d < 2; d++) {
            const M3<T> m = link_from_rows(s + kLinkVals * d);
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    u[18 * d + 2 * (3 * i + j)] = m.re[i][j];
                    u[18 * d + 2 * (3 * i + j) + 1] = m.im[i][j];
                }
        }
#pragma unroll
        for (int d = 0; d < 2; d++)
#pragma unroll
            for (int j = 0; j < LC; j++) {
                Chunk w;
#pragma unroll
                for (int k = 0; k < NV; k++) {
                    const int i = j * NV + k;   // value of the link; FP32 pads 18, 19
                    w.v[k] = i < 18 ? u[18 * d + i] : T(0);
                }
                t.c[(size_t)(LC * d + j) * R + r] = w;
            }
    }
}

// E_i^{n+1/2}(x) and U_i^{n+1}(x), i = d + 1, from E_i^{n-1/2}(x) = ein, the
// force fe and U_i(x) = u; with F, also this site's half of the electric
// site field (eb) and the half transported to x+i (t), which the caller
// stores or exchanges
template <typename T, bool ST>
__device__ __forceinline__ void update_link(const T *ein, T *__restrict__ Eout, const M3<T> &u,
                                            T *__restrict__ Uout, size_t n2, size_t x, int d, const T *fe, T dtau,
                                            T s, int reunit, bool site_fields, T inv_tau, T *eb, T *t) {
    T e[8];
#pragma unroll
    for (int a = 0; a < 8; a++) {
        e[a] = ein[a];
        eb[a] = e[a];
        e[a] += dtau * fe[a];
    }
    chunk_store_n_l<8, stream_policy(ST)>(Eout, n2, x, 8 * d, e);   // the new state is streamed (ST)
    M3<T> un = mul(expi_alg(e, s), u);
    if (reunit) un = reunitarize(un);
    T uv[18];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            uv[2 * (3 * i + j)] = un.re[i][j];
            uv[2 * (3 * i + j) + 1] = un.im[i][j];
        }
    // the new links stay cached: the next step stages them, halo included,
    // into its tiles (streaming them cost the FP64 step 4.5 us)
    chunk_store_link_l(Uout, n2, x, d, uv);
    if (site_fields) {
#pragma unroll
        for (int a = 0; a < 8; a++) eb[a] = T(0.25) * inv_tau * (eb[a] + e[a]);   // Ebar / (2 tau)
        transport_dn<kHermFS<T>>(u, eb, t);
    }
}

// One link direction of one site of the leapfrog step n -> n+1: the two
// lanes of a pair (d = 0, 1) share the site (ix, iy) = (x0 + lx, y0 + ly) of
// the staged tile, and lane d owns direction i = d + 1 (j is the other one).
// Every thread of the workgroup calls this (active: the site lies on the
// lattice), since it synchronises the workgroup (once, three times when it
// writes site fields).  First the plaquette
// at x is assembled from the halves U_i(x) U_j(x+i) of both lanes and its
// algebra stored in the tile, with those of the tile's lower and left halo
// sites (computed by the first threads); then lane d reads the staple
// plaquette at y = x - j and the clover's corner plaquette from the tile,
// forms its transported scalars Phi_{+-i} (phi read from the state), and
// updates E_i and U_i; the Laplacian of phi, the clover and the pi, phi
// update are shared across the pair.  For i = 1, 2:
//   E_1 += dtau { -tau ([P(x)]_X - U_2^dag(x-2)[P(x-2)]_X U_2(x-2)) - (i/tau)[phi, Phi_{+1}] }
//   E_2 += dtau { -tau (U_1^dag(x-1)[P(x-1)]_X U_1(x-1) - [P(x)]_X) - (i/tau)[phi, Phi_{+2}] }
//   pi  += (dtau/tau) sum_i (Phi_{+i} + Phi_{-i} - 2 phi)
//   U_i <- exp(i dtau E_i / tau_{n+1/2}) U_i,   phi += dtau tau_{n+1/2} pi
// If F is non-null the same pass writes the local-frame site fields at tau_n
// that the particle push reads (NGP reading of the colored particle-in-cell
// coupling):
//   E_i = 1/2 [Ebar_i(x) + U_i^dag(x-i) Ebar_i(x-i) U_i(x-i)] / tau,
//         Ebar = (E^{n-1/2} + E^{n+1/2}) / 2,
//   E_z = (pi^{n-1/2} + pi^{n+1/2}) / 2,
//   B_x = -D_2 phi / tau, B_y = D_1 phi / tau, D_i phi = (Phi_{+i} - Phi_{-i}) / 2,
//   B_z = -(1/4) (sum of the four plaquettes at x, each transported to x).
// The second half of E_i at x+i needs U_i(x) and Ebar_i(x), which lane d
// owns: it hands that half to the lane of x+i through LDS, which adds it to
// its own, or, at the sites of half_stored, stores it in x+i's slots 48..63
// for the readers to add.
template <typename T, int SX, int SY, bool ST = kStreamed<T>>
__device__ __forceinline__ void field_step_link(LinkTile<T, SX, SY> &tl, int N, const FieldPtrs<T> &in,
                                                const FieldPtrs<T> &out, T *__restrict__ F, int x0, int y0, int lx,
                                                int ly, int d, int tid, bool active, T tau, T dtau, T tau_h,
                                                int reunit) {
    using Tl = LinkTile<T, SX, SY>;
    constexpr int RX = Tl::RX;
    const size_t n2 = plane_pitch(N);
    const bool d0 = d == 0;
    const int ix = x0 + lx, iy = y0 + ly;
    // region indices of the neighbours
    const int rx = (lx + 1) + RX * (ly + 1);
    const int di = d0 ? 1 : RX;                      // step along i
    const int rpi = rx + di, rmi = rx - di;          // x + i, x - i
    const int ry = rx - (d0 ? RX : 1);               // y = x - j
    const int rz = rx - 1 - RX;                      // z = x - 1 - 2
    const int li = d, lj = 1 - d;                    // tile links of U_i, U_j
    // lattice indices for the global reads and writes
    const int ixp = ix + 1 == N ? 0 : ix + 1, iyp = iy + 1 == N ? 0 : iy + 1;
    const int ixm = ix == 0 ? N - 1 : ix - 1, iym = iy == 0 ? N - 1 : iy - 1;
    const size_t x = (size_t)ix + (size_t)N * iy;
    const size_t xpi = d0 ? (size_t)ixp + (size_t)N * iy : (size_t)ix + (size_t)N * iyp;
    const size_t xmi = d0 ? (size_t)ixm + (size_t)N * iy : (size_t)ix + (size_t)N * iym;
    const T inv_tau = T(1) / tau;
    const T sgn = d0 ? T(1) : T(-1);

    // phi at x and x +- i, in flight during the plaquettes
    T ph[8], php[8], phm[8];
    if (active) {
        chunk_load_a(in.phi, n2, x, 0, ph);
        chunk_load_a(in.phi, n2, xpi, 0, php);
        chunk_load_a(in.phi, n2, xmi, 0, phm);
    }
    // [P(x)]_X, P(x) = h0 h1^dag with the half products h0 = U_1(x) U_2(x+1)
    // (lane 0) and h1 = U_2(x) U_1(x+2) (lane 1); lane 1 forms h1 h0^dag =
    // P(x)^dag, whose projection is -[P(x)]_X.  Lane 0 stores the algebra,
    // computed exactly as for the halo sites, so the stored values do not
    // depend on the tiling.
    T px[8];
    if (active) {
        const M3<T> h = mul(tl.m(li, rx), tl.m(lj, rpi));
        alg_proj(mul_nd(h, pair_swap(h)), px);
#pragma unroll
        for (int a = 0; a < 8; a++) px[a] *= sgn;
        if (d0) tl.put_plaq(Tl::pidx(lx + 1, ly + 1), px);
    }
    // the halo plaquettes: region row 0 (rx = 0..SX) and column 0 (ry = 1..SY),
    // whole, one per thread, as h0 h1^dag like the block's
    for (int hh = tid; hh < SX + SY + 1; hh += 2 * SX * SY) {
        const int hx = hh <= SX ? hh : 0, hy = hh <= SX ? 0 : hh - SX;
        const int r = hx + RX * hy;
        const M3<T> h0 = mul(tl.m(0, r), tl.m(1, r + 1)), h1 = mul(tl.m(1, r), tl.m(0, r + RX));
        T v[8];
        alg_proj(mul_nd(h0, h1), v);
        tl.put_plaq(Tl::pidx(hx, hy), v);
    }
    __syncthreads();
    // this lane's half of E_i at x and the half it transports to x+i
    T eb[8], tr[8];
    if (active) {
        const M3<T> ui = tl.m(li, rx);   // U_i(x)
        T fe[8], cl[8];
        {
            // staple: U_j^dag(y) [P(y)]_X U_j(y)
            T pa[8], t[8];
            tl.plaq(Tl::pidx(lx + 1 - d, ly + d), pa);
            transport_dn<kHermPlaq>(tl.m(lj, ry), pa, t);
#pragma unroll
            for (int a = 0; a < 8; a++) {
                fe[a] = -tau * sgn * (px[a] - t[a]);
                cl[a] = px[a] + (t[a] + pair_swap(t[a]));
            }
        }
        if (F) {
            // fourth clover plaquette P(z), moved to x along z -> z+1 -> x, i.e.
            // by C = U_1(z) U_2(z+1)
            T pa[8], t[8];
            tl.plaq(Tl::pidx(lx, ly), pa);
            transport_dn<kHermPlaq>(mul(tl.m(0, rz), tl.m(1, rz + 1)), pa, t);
#pragma unroll
            for (int a = 0; a < 8; a++) t[a] = T(-0.25) * (cl[a] + t[a]);
            store_half(F, n2, x, 40, t, d);   // B_z
        }
        // E_i(x) and this lane's half of pi, read once per step (streamed)
        T ein[8], pv[4];
        if constexpr (kEarlyEP<T>) {
            chunk_load_n_l<8, stream_policy(ST)>(in.E, n2, x, 8 * d, ein);
            chunk_load_n_l<4, stream_policy(ST)>(in.pi, n2, x, 4 * d, pv);
        }
        // scalar couplings: Phi_{+i} in the E_i force, all four in the pi force
        T fpi[8];
        {
            T c[8], pf[8], pb[8];
            transport_nd<kHermFS<T>>(ui, php, pf);   // Phi_{+i}
            alg_comm(ph, pf, c);                        // -i[phi, Phi_{+i}]
            transport_dn<kHermFS<T>>(tl.m(li, rmi), phm, pb);   // Phi_{-i}
#pragma unroll
            for (int a = 0; a < 8; a++) {
                fe[a] = fma(inv_tau, c[a], fe[a]);
                const T l = pf[a] + pb[a];
                fpi[a] = inv_tau * ((l + pair_swap(l)) - T(4) * ph[a]);
                pf[a] = T(0.5) * sgn * inv_tau * (pf[a] - pb[a]);
            }
            // B_y = D_1 phi / tau (lane 0, slot 32), B_x = -D_2 phi / tau (lane 1, slot 24)
            if (F) store_rec(F, n2, x, 32 - 8 * d, pf);
        }
        if constexpr (!kEarlyEP<T>) chunk_load_n_l<8, stream_policy(ST)>(in.E, n2, x, 8 * d, ein);
        update_link<T, ST>(ein, out.E, ui, out.U, n2, x, d, fe, dtau, dtau / tau_h, reunit, F != nullptr, inv_tau, eb,
                           tr);
        // pi, phi and E_z: lane d takes colour components 4d..4d+3
        T pn[4], phn[4], ez[4];
        if constexpr (!kEarlyEP<T>) chunk_load_n_l<4, stream_policy(ST)>(in.pi, n2, x, 4 * d, pv);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            pn[k] = pv[k] + dtau * (d0 ? fpi[k] : fpi[4 + k]);
            phn[k] = (d0 ? ph[k] : ph[4 + k]) + dtau * tau_h * pn[k];
            ez[k] = T(0.5) * (pv[k] + pn[k]);
        }
        chunk_store_n_l<4, stream_policy(ST)>(out.pi, n2, x, 4 * d, pn);
        chunk_store_n_l<4, stream_policy(ST)>(out.phi, n2, x, 4 * d, phn);
        if (F) chunk_store_n_l<4>(F, n2, x, 16 + 4 * d, ez);
    }
    if (F) {
        // E_i site fields: the half transported from x - i is added here when
        // that link is in this workgroup, else stored apart (half_stored).
        // The exchange reuses the tile's LDS once every lane is done with it.
        static_assert(SX % kHalfX == 0 && SY % kHalfY == 0, "tile shape breaks the E_i half rule");
        T *ex = reinterpret_cast<T *>(&tl.c[0]);   // [2][8][SX * SY]
        constexpr int S = SX * SY;
        static_assert(16 * S * sizeof(T) <= sizeof(tl.c), "exchange larger than the link tile");
        __syncthreads();
        if (active) {
            const int ixt = d0 ? ixp : ix, iyt = d0 ? iy : iyp;
            if (half_stored(d, ixt, iyt)) {
                store_rec(F, n2, xpi, 48 + 8 * d, tr);
            } else {   // x+i lies in this tile (the rule keeps x+i off tile edges)
                const int st = (lx + (d0 ? 1 : 0)) + SX * (ly + (d0 ? 0 : 1));
#pragma unroll
                for (int a = 0; a < 8; a++) ex[(d * 8 + a) * S + st] = tr[a];
            }
        }
        __syncthreads();
        if (active) {
            if (!half_stored(d, ix, iy)) {
                const int so = lx + SX * ly;
#pragma unroll
                for (int a = 0; a < 8; a++) eb[a] = eb[a] + ex[(d * 8 + a) * S + so];
            }
            store_rec(F, n2, x, 8 * d, eb);
        }
    }
}

}  // namespace gl
