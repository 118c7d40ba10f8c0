// fields_dev.hpp -- per-site device functions of the leapfrog step and of the
// local-frame site fields, shared by the single-event and the batched kernels.
// The scheme and the site-field reading are described in fields.hip.
#pragma once
#include "internal.hpp"
#include "su3.hpp"

namespace gl {

template <typename T>
__device__ __forceinline__ void store_rec(T *__restrict__ F, size_t n2, size_t x, int slot, const T *v) {
    store_a(F + (size_t)slot * n2, n2, x, v);
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

// -(i/tau)[phi, Phi] as a hermitian matrix
template <typename T>
__device__ __forceinline__ M3<T> comm_term(const M3<T> &ph, const M3<T> &Ph, T inv_tau) {
    M3<T> c = sub(mul(ph, Ph), mul(Ph, ph));
    M3<T> r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {   // -(i/tau) * (cr + i ci) = (ci - i cr)/tau
            r.re[i][j] = c.im[i][j] * inv_tau;
            r.im[i][j] = -c.re[i][j] * inv_tau;
        }
    return r;
}

// one site of the leapfrog step; (ix, iy) must lie on the lattice
template <typename T>
__device__ __forceinline__ void field_step_site(int N, const FieldPtrs<T> &in, const FieldPtrs<T> &out, int ix,
                                                int iy, T tau, T dtau, T tau_h, int reunit) {
    const size_t n2 = plane_pitch(N);
    Nbr nb = neighbours(ix, iy, N);
    const T *U1 = in.U, *U2 = in.U + 18 * n2;

    const T inv_tau = T(1) / tau;
    M3<T> ph = [&] { T v[8]; load_a(in.phi, n2, nb.x, v); return herm_from_alg(v); }();

    T fe1[8], fe2[8], fpi[8];
    {
        M3<T> u1x = load_m(U1, n2, nb.x);
        M3<T> u2x = load_m(U2, n2, nb.x);
        M3<T> Px;
        {
            M3<T> u2xp1 = load_m(U2, n2, nb.xp1);
            M3<T> u1xp2 = load_m(U1, n2, nb.xp2);
            M3<T> P = plaq(u1x, u2xp1, u1xp2, u2x);
            T pa[8];
            alg_proj(P, pa);
            Px = herm_from_alg(pa);
        }
        // E_1 force: -tau([P(x)] - U_2^dag(x-2)[P(x-2)]U_2(x-2))
        {
            M3<T> u2m = load_m(U2, n2, nb.xm2);
            M3<T> u1m = load_m(U1, n2, nb.xm2);
            M3<T> u2pm = load_m(U2, n2, nb.xp1m2);
            M3<T> P = plaq(u1m, u2pm, u1x, u2m);
            T pa[8];
            alg_proj(P, pa);
            T t[8];
            transport_dn(u2m, herm_from_alg(pa), t);
            T px[8];
            alg_from_herm(Px, px);
#pragma unroll
            for (int a = 0; a < 8; a++) fe1[a] = -tau * (px[a] - t[a]);
        }
        // E_2 force: -tau(U_1^dag(x-1)[P(x-1)]U_1(x-1) - [P(x)])
        {
            M3<T> u1m = load_m(U1, n2, nb.xm1);
            M3<T> u2m = load_m(U2, n2, nb.xm1);
            M3<T> u1mp = load_m(U1, n2, nb.xm1p2);
            M3<T> P = plaq(u1m, u2x, u1mp, u2m);
            T pa[8];
            alg_proj(P, pa);
            T t[8];
            transport_dn(u1m, herm_from_alg(pa), t);
            T px[8];
            alg_from_herm(Px, px);
#pragma unroll
            for (int a = 0; a < 8; a++) fe2[a] = -tau * (t[a] - px[a]);
        }
        // scalar couplings: Phi_{+-i}
        M3<T> lap = m_zero<T>();
        {
            T v[8];
            load_a(in.phi, n2, nb.xp1, v);
            M3<T> Pf = mul_nd(mul(u1x, herm_from_alg(v)), u1x);
            T c[8];
            alg_from_herm(comm_term(ph, Pf, inv_tau), c);
#pragma unroll
            for (int a = 0; a < 8; a++) fe1[a] += c[a];
            lap = add(lap, Pf);
            load_a(in.phi, n2, nb.xp2, v);
            Pf = mul_nd(mul(u2x, herm_from_alg(v)), u2x);
            alg_from_herm(comm_term(ph, Pf, inv_tau), c);
#pragma unroll
            for (int a = 0; a < 8; a++) fe2[a] += c[a];
            lap = add(lap, Pf);
        }
        {
            T v[8];
            M3<T> u1m = load_m(U1, n2, nb.xm1);
            load_a(in.phi, n2, nb.xm1, v);
            lap = add(lap, mul(mul_dn(u1m, herm_from_alg(v)), u1m));
            M3<T> u2m = load_m(U2, n2, nb.xm2);
            load_a(in.phi, n2, nb.xm2, v);
            lap = add(lap, mul(mul_dn(u2m, herm_from_alg(v)), u2m));
        }
        T l[8], p0[8];
        alg_from_herm(lap, l);
        alg_from_herm(ph, p0);
#pragma unroll
        for (int a = 0; a < 8; a++) fpi[a] = inv_tau * (l[a] - T(4) * p0[a]);

        // updates
        T e[8];
        const T s = dtau / tau_h;
        load_a(in.E, n2, nb.x, e);
#pragma unroll
        for (int a = 0; a < 8; a++) e[a] += dtau * fe1[a];
        store_a(out.E, n2, nb.x, e);
        M3<T> un = mul(expi_alg(e, s), u1x);
        if (reunit) un = reunitarize(un);
        store_m(out.U, n2, nb.x, un);
        load_a(in.E + 8 * n2, n2, nb.x, e);
#pragma unroll
        for (int a = 0; a < 8; a++) e[a] += dtau * fe2[a];
        store_a(out.E + 8 * n2, n2, nb.x, e);
        un = mul(expi_alg(e, s), u2x);
        if (reunit) un = reunitarize(un);
        store_m(out.U + 18 * n2, n2, nb.x, un);
    }
    T p[8], f[8];
    load_a(in.pi, n2, nb.x, p);
    load_a(in.phi, n2, nb.x, f);
#pragma unroll
    for (int a = 0; a < 8; a++) {
        p[a] += dtau * fpi[a];
        f[a] += dtau * tau_h * p[a];
    }
    store_a(out.pi, n2, nb.x, p);
    store_a(out.phi, n2, nb.x, f);
}

template <typename T>
__device__ __forceinline__ void site_fields_site(int N, const FieldPtrs<T> &o, const FieldPtrs<T> &nw,
                                                 T *__restrict__ F, int ix, int iy, T tau) {
    const size_t n2 = plane_pitch(N);
    Nbr nb = neighbours(ix, iy, N);
    const T *U1 = o.U, *U2 = o.U + 18 * n2;
    const T inv_tau = T(1) / tau;
    T out[8];
    // electric: E_i^s = 1/2 [Ebar_i(x) + U_i^dag(x-i) Ebar_i(x-i) U_i(x-i)]
#pragma unroll
    for (int d = 0; d < 2; d++) {
        size_t xm = d == 0 ? nb.xm1 : nb.xm2;
        const T *Eo = o.E + 8 * n2 * d, *En = nw.E + 8 * n2 * d;
        T a[8], b[8], t[8];
        load_a(Eo, n2, nb.x, a);
        load_a(En, n2, nb.x, b);
        T c[8], cm[8];
#pragma unroll
        for (int k = 0; k < 8; k++) c[k] = T(0.5) * (a[k] + b[k]);
        load_a(Eo, n2, xm, a);
        load_a(En, n2, xm, b);
#pragma unroll
        for (int k = 0; k < 8; k++) cm[k] = T(0.5) * (a[k] + b[k]);
        M3<T> um = load_m(d == 0 ? U1 : U2, n2, xm);
        transport_dn(um, herm_from_alg(cm), t);
#pragma unroll
        for (int k = 0; k < 8; k++) out[k] = T(0.5) * inv_tau * (c[k] + t[k]);
        store_rec(F, n2, nb.x, 8 * d, out);
    }
    {
        T a[8], b[8];
        load_a(o.pi, n2, nb.x, a);
        load_a(nw.pi, n2, nb.x, b);
#pragma unroll
        for (int k = 0; k < 8; k++) out[k] = T(0.5) * (a[k] + b[k]);
        store_rec(F, n2, nb.x, 16, out);
    }
    // magnetic from phi: D_i phi = 1/2 (Phi_{+i} - Phi_{-i})
    M3<T> u1x = load_m(U1, n2, nb.x), u2x = load_m(U2, n2, nb.x);
#pragma unroll
    for (int d = 0; d < 2; d++) {
        size_t xp = d == 0 ? nb.xp1 : nb.xp2, xm = d == 0 ? nb.xm1 : nb.xm2;
        T v[8];
        load_a(o.phi, n2, xp, v);
        const M3<T> &ux = d == 0 ? u1x : u2x;
        M3<T> Pf = mul_nd(mul(ux, herm_from_alg(v)), ux);
        M3<T> um = load_m(d == 0 ? U1 : U2, n2, xm);
        load_a(o.phi, n2, xm, v);
        M3<T> Pb = mul(mul_dn(um, herm_from_alg(v)), um);
        T dphi[8];
        alg_from_herm(sub(Pf, Pb), dphi);
        // B_x = -D_2 phi / tau (slot 3), B_y = +D_1 phi / tau (slot 4)
        T sgn = d == 0 ? T(0.5) : T(-0.5);
#pragma unroll
        for (int k = 0; k < 8; k++) out[k] = sgn * inv_tau * dphi[k];
        store_rec(F, n2, nb.x, 8 * (d == 0 ? 4 : 3), out);
    }
    // clover
    T cl[8];
    {
        M3<T> P = plaq(u1x, load_m(U2, n2, nb.xp1), load_m(U1, n2, nb.xp2), u2x);
        alg_proj(P, cl);
    }
    {
        M3<T> u1m = load_m(U1, n2, nb.xm1);
        M3<T> P = plaq(u1m, u2x, load_m(U1, n2, nb.xm1p2), load_m(U2, n2, nb.xm1));
        T pa[8], t[8];
        alg_proj(P, pa);
        transport_dn(u1m, herm_from_alg(pa), t);
#pragma unroll
        for (int k = 0; k < 8; k++) cl[k] += t[k];
    }
    M3<T> u2m = load_m(U2, n2, nb.xm2);
    {
        M3<T> P = plaq(load_m(U1, n2, nb.xm2), load_m(U2, n2, nb.xp1m2), u1x, u2m);
        T pa[8], t[8];
        alg_proj(P, pa);
        transport_dn(u2m, herm_from_alg(pa), t);
#pragma unroll
        for (int k = 0; k < 8; k++) cl[k] += t[k];
    }
    {
        M3<T> u1mm = load_m(U1, n2, nb.xm1m2);
        M3<T> P = plaq(u1mm, u2m, load_m(U1, n2, nb.xm1), load_m(U2, n2, nb.xm1m2));
        M3<T> W = mul(u1mm, u2m);   // path x-1-2 -> x-2 -> x
        T pa[8], t[8];
        alg_proj(P, pa);
        transport_dn(W, herm_from_alg(pa), t);
#pragma unroll
        for (int k = 0; k < 8; k++) cl[k] += t[k];
    }
#pragma unroll
    for (int k = 0; k < 8; k++) out[k] = T(-0.25) * cl[k];
    store_rec(F, n2, nb.x, 40, out);
    load_a(o.phi, n2, nb.x, out);
    store_rec(F, n2, nb.x, 48, out);
}

}  // namespace gl
