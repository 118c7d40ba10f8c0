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

// One site of the leapfrog step n -> n+1; (ix, iy) must lie on the lattice.
// If F is non-null the same pass writes the local-frame site fields at tau_n
// that the particle push reads (NGP reading of the colored particle-in-cell
// coupling), reusing the plaquettes and transported scalars of the forces:
//   E_i = 1/2 [Ebar_i(x) + U_i^dag(x-i) Ebar_i(x-i) U_i(x-i)] / tau,
//         Ebar = (E^{n-1/2} + E^{n+1/2}) / 2,
//   E_z = (pi^{n-1/2} + pi^{n+1/2}) / 2,
//   B_x = -D_2 phi / tau, B_y = D_1 phi / tau, D_i phi = (Phi_{+i} - Phi_{-i}) / 2,
//   B_z = -(1/4) (sum of the four plaquettes at x, each transported to x).
// The second half of E_i belongs to the site x+i; this thread owns the link
// U_i(x) and Ebar_i(x) it needs, so it stores that half at x+i in a plane of
// its own (slots 48..63) and the push adds the two halves.
// Keeps the instruction scheduler from hoisting the next phase's loads above
// this point: with every load of the step in flight at once the kernel needs
// more than twice the registers, and the lost occupancy costs more than the
// overlap gains.
__device__ __forceinline__ void phase_fence() { __builtin_amdgcn_sched_barrier(0); }

// E_i^{n+1/2}(x) and U_i^{n+1}(x) from the force fe; with F, also this
// site's half of the electric site field and the transported half of x+i
template <typename T>
__device__ __forceinline__ void update_link(const T *__restrict__ Ein, T *__restrict__ Eout, const T *__restrict__ Uin,
                                            T *__restrict__ Uout, size_t n2, size_t x, size_t xpi, const T *fe, T dtau,
                                            T s, int reunit, T *__restrict__ F, int slot, T inv_tau) {
    T e[8], eb[8];
    load_a(Ein, n2, x, e);
#pragma unroll
    for (int a = 0; a < 8; a++) {
        eb[a] = e[a];
        e[a] += dtau * fe[a];
    }
    store_a(Eout, n2, x, e);
    const M3<T> u = load_m(Uin, n2, x);
    M3<T> un = mul(expi_alg(e, s), u);
    if (reunit) un = reunitarize(un);
    store_m(Uout, n2, x, un);
    if (F) {
        T t[8];
#pragma unroll
        for (int a = 0; a < 8; a++) eb[a] = T(0.25) * inv_tau * (eb[a] + e[a]);   // Ebar / (2 tau)
        store_rec(F, n2, x, slot, eb);
        transport_dn(u, herm_from_alg(eb), t);
        store_rec(F, n2, xpi, 48 + slot, t);
    }
}

// Phi_{+i}(x) = U_i(x) phi(x+i) U_i^dag(x) and Phi_{-i}(x) = U_i^dag(x-i) phi(x-i) U_i(x-i)
// as algebra components; adds -(i/tau)[phi(x), Phi_{+i}] to the E_i force
template <typename T>
__device__ __forceinline__ void scalar_links(const T *__restrict__ Ui, const T *__restrict__ phi, size_t n2, size_t x,
                                             size_t xp, size_t xm, const T *ph, T inv_tau, T *fe, T *pf, T *pb) {
    T v[8], c[8];
    const M3<T> u = load_m(Ui, n2, x);
    load_a(phi, n2, xp, v);
    M3<T> Pf = mul_nd(mul(u, herm_from_alg(v)), u);
    alg_from_herm(comm_term(herm_from_alg(ph), Pf, inv_tau), c);
#pragma unroll
    for (int a = 0; a < 8; a++) fe[a] += c[a];
    alg_from_herm(Pf, pf);
    const M3<T> um = load_m(Ui, n2, xm);
    load_a(phi, n2, xm, v);
    alg_from_herm(mul(mul_dn(um, herm_from_alg(v)), um), pb);
}

// One site of the leapfrog step n -> n+1; (ix, iy) must lie on the lattice.
// If F is non-null the same pass writes the local-frame site fields at tau_n
// that the particle push reads (NGP reading of the colored particle-in-cell
// coupling), reusing the plaquettes and transported scalars of the forces:
//   E_i = 1/2 [Ebar_i(x) + U_i^dag(x-i) Ebar_i(x-i) U_i(x-i)] / tau,
//         Ebar = (E^{n-1/2} + E^{n+1/2}) / 2,
//   E_z = (pi^{n-1/2} + pi^{n+1/2}) / 2,
//   B_x = -D_2 phi / tau, B_y = D_1 phi / tau, D_i phi = (Phi_{+i} - Phi_{-i}) / 2,
//   B_z = -(1/4) (sum of the four plaquettes at x, each transported to x).
// The second half of E_i belongs to the site x+i; this thread owns the link
// U_i(x) and Ebar_i(x) it needs, so it stores that half at x+i in a plane of
// its own (slots 48..63) and the push adds the two halves.  Each slot is
// stored as soon as it is known, which keeps few values live.
template <typename T>
__device__ __forceinline__ void field_step_site(int N, const FieldPtrs<T> &in, const FieldPtrs<T> &out,
                                                T *__restrict__ F, int ix, int iy, T tau, T dtau, T tau_h,
                                                int reunit) {
    const size_t n2 = plane_pitch(N);
    const Nbr nb = neighbours(ix, iy, N);
    const T *U1 = in.U, *U2 = in.U + 18 * n2;
    const T inv_tau = T(1) / tau;

    T fe1[8], fe2[8], cl[8];
    {
        T px[8];   // [P(x)]_X
        {
            const M3<T> P = plaq(load_m(U1, n2, nb.x), load_m(U2, n2, nb.xp1), load_m(U1, n2, nb.xp2),
                                 load_m(U2, n2, nb.x));
            alg_proj(P, px);
        }
        phase_fence();
        // E_1 force: -tau([P(x)] - U_2^dag(x-2)[P(x-2)]U_2(x-2))
        {
            const M3<T> u2m = load_m(U2, n2, nb.xm2);
            const M3<T> P = plaq(load_m(U1, n2, nb.xm2), load_m(U2, n2, nb.xp1m2), load_m(U1, n2, nb.x), u2m);
            T pa[8], t[8];
            alg_proj(P, pa);
            transport_dn(u2m, herm_from_alg(pa), t);
#pragma unroll
            for (int a = 0; a < 8; a++) {
                fe1[a] = -tau * (px[a] - t[a]);
                cl[a] = px[a] + t[a];
            }
        }
        phase_fence();
        // E_2 force: -tau(U_1^dag(x-1)[P(x-1)]U_1(x-1) - [P(x)])
        {
            const M3<T> u1m = load_m(U1, n2, nb.xm1);
            const M3<T> P = plaq(u1m, load_m(U2, n2, nb.x), load_m(U1, n2, nb.xm1p2), load_m(U2, n2, nb.xm1));
            T pa[8], t[8];
            alg_proj(P, pa);
            transport_dn(u1m, herm_from_alg(pa), t);
#pragma unroll
            for (int a = 0; a < 8; a++) {
                fe2[a] = -tau * (t[a] - px[a]);
                cl[a] += t[a];
            }
        }
    }
    phase_fence();
    if (F) {
        // fourth clover plaquette P(x-1-2), moved to x along x-1-2 -> x-2 -> x
        const M3<T> u1mm = load_m(U1, n2, nb.xm1m2);
        const M3<T> u2m = load_m(U2, n2, nb.xm2);
        const M3<T> P = plaq(u1mm, u2m, load_m(U1, n2, nb.xm1), load_m(U2, n2, nb.xm1m2));
        T pa[8], t[8];
        alg_proj(P, pa);
        transport_dn(mul(u1mm, u2m), herm_from_alg(pa), t);
#pragma unroll
        for (int a = 0; a < 8; a++) t[a] = T(-0.25) * (cl[a] + t[a]);
        store_rec(F, n2, nb.x, 40, t);   // B_z
    }
    phase_fence();
    // scalar couplings and the pi force (Laplacian of phi)
    T ph[8], fpi[8];
    load_a(in.phi, n2, nb.x, ph);
    {
        T pf[8], pb[8];
        scalar_links(U1, in.phi, n2, nb.x, nb.xp1, nb.xm1, ph, inv_tau, fe1, pf, pb);
#pragma unroll
        for (int a = 0; a < 8; a++) {
            fpi[a] = pf[a] + pb[a];
            pf[a] = T(0.5) * inv_tau * (pf[a] - pb[a]);
        }
        if (F) store_rec(F, n2, nb.x, 32, pf);   // B_y = D_1 phi / tau
        phase_fence();
        scalar_links(U2, in.phi, n2, nb.x, nb.xp2, nb.xm2, ph, inv_tau, fe2, pf, pb);
#pragma unroll
        for (int a = 0; a < 8; a++) {
            fpi[a] = inv_tau * (fpi[a] + pf[a] + pb[a] - T(4) * ph[a]);
            pf[a] = T(-0.5) * inv_tau * (pf[a] - pb[a]);
        }
        if (F) store_rec(F, n2, nb.x, 24, pf);   // B_x = -D_2 phi / tau
    }
    phase_fence();
    const T s = dtau / tau_h;
    update_link(in.E, out.E, U1, out.U, n2, nb.x, nb.xp1, fe1, dtau, s, reunit, F, 0, inv_tau);
    phase_fence();
    update_link(in.E + 8 * n2, out.E + 8 * n2, U2, out.U + 18 * n2, n2, nb.x, nb.xp2, fe2, dtau, s, reunit, F, 8,
                inv_tau);
    T p[8], ez[8];
    load_a(in.pi, n2, nb.x, p);
#pragma unroll
    for (int a = 0; a < 8; a++) {
        ez[a] = p[a];
        p[a] += dtau * fpi[a];
        ph[a] += dtau * tau_h * p[a];
        ez[a] = T(0.5) * (ez[a] + p[a]);
    }
    store_a(out.pi, n2, nb.x, p);
    store_a(out.phi, n2, nb.x, ph);
    if (F) store_rec(F, n2, nb.x, 16, ez);   // E_z
}

}  // namespace gl
