// Drives every entry point of the CPU oracle on small inputs, for a build
// with AddressSanitizer and UndefinedBehaviorSanitizer (tests only): any
// out-of-bounds access, use after free, leak or undefined operation in the
// oracle makes the sanitizer report and the process fail.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../oracle/glasma_oracle.h"

int main() {
    // algebra and random numbers
    double T[18], U18[18], X[8], M[18];
    for (int a = 0; a < 8; a++) {
        orc_generator(a, T);
        for (int b = 0; b < 8; b++)
            for (int c = 0; c < 8; c++) (void)orc_dsym(a, b, c);
    }
    double x8[8] = {0.3, -0.2, 0.1, 0.7, -0.4, 0.05, 0.2, -0.6};
    orc_expi(x8, U18);
    orc_expm(U18, M);
    orc_proj(M, X);
    uint32_t key[2] = {1u, 2u}, ctr[4] = {3u, 4u, 5u, 6u}, out[4];
    orc_philox(key, ctr, out);
    (void)orc_u53(out[0], out[1]);
    // FFT sizes with radix 2 and 3, Poisson with and without a UV cut
    for (int n : {1, 2, 3, 4, 6, 9, 12, 16}) {
        std::vector<double> d(2 * n);
        for (int i = 0; i < 2 * n; i++) d[i] = std::sin(0.7 * i);
        if (orc_fft(n, d.data(), -1) != 0) return 2;
    }
    for (int N : {4, 6, 8}) {
        std::vector<double> src(N * N), o(N * N);
        for (int i = 0; i < N * N; i++) src[i] = std::cos(1.3 * i);
        if (orc_poisson(N, 0.04, src.data(), o.data()) != 0) return 3;
        if (orc_poisson_uv(N, 0.04, 2.0, src.data(), o.data()) != 0) return 4;
    }
    // the whole initial condition, field steps with site fields, diagnostics
    const int N = 8, n2 = N * N;
    std::vector<double> U(2 * n2 * 18), E(2 * n2 * 8), phi(n2 * 8), pi(n2 * 8), F(n2 * 48), G(n2 * 8), FE(2 * n2 * 8),
        Fpi(n2 * 8);
    double res = 0;
    if (orc_init_glasma_uv(N, 0.5, 0.04, 3.0, 2, 17, 0.125, U.data(), E.data(), phi.data(), pi.data(), &res) != 0)
        return 5;
    // the nucleus links of both nuclei ([2][n2][18] each) for the matching and pi0
    std::vector<double> V(n2 * 18), UA(2 * n2 * 18), UB(2 * n2 * 18), p0(n2 * 8), rho(n2 * 8);
    orc_mv_charges(N, 0.5, 17, 1, 1, rho.data());
    if (orc_wilson_line(N, 0.5, 0.04, 2, 17, 0, V.data()) != 0) return 6;
    orc_nucleus_links(N, V.data(), UA.data());
    if (orc_wilson_line_uv(N, 0.5, 0.04, 3.0, 2, 17, 1, V.data()) != 0) return 6;
    orc_nucleus_links(N, V.data(), UB.data());
    double Ur[18], rr = 0;
    (void)orc_match_link(UA.data(), UB.data(), Ur, 1e-13, 100, &rr);
    orc_pi0(N, U.data(), UA.data(), UB.data(), p0.data());
    for (int n = 1; n < 6; n++) orc_field_step(N, n, 0.125, U.data(), E.data(), phi.data(), pi.data(), F.data());
    int sites[3] = {0, 9, n2 - 1};
    std::vector<double> Us(3 * 36), Es(3 * 16), ps(3 * 8), pis(3 * 8), Fs(3 * 48);
    orc_field_step_sites(N, 6, 0.125, U.data(), E.data(), phi.data(), pi.data(), 3, sites, Us.data(), Es.data(),
                         ps.data(), pis.data(), Fs.data());
    orc_forces(N, 0.75, U.data(), phi.data(), FE.data(), Fpi.data());
    double en[4];
    orc_energy(N, 0.75, U.data(), E.data(), phi.data(), pi.data(), en);
    orc_gauss(N, U.data(), E.data(), phi.data(), pi.data(), G.data());
    // particles of two species through a few coupled steps
    const int np = 40;
    std::vector<int> cell(2 * np), species(np);
    std::vector<double> off(2 * np), eta(np), p(3 * np), Q(8 * np), pv(3 * np);
    orc_particles_init(N, 5, 0, 0, 0.3, np / 2, cell.data(), off.data(), eta.data(), p.data(), Q.data(), pv.data());
    orc_particles_init(N, 5, 1, 1, 1.2, np / 2, cell.data() + np, off.data() + np, eta.data() + np / 2,
                       p.data() + 3 * np / 2, Q.data() + 8 * np / 2, pv.data() + 3 * np / 2);
    for (int i = 0; i < np; i++) species[i] = i < np / 2 ? 0 : 1;
    double mass[2] = {0.4, 0.0}, series[8] = {0};
    int nform[2] = {1, 1};
    std::vector<double> U0(U), phi0(phi);
    for (int n = 6; n < 10; n++) {
        U0 = U;
        phi0 = phi;
        orc_field_step(N, n, 0.125, U.data(), E.data(), phi.data(), pi.data(), F.data());
        orc_particle_step(N, n, 0.125, U0.data(), phi0.data(), F.data(), np, cell.data(), off.data(), eta.data(),
                          p.data(), Q.data(), pv.data(), species.data(), 2, mass, nform, series);
    }
    // the whole coupled run
    const int steps = 4, kinds[2] = {0, 1}, nps[2] = {10, 6};
    double masses[2] = {0.4, 0.0}, p0s[2] = {0.2, 1.0};
    int nforms[2] = {2, 1};
    std::vector<int> c2(2 * 16), s2(16);
    std::vector<double> o2(2 * 16), e2(16), pp2(3 * 16), q2(8 * 16), pv2(3 * 16), ser(steps * 2 * 4);
    if (orc_run(N, 0.5, 0.04, 1, 23, 0.125, steps, 2, kinds, masses, p0s, nforms, nps, U.data(), E.data(),
                phi.data(), pi.data(), c2.data(), o2.data(), e2.data(), pp2.data(), q2.data(), pv2.data(), s2.data(),
                ser.data()) != 0)
        return 7;
    for (double v : ser)
        if (!std::isfinite(v)) return 8;
    std::printf("oracle sanitizer drive ok\n");
    return 0;
}
