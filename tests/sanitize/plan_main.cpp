// Driver for the host-side plan arithmetic (paper_1203_3583_amd/csrc/plan_host.cpp)
// built with AddressSanitizer and UndefinedBehaviorSanitizer: parameter checks,
// workspace layouts, Gauss-Legendre rules, the kernel's Fourier transform and the
// FFT twiddle tables over every supported size, plus invalid parameters.
// Exit status 0 when every property holds; the sanitizers abort on the first
// memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <limits>
#include <vector>

#include "plan_host.h"

using namespace asf::host;

static int failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

static asf_params params(int mx, int my, double tol) {
    asf_params p{};
    p.lambda = 532e-9;
    p.z0 = 0.2;
    p.p2x = p.p2y = 8e-6;
    p.mx = mx;
    p.my = my;
    p.tol = tol;
    p.flags = 0;
    p.x0 = p.y0 = 0.0;
    return p;
}

int main() {
    // Gauss-Legendre: weights sum to 2, exact for polynomials of degree < 2n, nodes
    // ascending and symmetric in (-1, 1)
    for (int n : {1, 2, 3, 7, 10, 64, 200}) {
        std::vector<double> x, w;
        gauss_legendre(n, x, w);
        double s0 = 0, s2 = 0, se = 0;
        for (int i = 0; i < n; ++i) {
            CHECK(x[i] > -1.0 && x[i] < 1.0 && w[i] > 0.0);
            if (i) CHECK(x[i] > x[i - 1]);
            CHECK(std::fabs(x[i] + x[n - 1 - i]) < 1e-15);
            s0 += w[i];
            s2 += w[i] * x[i] * x[i];
            se += w[i] * std::exp(x[i]);
        }
        CHECK(std::fabs(s0 - 2.0) < 1e-13);
        if (n >= 2) CHECK(std::fabs(s2 - 2.0 / 3.0) < 1e-13);
        if (n >= 10) CHECK(std::fabs(se - (std::exp(1.0) - std::exp(-1.0))) < 1e-13);
    }
    // kernel transform: positive, even in m, decreasing over the kept modes, and at
    // m = 0 the kernel's integral (Simpson's rule on 20001 points as a cross-check)
    for (int w = 2; w <= 9; ++w) {
        const double beta = 2.30 * w;
        for (int nf : {32, 256, 4096, 16384}) {
            const std::vector<double> ph = psi_hat(nf / 4, nf, w, beta);
            CHECK((int)ph.size() == nf / 4 + 1);
            for (size_t m = 1; m < ph.size(); ++m) CHECK(ph[m] > 0.0 && ph[m] < ph[m - 1]);
            const int K = 20000;
            double simpson = 0.0;
            for (int k = 0; k <= K; ++k) {
                const double z = -0.5 * w + w * (double)k / K;
                const double a = 1.0 - (2.0 * z / w) * (2.0 * z / w);
                const double f = std::exp(beta * (std::sqrt(a > 0 ? a : 0) - 1.0));
                simpson += f * (k == 0 || k == K ? 1 : (k % 2 ? 4 : 2));
            }
            simpson *= (double)w / K / 3.0;
            CHECK(std::fabs(ph[0] - simpson) < 1e-6 * simpson);
        }
    }
    // twiddles: the table size the layout reserves, unit modulus
    for (int len = 32; len <= 16384; len *= 2) {
        const std::vector<Cf> t = stage_twiddles(len);
        CHECK(t.size() == fft_twiddle_entries(len));
        for (const Cf &c : t) CHECK(std::fabs(std::hypot((double)c.re, (double)c.im) - 1.0) < 2e-7);
    }
    // layouts over every supported grid and a range of point counts and tolerances
    for (int mx = 16; mx <= 8192; mx *= 2)
        for (int my = 16; my <= 8192; my *= 4)
            for (long long n : {1LL, 37LL, 65536LL, 4194304LL})
                for (double tol : {1e-7, 1e-5, 1e-2, 1e-1}) {
                    asf_params p = params(mx, my, tol);
                    Layout L;
                    CHECK(make_layout(n, &p, L) == ASF_OK);
                    CHECK(L.total % kAlign == 0 && L.w >= 2 && L.w <= 9);
                    CHECK(L.ntx * L.tile_x == L.nfx && L.nty * L.tile_y == L.nfy);
                    const size_t seg[] = {L.off_status, L.off_status2, L.off_tile_start, L.off_cursor,
                                          L.off_cursor2, L.off_slab, L.off_cell, L.off_frac, L.off_fine,
                                          L.off_mid, L.off_dx, L.off_dy, L.off_twx, L.off_twy, L.off_w16};
                    for (size_t i = 1; i < sizeof seg / sizeof seg[0]; ++i) CHECK(seg[i] > seg[i - 1]);
                    for (size_t s : seg) CHECK(s % kAlign == 0);
                    CHECK(L.off_frac - L.off_cell >= 8 * (size_t)L.slot_cap);
                    CHECK(L.off_fine - L.off_frac >= 16 * (size_t)L.slot_cap);
                    CHECK(L.off_mid - L.off_fine >= 8 * (size_t)L.nfx * L.nfy);
                    CHECK(L.total >= L.off_w16 + 128);
                }
    // invalid parameters: the right code, a message, and no layout
    const double bad[] = {0.0, -1.0, std::numeric_limits<double>::infinity(), std::numeric_limits<double>::quiet_NaN()};
    for (double v : bad) {
        for (int which = 0; which < 4; ++which) {
            asf_params p = params(64, 64, 1e-5);
            double *f[] = {&p.lambda, &p.z0, &p.p2x, &p.p2y};
            *f[which] = v;
            Layout L;
            CHECK(make_layout(100, &p, L) == ASF_EINVAL && last_error()[0] != 0);
        }
    }
    {
        Layout L;
        asf_params p = params(64, 64, 1e-5);
        CHECK(make_layout(0, &p, L) == ASF_EINVAL);
        CHECK(make_layout(int64_t(1) << 30, &p, L) == ASF_EINVAL);
        CHECK(make_layout(100, nullptr, L) == ASF_EINVAL);
        p.tol = 1e-9;
        CHECK(make_layout(100, &p, L) == ASF_EINVAL);
        p = params(100, 64, 1e-5);
        CHECK(make_layout(100, &p, L) == ASF_ESIZE);
        p = params(64, 16384, 1e-5);
        CHECK(make_layout(100, &p, L) == ASF_ESIZE);
        p = params(64, 64, 1e-5);
        p.flags = 0x80;
        CHECK(make_layout(100, &p, L) == ASF_EINVAL);
        p = params(64, 64, 1e-5);
        p.x0 = std::numeric_limits<double>::infinity();
        CHECK(make_layout(100, &p, L) == ASF_EINVAL);
    }
    // line layouts
    for (int m = 16; m <= 8192; m *= 2)
        for (int n : {1, 1000, kLineMaxPoints}) {
            asf_line_params q{};
            q.lambda = 633e-9;
            q.z0 = 1.0;
            q.p2 = 10e-6;
            q.x0 = 0.0;
            q.m = m;
            q.tol = 1e-5;
            q.flags = 0;
            LineLayout L;
            CHECK(make_line_layout(n, &q, L) == ASF_OK);
            CHECK(L.total % kAlign == 0 && L.off_dd > L.off_tw && L.off_tw > L.off_coef);
            CHECK(L.off_tw - L.off_coef >= 8 * (size_t)L.n * L.w);
            q.m = m + 1;
            CHECK(make_line_layout(n, &q, L) == ASF_ESIZE);
        }
    {
        asf_line_params q{};
        q.lambda = 633e-9;
        q.z0 = 1.0;
        q.p2 = 10e-6;
        q.m = 64;
        q.tol = 1e-5;
        LineLayout L;
        CHECK(make_line_layout(kLineMaxPoints + 1, &q, L) == ASF_EINVAL);
        CHECK(make_line_layout(0, &q, L) == ASF_EINVAL);
    }
    for (double a : {0.0, 1e6, -3.5e6, 2.3e-3, 1e300})
        CHECK(std::fabs(reduce(a)) <= kPi + 1e-12);
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::puts("plan arithmetic sanitizer driver: ok");
    return 0;
}
