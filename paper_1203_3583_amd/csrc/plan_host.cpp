// Host-side plan arithmetic (see plan_host.h): no HIP calls, no device types.
#include "plan_host.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

namespace asf {
namespace host {

namespace {
thread_local std::string g_err;
constexpr int kQuadNodes = 200;
constexpr size_t kC64 = 8;     // bytes of a complex64 value
}  // namespace

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

const char *last_error() { return g_err.c_str(); }

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int log2i(int v) {
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

int check_params(int64_t n, const asf_params *p) {
    if (!p) return fail(ASF_EINVAL, "params is NULL");
    // slot indices are 32-bit: 4 n_src slots must stay below 2^32
    if (n < 1 || n >= (int64_t(1) << 30)) return fail(ASF_EINVAL, "n_src must be in [1, 2^30 - 1], got %lld", (long long)n);
    const double v[4] = {p->lambda, p->z0, p->p2x, p->p2y};
    const char *names[4] = {"lambda", "z0", "p2x", "p2y"};
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(v[i]) || !(v[i] > 0.0)) return fail(ASF_EINVAL, "%s must be finite and > 0", names[i]);
    if (!std::isfinite(p->tol) || p->tol < 1e-7 || p->tol > 1e-1) return fail(ASF_EINVAL, "tol must be in [1e-7, 1e-1]");
    if (!std::isfinite(p->x0) || !std::isfinite(p->y0)) return fail(ASF_EINVAL, "x0, y0 must be finite");
    if (p->flags & ~(ASF_FFT_MASK | ASF_INCIDENT_NONE)) return fail(ASF_EINVAL, "unknown flag bits 0x%x", p->flags);
    if (!is_pow2(p->mx) || !is_pow2(p->my) || p->mx < 16 || p->my < 16 || p->mx > 8192 || p->my > 8192)
        return fail(ASF_ESIZE, "mx, my must be powers of two in [16, 8192], got %d x %d", p->mx, p->my);
    return ASF_OK;
}

int spread_width(double tol) {
    int w = (int)std::ceil(-std::log10(tol) - 1e-9) + 2;
    if (w < 2) w = 2;
    if (w > 9) w = 9;
    return w;
}

size_t fft_twiddle_entries(int len) {
    // stages with span NS > 1 store 16 NS entries each
    const int log = log2i(len);
    const int r0 = 1 << (log % 4);
    const int n16 = log / 4;
    size_t total = 0;
    for (int s = 0; s < n16; ++s) {
        const int ns = r0 << (4 * s);
        if (ns > 1) total += 16 * (size_t)ns;
    }
    return total;
}

int make_layout(int64_t n, const asf_params *p, Layout &L) {
    int rc = check_params(n, p);
    if (rc) return rc;
    L.n = n;
    L.mx = p->mx;
    L.my = p->my;
    L.nfx = 2 * p->mx;
    L.nfy = 2 * p->my;
    L.w = spread_width(p->tol);
    L.beta = 2.30 * L.w;
    L.tile_x = L.nfx < kTileXMax ? L.nfx : kTileXMax;
    L.tile_y = L.nfy < kTileYMax ? L.nfy : kTileYMax;
    L.ntx = L.nfx / L.tile_x;
    L.nty = L.nfy / L.tile_y;
    L.ntiles = L.ntx * L.nty;
    L.slot_cap = 4 * n;
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.off_status = take(kAlign);
    L.off_status2 = take(kAlign);
    L.off_tile_start = take(sizeof(uint32_t) * (L.ntiles + 1));
    L.off_cursor = take(sizeof(uint32_t) * L.ntiles);
    L.off_cursor2 = take(sizeof(uint32_t) * L.ntiles);
    L.off_slab = take(2 * sizeof(uint32_t) * L.ntiles);
    // records: (cell, perm) in 8-byte words, (frac, phase) in 16-byte words
    L.off_cell = take(8 * (size_t)L.slot_cap);
    L.off_perm = L.off_cell + sizeof(uint32_t);
    L.off_frac = take(16 * (size_t)L.slot_cap);
    L.off_phase = L.off_frac + 8;
    L.off_fine = take(kC64 * (size_t)L.nfx * L.nfy);
    L.off_mid = take(kC64 * (size_t)L.my * L.nfx);
    L.off_dx = take(kC64 * L.mx);
    L.off_dy = take(kC64 * L.my);
    L.off_twx = take(kC64 * fft_twiddle_entries(L.nfx));
    L.off_twy = take(kC64 * fft_twiddle_entries(L.nfy));
    L.off_w16 = take(kC64 * 16);
    // the spreading kernel folds the halo of a tile back in on grids narrower than
    // a tile plus w - 1 cells each side; only wider grids cut crowded tiles
    L.split = L.nfx >= L.tile_x + 2 * (L.w - 1) && L.nfy >= L.tile_y + 2 * (L.w - 1);
    L.off_split = take(sizeof(uint32_t) * L.ntiles);
    L.off_split_meta = take(kAlign);
    L.off_slot_owner = take(sizeof(uint32_t) * kSplitSlotsHost);
    L.off_combine = take(sizeof(uint32_t) * kSplitSlotsHost);
    // two 64-bit integer sums (Re, Im) per cell and slice
    L.off_partial = take(L.split ? 16 * (size_t)kSplitSlotsHost * L.tile_x * L.tile_y : 0);
    L.off_live = take((size_t)L.ntiles + L.ntx);
    L.total = o;
    return ASF_OK;
}

int make_line_layout(int64_t n, const asf_line_params *p, LineLayout &L) {
    if (!p) return fail(ASF_EINVAL, "params is NULL");
    if (n < 1 || n > kLineMaxPoints)
        return fail(ASF_EINVAL, "n_src must be in [1, %d], got %lld", kLineMaxPoints, (long long)n);
    const double v[3] = {p->lambda, p->z0, p->p2};
    const char *names[3] = {"lambda", "z0", "p2"};
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(v[i]) || !(v[i] > 0.0)) return fail(ASF_EINVAL, "%s must be finite and > 0", names[i]);
    if (!std::isfinite(p->x0)) return fail(ASF_EINVAL, "x0 must be finite");
    if (!std::isfinite(p->tol) || p->tol < 1e-7 || p->tol > 1e-1) return fail(ASF_EINVAL, "tol must be in [1e-7, 1e-1]");
    if (p->flags & ~ASF_INCIDENT_NONE) return fail(ASF_EINVAL, "unknown flag bits 0x%x", p->flags);
    if (!is_pow2(p->m) || p->m < 16 || p->m > 8192)
        return fail(ASF_ESIZE, "m must be a power of two in [16, 8192], got %d", p->m);
    L.n = (int)n;
    L.m = p->m;
    L.nf = 2 * p->m;
    L.w = spread_width(p->tol);
    L.beta = 2.30 * L.w;
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.off_status = take(kAlign);
    L.off_first = take(sizeof(uint32_t) * (L.nf + 1));
    L.off_perm = take(sizeof(uint32_t) * L.n);
    L.off_cell = take(sizeof(uint32_t) * L.n);
    L.off_coef = take(kC64 * (size_t)L.n * L.w);
    L.off_tw = take(kC64 * (L.nf / 2));
    L.off_dd = take(kC64 * L.m);
    L.total = o;
    return ASF_OK;
}

// Gauss-Legendre quadrature (Abramowitz and Stegun, Handbook of Mathematical
// Functions, 25.4.29): the nodes are the roots of the Legendre polynomial P_n and
// the weights 2 / ((1 - x^2) P_n'(x)^2).  Each positive root is found by Newton's
// method from the asymptotic estimate cos(pi (4i + 3) / (4n + 2)) of the
// (i+1)-th largest; P_n comes from Bonnet's recurrence
// (k + 1) P_{k+1} = (2k + 1) x P_k - k P_{k-1} and its derivative from
// (x^2 - 1) P_n' = n (x P_n - P_{n-1}).  The negative roots mirror them.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &wq) {
    x.assign(n, 0.0);
    wq.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double t = std::cos(kPi * (4.0 * i + 3.0) / (4.0 * n + 2.0));
        double deriv = 0.0;
        for (int iter = 0; iter < 100; ++iter) {
            double p_prev = 1.0, p_cur = t;   // P_0(t), P_1(t)
            for (int k = 1; k < n; ++k) {
                const double p_next = ((2.0 * k + 1.0) * t * p_cur - k * p_prev) / (k + 1.0);
                p_prev = p_cur;
                p_cur = p_next;
            }
            deriv = n * (t * p_cur - p_prev) / (t * t - 1.0);
            const double step = p_cur / deriv;
            t -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        x[n - 1 - i] = t;
        x[i] = -t;
        wq[i] = wq[n - 1 - i] = 2.0 / ((1.0 - t * t) * deriv * deriv);
    }
}

// Fourier transform of psi(z) = exp(beta (sqrt(1 - (2z/w)^2) - 1)) at mode m of an nf grid:
// int psi(z) exp(-2 pi i m z / nf) dz = (w/2) int_{-1}^{1} es(u) cos(pi m w u / nf) du.
std::vector<double> psi_hat(int nmodes_half, int nf, int w, double beta) {
    std::vector<double> xq, wq;
    gauss_legendre(kQuadNodes, xq, wq);
    std::vector<double> es(kQuadNodes);
    for (int q = 0; q < kQuadNodes; ++q) es[q] = std::exp(beta * (std::sqrt(1.0 - xq[q] * xq[q]) - 1.0));
    std::vector<double> out(nmodes_half + 1);
    for (int m = 0; m <= nmodes_half; ++m) {
        double s = 0.0;
        for (int q = 0; q < kQuadNodes; ++q) s += wq[q] * es[q] * std::cos(kPi * m * w * xq[q] / nf);
        out[m] = 0.5 * w * s;
    }
    return out;
}

// Twiddle tables of the radix-16 Stockham stages of a length-len FFT, in the
// order the kernels read them: for each stage with span ns > 1 (ns = r0 16^s),
// entry (k, g, i) = exp(-2 pi i r k / (16 ns)) with r = g + 4 i, k < ns, g, i < 4.
std::vector<Cf> stage_twiddles(int len) {
    const int log = log2i(len);
    const int r0 = 1 << (log % 4), n16 = log / 4;
    std::vector<Cf> t;
    t.reserve(fft_twiddle_entries(len));
    for (int s = 0; s < n16; ++s) {
        const int ns = r0 << (4 * s);
        if (ns <= 1) continue;
        for (int k = 0; k < ns; ++k)
            for (int g = 0; g < 4; ++g)
                for (int i = 0; i < 4; ++i) {
                    const int r = g + 4 * i;
                    const double a = 2.0 * kPi * (double)(r * k) / (16.0 * ns);
                    t.push_back(Cf{(float)std::cos(a), (float)-std::sin(a)});
                }
    }
    return t;
}

double reduce(double a) { return std::remainder(a, 2.0 * kPi); }

}  // namespace host
}  // namespace asf
