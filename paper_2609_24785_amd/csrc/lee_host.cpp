// Host-side set-up of one instance, FP64: fluid mask and row intervals, ghost
// points, boundary points, elliptical clouds, least-squares read-out by
// Householder QR, 1-D Lagrange / Birkhoff composition, ADE coefficients.
//
// Compiled without floating-point contraction so that every predicate
// (mask, ellipse, half-plane) is the same correctly rounded FP64 expression
// as written; ghost and cloud lists are therefore reproducible bit-for-bit by
// any implementation that evaluates the same expressions.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>

#include "lee_internal.h"

namespace lee {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

lee_status fail(lee_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

}  // namespace lee

extern "C" const char *lee_last_error(void) { return lee::g_err.c_str(); }

namespace lee {

// Wall coupling limits with the selective filter on.  The Neumann ghost value
// carries h du_n/dt = h s Y(s) p_BP, which feeds the boundary pressure back
// with gain h |s Y(s)|: spectral radii of the step map on coarse cylinders
// stay at the rigid wall's while the high-frequency gain h lim_{s->oo} s Y(s)
// is at most 1.5 (growth from about 1.6) and the peak gain
// h max_w |i w Y(i w)| at most 3.5 (growth from about 4, resonances at
// w h = 0.5 to 2).  (Without the filter the scheme carries the wall's
// tangency growth anyway and nothing is rejected.)
static constexpr double COUPLING_MAX = 1.5;
static constexpr double PEAK_MAX = 3.0;

// max over w > 0 of |i w Y(i w)| for the mass-spring-damper wall: with
// u = w^2, |i w Y|^2 = u^2 / ((K - M u)^2 + R^2 u); setting its derivative in
// u to zero gives u* = 2 K^2 / (2 K M - R^2) when 2 K M > R^2; otherwise the
// gain rises to its limit 1/M as w grows.
static double msd_peak_gain(double R, double M, double K)
{
    const double den = 2.0 * K * M - R * R;
    if (den <= 0.0) return 1.0 / M;
    const double u = 2.0 * K * K / den;
    return u / std::sqrt((K - M * u) * (K - M * u) + R * R * u);
}

// The same for a multi-pole admittance (eq. Yrational without direct term):
// the largest of its limit `lim` and of |i w Y(i w)| at the pole moduli and
// imaginary parts and at 2401 log-spaced frequencies from 1e-4 to 1e8.
static double poles_peak_gain(const lee_impedance *z, double lim)
{
    auto gain = [&](double w) {
        const std::complex<double> s(0.0, w);
        std::complex<double> y(0.0, 0.0);
        for (int i = 0; i < z->n_real; ++i) y += z->real_res[i] / (s - z->real_pole[i]);
        for (int i = 0; i < z->n_pair; ++i) {
            const std::complex<double> q(z->pair_B[i], z->pair_C[i]), p(z->pair_alpha[i], z->pair_beta[i]);
            y += q / (s - p) + std::conj(q) / (s - std::conj(p));
        }
        return std::abs(s * y);
    };
    double best = std::fabs(lim);
    for (int e = 0; e <= 2400; ++e) best = std::max(best, gain(std::pow(10.0, -4.0 + e / 200.0)));
    for (int i = 0; i < z->n_real; ++i) best = std::max(best, gain(std::fabs(z->real_pole[i])));
    for (int i = 0; i < z->n_pair; ++i) {
        best = std::max(best, gain(std::abs(std::complex<double>(z->pair_alpha[i], z->pair_beta[i]))));
        best = std::max(best, gain(std::fabs(z->pair_beta[i])));
    }
    return best;
}

static double node_x(const lee_case_desc &d, long i) { return d.x0 + (double)i * d.h; }
static double node_y(const lee_case_desc &d, long j) { return d.y0 + (double)j * d.h; }

// Level set, positive in the fluid (Sec. 3.1).
static double level(const lee_case_desc &d, double x, double y)
{
    if (d.wall_kind == LEE_WALL_LINE) return (x - d.wall_cx) * d.wall_nx + (y - d.wall_cy) * d.wall_ny;
    if (d.wall_kind == LEE_WALL_CIRCLE) {
        double dx = x - d.wall_cx, dy = y - d.wall_cy;
        return dx * dx + dy * dy - d.wall_rc * d.wall_rc;
    }
    return 1.0;
}

lee_status host_setup(const lee_case_desc *dp, Host *H)
{
    if (!dp) return fail(LEE_E_ARG, "null description");
    const lee_case_desc &d = *dp;
    if (d.nx < 16 || d.ny < 16 || d.nx > (1 << 15) || d.ny > (1 << 15))
        return fail(LEE_E_ARG, "nx, ny must lie in [16, 32768]");
    if (!(d.h > 0.0) || !(d.cfl > 0.0) || d.cfl > 1.0) return fail(LEE_E_ARG, "h > 0 and 0 < cfl <= 1 required");
    if (d.stencil_half != 3 && d.stencil_half != 5) return fail(LEE_E_ARG, "stencil_half must be 3 or 5");
    if (d.filter_sigma < 0.0 || d.filter_sigma > 0.5) return fail(LEE_E_ARG, "filter_sigma in [0, 0.5]");
    if (d.filter_explicit != 0 && d.filter_explicit != 1) return fail(LEE_E_ARG, "filter_explicit must be 0 or 1");
    if (d.filter_sigma > 0.0 && d.stencil_half != 5)
        return fail(LEE_E_ARG, "the 11-point filter needs stencil_half = 5 (five ghost layers)");
    if (d.sponge_cells < 0 || d.sponge_sigma < 0.0) return fail(LEE_E_ARG, "negative sponge");
    if (d.precision != LEE_F32 && d.precision != LEE_F64) return fail(LEE_E_ARG, "precision");
    if (d.wall_kind < LEE_WALL_NONE || d.wall_kind > LEE_WALL_CIRCLE) return fail(LEE_E_ARG, "wall_kind");
    if (d.wall_kind == LEE_WALL_LINE) {
        double n2 = d.wall_nx * d.wall_nx + d.wall_ny * d.wall_ny;
        if (std::fabs(n2 - 1.0) > 1e-12) return fail(LEE_E_ARG, "line normal must be a unit vector");
    }
    if (d.wall_kind == LEE_WALL_CIRCLE && !(d.wall_rc > 0.0)) return fail(LEE_E_ARG, "circle radius");
    if (d.ic_kind < LEE_IC_NONE || d.ic_kind > LEE_IC_PACKET) return fail(LEE_E_ARG, "ic_kind");
    if (d.src_kind != LEE_SRC_NONE && d.src_kind != LEE_SRC_MONOPOLE) return fail(LEE_E_ARG, "src_kind");
    if (d.ic_kind == LEE_IC_PULSE && !(d.ic[3] > 0.0)) return fail(LEE_E_ARG, "pulse half-width");
    if (d.src_kind == LEE_SRC_MONOPOLE && !(d.src[3] > 0.0)) return fail(LEE_E_ARG, "source half-width");

    H->d = d;
    H->dt = d.cfl * d.h;
    H->reach = d.filter_sigma > 0.0 ? std::max(d.stencil_half, 5) : d.stencil_half;
    const int nx = d.nx, ny = d.ny;
    H->fluid.assign((size_t)nx * ny, 0);
    for (int j = 0; j < ny; ++j) {
        double y = node_y(d, j);
        for (int i = 0; i < nx; ++i) H->fluid[(size_t)j * nx + i] = level(d, node_x(d, i), y) > 0.0 ? 1 : 0;
    }
    // row intervals: at most two fluid runs per row
    H->iv.assign((size_t)ny * 4, 0);
    H->fluid_nodes = 0;
    for (int j = 0; j < ny; ++j) {
        const uint8_t *row = &H->fluid[(size_t)j * nx];
        int runs = 0;
        for (int i = 0; i < nx;) {
            if (!row[i]) { ++i; continue; }
            int a = i;
            while (i < nx && row[i]) ++i;
            if (runs >= 2) return fail(LEE_E_GEOMETRY, "more than two fluid intervals in a grid row");
            H->iv[(size_t)j * 4 + 2 * runs] = a;
            H->iv[(size_t)j * 4 + 2 * runs + 1] = i;
            H->fluid_nodes += i - a;
            ++runs;
        }
    }
    // radiation band: the band and everything its stencils read is fluid, and
    // the centre keeps a grid step from every band node
    if (d.radiation != 0) {
        if (d.radiation != 1) return fail(LEE_E_ARG, "radiation must be 0 or 1");
        const int W = d.stencil_half, reach = W + 6;
        if (nx <= 2 * reach || ny <= 2 * reach) return fail(LEE_E_ARG, "radiation condition: grid too small");
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int e = std::min(std::min(i, j), std::min(nx - 1 - i, ny - 1 - j));
                if (e >= reach) continue;
                if (!H->fluid[(size_t)j * nx + i])
                    return fail(LEE_E_ARG, "radiation condition: the wall comes within reach of the outer band");
                if (e < W && std::hypot(node_x(d, i) - d.rad_xc, node_y(d, j) - d.rad_yc) < d.h)
                    return fail(LEE_E_ARG, "radiation condition: centre too close to the outer band");
            }
    }
    // ghost points: solid nodes reached by a fluid node's stencil along x or y
    H->gidx.clear();
    if (d.wall_kind != LEE_WALL_NONE) {
        const int R = H->reach;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                if (H->fluid[(size_t)j * nx + i]) continue;
                bool hit = false;
                for (int k = 1; k <= R && !hit; ++k) {
                    if (i + k < nx && H->fluid[(size_t)j * nx + i + k]) hit = true;
                    if (i - k >= 0 && H->fluid[(size_t)j * nx + i - k]) hit = true;
                    if (j + k < ny && H->fluid[(size_t)(j + k) * nx + i]) hit = true;
                    if (j - k >= 0 && H->fluid[(size_t)(j - k) * nx + i]) hit = true;
                }
                if (hit) H->gidx.push_back(j * nx + i);
            }
    }
    return LEE_OK;
}

// ---------------------------------------------------------------------------
// dense helpers (column-major N x M)

// One-sided Jacobi: singular values of A (copied).
static void jacobi_singular_values(std::vector<double> A, int N, int M, std::vector<double> &sv)
{
    for (int sweep = 0; sweep < 80; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < M - 1; ++p)
            for (int q = p + 1; q < M; ++q) {
                double al = 0, be = 0, ga = 0;
                double *ap = &A[(size_t)p * N], *aq = &A[(size_t)q * N];
                for (int n = 0; n < N; ++n) { al += ap[n] * ap[n]; be += aq[n] * aq[n]; ga += ap[n] * aq[n]; }
                if (std::fabs(ga) <= 1e-15 * std::sqrt(al * be) || ga == 0.0) continue;
                rotated = true;
                double zeta = (be - al) / (2.0 * ga);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int n = 0; n < N; ++n) {
                    double x = ap[n], y = aq[n];
                    ap[n] = c * x - s * y;
                    aq[n] = s * x + c * y;
                }
            }
        if (!rotated) break;
    }
    sv.assign(M, 0.0);
    for (int m = 0; m < M; ++m) {
        double s = 0;
        for (int n = 0; n < N; ++n) s += A[(size_t)m * N + n] * A[(size_t)m * N + n];
        sv[m] = std::sqrt(s);
    }
}

// W (5 x N, row-major) = E V^+ for the column-scaled V by Householder QR.
static void lsq_readout_qr(const std::vector<double> &Vs, const std::vector<double> &cs, int N, int M,
                           const std::vector<double> &E /* 5 x M row-major */, std::vector<double> &W)
{
    std::vector<double> A = Vs;                   // column-major N x M, becomes R + reflectors
    std::vector<double> V((size_t)M * N, 0.0);    // reflector k in V[k*N + k .. N-1]
    std::vector<double> betas(M, 0.0);
    for (int k = 0; k < M; ++k) {
        double *col = &A[(size_t)k * N];
        double nrm = 0;
        for (int n = k; n < N; ++n) nrm += col[n] * col[n];
        nrm = std::sqrt(nrm);
        double alpha = col[k] >= 0 ? -nrm : nrm;
        double *v = &V[(size_t)k * N];
        for (int n = k; n < N; ++n) v[n] = col[n];
        v[k] -= alpha;
        double vv = 0;
        for (int n = k; n < N; ++n) vv += v[n] * v[n];
        double beta = vv > 0 ? 2.0 / vv : 0.0;
        betas[k] = beta;
        for (int c = k; c < M; ++c) {           // A <- H_k A
            double *a = &A[(size_t)c * N];
            double dot = 0;
            for (int n = k; n < N; ++n) dot += v[n] * a[n];
            dot *= beta;
            for (int n = k; n < N; ++n) a[n] -= dot * v[n];
        }
    }
    // G (5 x M) solves G R = E diag(cs)
    std::vector<double> G(5 * (size_t)M, 0.0);
    for (int i = 0; i < 5; ++i)
        for (int c = 0; c < M; ++c) {
            double s = E[(size_t)i * M + c] * cs[c];
            for (int k = 0; k < c; ++k) s -= G[(size_t)i * M + k] * A[(size_t)c * N + k];
            G[(size_t)i * M + c] = s / A[(size_t)c * N + c];
        }
    // W = [G 0] H_{M-1} ... H_0
    W.assign(5 * (size_t)N, 0.0);
    for (int i = 0; i < 5; ++i)
        for (int c = 0; c < M; ++c) W[(size_t)i * N + c] = G[(size_t)i * M + c];
    for (int k = M - 1; k >= 0; --k) {
        const double *v = &V[(size_t)k * N];
        for (int i = 0; i < 5; ++i) {
            double *w = &W[(size_t)i * N];
            double dot = 0;
            for (int n = k; n < N; ++n) dot += w[n] * v[n];
            dot *= betas[k];
            for (int n = k; n < N; ++n) w[n] -= dot * v[n];
        }
    }
}

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int k = 0; k < e; ++k) r *= x;
    return r;
}

// Least-squares read-out at P_0..P_4 with degree fallback; returns the degree
// used (0: no usable fit, W = 0).
static int readout(const std::vector<double> &xp, const std::vector<double> &yp, std::vector<double> &W)
{
    const int N = (int)xp.size();
    for (int k = 4; k >= 1; --k) {
        const int M = (k + 1) * (k + 2) / 2;
        if (N < M) continue;
        std::vector<int> ea, eb;                 // graded monomials x'^a y'^b
        for (int dd = 0; dd <= k; ++dd)
            for (int a = dd; a >= 0; --a) { ea.push_back(a); eb.push_back(dd - a); }
        std::vector<double> V((size_t)N * M), cs(M);
        for (int c = 0; c < M; ++c) {
            double s = 0;
            for (int n = 0; n < N; ++n) {
                double v = ipow(xp[n], ea[c]) * ipow(yp[n], eb[c]);
                V[(size_t)c * N + n] = v;
                s += v * v;
            }
            if (s == 0.0) { cs[c] = 0.0; continue; }
            cs[c] = 1.0 / std::sqrt(s);
        }
        bool zero_col = false;
        for (int c = 0; c < M; ++c) zero_col |= (cs[c] == 0.0);
        if (zero_col) continue;
        for (int c = 0; c < M; ++c)
            for (int n = 0; n < N; ++n) V[(size_t)c * N + n] *= cs[c];
        std::vector<double> sv;
        jacobi_singular_values(V, N, M, sv);
        double smax = *std::max_element(sv.begin(), sv.end());
        double smin = *std::min_element(sv.begin(), sv.end());
        if (!(smin > 1e-10 * smax)) continue;
        std::vector<double> E(5 * (size_t)M, 0.0);
        for (int i = 0; i < 5; ++i)
            for (int c = 0; c < M; ++c) E[(size_t)i * M + c] = eb[c] == 0 ? ipow((double)i, ea[c]) : 0.0;
        lsq_readout_qr(V, cs, N, M, E, W);
        return k;
    }
    W.assign(5 * (size_t)N, 0.0);
    return 0;
}

// l_j(s) on nodes 0..4
static void lagrange5(double s, double L[5])
{
    for (int j = 0; j < 5; ++j) {
        double v = 1.0;
        for (int m = 0; m < 5; ++m)
            if (m != j) v *= (s - m) / (double)(j - m);
        L[j] = v;
    }
}

// mu with Q(s) = mu_0 Q'(0) + sum_{i=1..4} mu_i Q(i) for all quartics
static void birkhoff5(double s, double mu[5])
{
    double A[5][6];
    for (int p = 0; p < 5; ++p) {
        A[p][0] = (p == 1) ? 1.0 : 0.0;
        for (int i = 1; i < 5; ++i) A[p][i] = ipow((double)i, p);
        A[p][5] = ipow(s, p);
    }
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        for (int r = c + 1; r < 5; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
        if (piv != c)
            for (int k = 0; k < 6; ++k) std::swap(A[c][k], A[piv][k]);
        for (int r = 0; r < 5; ++r) {
            if (r == c) continue;
            double f = A[r][c] / A[c][c];
            for (int k = c; k < 6; ++k) A[r][k] -= f * A[c][k];
        }
    }
    for (int c = 0; c < 5; ++c) mu[c] = A[c][5] / A[c][c];
}

static double rk4_abs(std::complex<double> z)
{
    std::complex<double> r = 1.0 + z + z * z / 2.0 + z * z * z / 6.0 + z * z * z * z / 24.0;
    return std::abs(r);
}

lee_status host_build(Host *H, const lee_impedance *z, int degree, lee_ghost_summary *out)
{
    if (H->built) return fail(LEE_E_STATE, "lee_build_ghosts called twice");
    if (degree != 4) return fail(LEE_E_ARG, "degree must be 4 (k = m = 4)");
    if (!z) return fail(LEE_E_ARG, "null impedance");
    const lee_case_desc &d = H->d;
    const int nx = d.nx, ny = d.ny;
    const double h = d.h;

    // ---- ADE coefficients (Sec. 2.5) ----
    H->ade_kind = 0;
    H->ade_ns = 2;
    std::fill(H->ade, H->ade + 4, 0.0);
    std::fill(H->poles, H->poles + 4, 0.0);
    if (z->kind == LEE_Z_MSD) {
        const double R = z->R, M = z->M, K = z->K;
        if (!(R > 0.0 && M > 0.0 && K > 0.0)) return fail(LEE_E_ARG, "M, R, K must be positive");
        const double a = R / (2.0 * M);
        const double disc = a * a - K / M;
        if (std::fabs(disc) <= 1e-9 * (K / M))
            return fail(LEE_E_CRITICAL_DAMPING, "critical damping R = 2 sqrt(K M): double pole");
        std::complex<double> s1, s2;
        if (disc < 0.0) {
            const double b = std::sqrt(-disc);
            s1 = {-a, b};
            s2 = {-a, -b};
            std::complex<double> q1 = s1 / (M * (s1 - s2));   // B1 + i C1
            H->ade_kind = 1;
            H->ade[0] = a;
            H->ade[1] = b;
            H->ade[2] = 2.0 * q1.real();    // u_n = 2 B1 Psi1 - 2 C1 Psi2
            H->ade[3] = -2.0 * q1.imag();
        } else {
            const double sq = std::sqrt(disc);
            const double l1 = -a + sq, l2 = -a - sq;
            s1 = l1;
            s2 = l2;
            H->ade_kind = 2;
            H->ade[0] = l1;
            H->ade[1] = l2;
            H->ade[2] = l1 / (M * (l1 - l2));
            H->ade[3] = l2 / (M * (l2 - l1));
        }
        H->poles[0] = s1.real(); H->poles[1] = s1.imag();
        H->poles[2] = s2.real(); H->poles[3] = s2.imag();
        if (rk4_abs(H->dt * s1) > 1.0 || rk4_abs(H->dt * s2) > 1.0)
            return fail(LEE_E_ADE_STIFF, "an ADE pole lies outside the RK4 stability region at this dt");
        if (H->d.filter_sigma > 0.0 && h / M > COUPLING_MAX)
            return fail(LEE_E_ADE_STIFF, "wall coupling gain h/M > 1.5 with the filter on: the Neumann ghost "
                                         "value feeds p_BP back and the coupled step map grows");
        if (H->d.filter_sigma > 0.0 && h * msd_peak_gain(R, M, K) > PEAK_MAX)
            return fail(LEE_E_ADE_STIFF, "wall peak coupling gain h max |i w Y(i w)| > 3 with the filter on "
                                         "(a lightly damped resonance): the coupled step map grows");
    } else if (z->kind == LEE_Z_POLES) {
        // multi-pole admittance (Sec. 2.3, eqs. Yrational, ADEgeneral, unGeneral):
        // real poles first (one state each), then each pair's two states
        const int nr = z->n_real, npr = z->n_pair;
        if (nr < 0 || npr < 0 || nr + 2 * npr < 1 || nr + 2 * npr > LEE_ADE_MAX_STATES)
            return fail(LEE_E_ARG, "a multi-pole wall needs 1 to 8 auxiliary states");
        std::vector<std::complex<double>> all;
        double gain = 0.0;                         // lim s Y(s) = sum A_k + 2 sum B_k
        int k = 0;
        for (int i = 0; i < nr; ++i, ++k) {
            const double lam = z->real_pole[i], A = z->real_res[i];
            if (!std::isfinite(lam) || !std::isfinite(A)) return fail(LEE_E_ARG, "non-finite pole or residue");
            if (!(lam < 0.0)) return fail(LEE_E_ARG, "a real pole must be negative");
            double *st = H->ade_st[k];
            st[0] = lam; st[1] = 0.0; st[2] = 0.0; st[3] = 1.0; st[4] = A;
            all.emplace_back(lam, 0.0);
            gain += A;
        }
        for (int i = 0; i < npr; ++i, k += 2) {
            const double al = z->pair_alpha[i], be = z->pair_beta[i], B = z->pair_B[i], C = z->pair_C[i];
            if (!std::isfinite(al) || !std::isfinite(be) || !std::isfinite(B) || !std::isfinite(C))
                return fail(LEE_E_ARG, "non-finite pole or residue");
            if (!(al < 0.0) || !(be > 0.0)) return fail(LEE_E_ARG, "a pole pair needs alpha < 0 and beta > 0");
            double *s1 = H->ade_st[k], *s2 = H->ade_st[k + 1];
            // dPsi1 = alpha Psi1 - beta Psi2 + p, dPsi2 = alpha Psi2 + beta Psi1,
            // u_n += 2 B Psi1 - 2 C Psi2
            s1[0] = al; s1[1] = -be; s1[2] = 0.0; s1[3] = 1.0; s1[4] = 2.0 * B;
            s2[0] = al; s2[1] = 0.0; s2[2] = be; s2[3] = 0.0; s2[4] = -2.0 * C;
            all.emplace_back(al, be);
            all.emplace_back(al, -be);
            gain += 2.0 * B;
        }
        H->ade_kind = 3;
        H->ade_ns = k;
        for (int i = 0; i < 2 && i < (int)all.size(); ++i) {
            H->poles[2 * i] = all[i].real();
            H->poles[2 * i + 1] = all[i].imag();
        }
        for (const auto &s : all)
            if (rk4_abs(H->dt * s) > 1.0)
                return fail(LEE_E_ADE_STIFF, "an ADE pole lies outside the RK4 stability region at this dt");
        if (H->d.filter_sigma > 0.0 && h * std::fabs(gain) > COUPLING_MAX)
            return fail(LEE_E_ADE_STIFF, "wall coupling gain h (sum A + 2 sum B) > 1.5 with the filter on: the "
                                         "Neumann ghost value feeds p_BP back and the coupled step map grows");
        if (H->d.filter_sigma > 0.0 && h * poles_peak_gain(z, gain) > PEAK_MAX)
            return fail(LEE_E_ADE_STIFF, "wall peak coupling gain h max |i w Y(i w)| > 3 with the filter on: "
                                         "the coupled step map grows");
    } else if (z->kind != LEE_Z_RIGID) {
        return fail(LEE_E_ARG, "impedance kind");
    }

    // ---- ghosts ----
    const int G = (int)H->gidx.size();
    H->bx.assign(G, 0); H->by.assign(G, 0); H->gnx.assign(G, 0); H->gny.assign(G, 0); H->r.assign(G, 0);
    H->cptr.assign(G + 1, 0);
    H->cidx.clear();
    H->deg.assign(G, 0);
    H->cut.assign(G, 0);
    H->w4.clear();
    H->beta.assign(2 * (size_t)G, 0.0);
    int n_degraded = 0, n_cut = 0;
    double rmin = 1e300, rmax = -1e300, wl1 = 0.0;
    const int WIN = 14;
    const double EA = 9.0, EB = 64.0, EC = 576.0;   // R_t^2, R_n^2, R_n^2 R_t^2 with k = 4
    for (int g = 0; g < G; ++g) {
        const int gi = H->gidx[g] % nx, gj = H->gidx[g] / nx;
        const double xg = node_x(d, gi), yg = node_y(d, gj);
        double bx, by, nxv, nyv, dist;
        if (d.wall_kind == LEE_WALL_LINE) {
            double phi = (xg - d.wall_cx) * d.wall_nx + (yg - d.wall_cy) * d.wall_ny;
            dist = -phi;
            nxv = d.wall_nx;
            nyv = d.wall_ny;
            bx = xg + dist * d.wall_nx;
            by = yg + dist * d.wall_ny;
        } else {
            double dx = xg - d.wall_cx, dy = yg - d.wall_cy;
            double rho = std::sqrt(dx * dx + dy * dy);
            if (rho == 0.0) return fail(LEE_E_GEOMETRY, "a ghost point sits at the circle centre");
            nxv = dx / rho;
            nyv = dy / rho;
            bx = d.wall_cx + d.wall_rc * nxv;
            by = d.wall_cy + d.wall_rc * nyv;
            dist = d.wall_rc - rho;
        }
        const double r = dist / h;
        H->bx[g] = bx; H->by[g] = by; H->gnx[g] = nxv; H->gny[g] = nyv; H->r[g] = r;
        rmin = std::min(rmin, r);
        rmax = std::max(rmax, r);
        // cloud
        std::vector<double> xp, yp;
        std::vector<int32_t> idx;
        bool cut = false;
        for (int jj = gj - WIN; jj <= gj + WIN; ++jj)
            for (int ii = gi - WIN; ii <= gi + WIN; ++ii) {
                const double x = node_x(d, ii), y = node_y(d, jj);
                const double ddx = x - bx, ddy = y - by;
                const double xq = (nxv * ddx + nyv * ddy) / h;
                const double yq = (-nyv * ddx + nxv * ddy) / h;
                const bool inside = EA * xq * xq + EB * yq * yq <= EC;
                if (!inside) continue;
                if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) { cut = true; continue; }
                if (!H->fluid[(size_t)jj * nx + ii]) continue;
                if (d.wall_kind == LEE_WALL_CIRCLE &&
                    !((x - d.wall_cx) * nxv + (y - d.wall_cy) * nyv >= 0.0))
                    continue;
                idx.push_back(jj * nx + ii);
                xp.push_back(xq);
                yp.push_back(yq);
            }
        const int N = (int)idx.size();
        H->cptr[g + 1] = H->cptr[g] + N;
        H->cidx.insert(H->cidx.end(), idx.begin(), idx.end());
        H->cut[g] = cut ? 1 : 0;
        std::vector<double> W;
        int k = 0;
        if (cut) {
            ++n_cut;
            W.assign(5 * (size_t)N, 0.0);
        } else {
            k = readout(xp, yp, W);
        }
        H->deg[g] = (int8_t)k;
        if (k != 4) ++n_degraded;
        double L[5] = {0, 0, 0, 0, 0}, mu[5] = {0, 0, 0, 0, 0};
        if (k > 0) {
            lagrange5(-r, L);
            birkhoff5(-r, mu);
        }
        H->beta[2 * (size_t)g] = L[0];
        H->beta[2 * (size_t)g + 1] = mu[0];
        double l1[4] = {0, 0, 0, 0};
        for (int n = 0; n < N; ++n) {
            double w0 = W[n], wf = 0, wd = 0, wn = 0;
            for (int i = 0; i < 5; ++i) wf += L[i] * W[(size_t)i * N + n];
            for (int i = 1; i < 5; ++i) {
                wd += L[i] * W[(size_t)i * N + n];
                wn += mu[i] * W[(size_t)i * N + n];
            }
            H->w4.push_back(w0); H->w4.push_back(wf); H->w4.push_back(wd); H->w4.push_back(wn);
            l1[0] += std::fabs(w0); l1[1] += std::fabs(wf); l1[2] += std::fabs(wd); l1[3] += std::fabs(wn);
        }
        for (int q = 0; q < 4; ++q) wl1 = std::max(wl1, l1[q]);
    }
    H->built = true;
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->G = G;
        out->nnz = (int64_t)H->cidx.size();
        out->n_degraded = n_degraded;
        out->n_cut = n_cut;
        out->r_min = G ? rmin : 0.0;
        out->r_max = G ? rmax : 0.0;
        out->w_l1_max = wl1;
        out->fluid_nodes = H->fluid_nodes;
        out->ade_kind = H->ade_kind;
        for (int q = 0; q < 4; ++q) out->poles[q] = H->poles[q];
        out->ade_states = H->ade_ns;
    }
    return LEE_OK;
}

lee_status host_probe_stencil(const Host *H, double x, double y, int32_t *i0, int32_t *j0, double w[16])
{
    const lee_case_desc &d = H->d;
    double wx[4], wy[4];
    int o[2];
    for (int ax = 0; ax < 2; ++ax) {
        double f = ((ax == 0 ? x : y) - (ax == 0 ? d.x0 : d.y0)) / d.h;
        int lo = (int)std::floor(f) - 1;
        double t = f - lo;
        double *ww = ax == 0 ? wx : wy;
        for (int a = 0; a < 4; ++a) {
            double v = 1.0;
            for (int m = 0; m < 4; ++m)
                if (m != a) v *= (t - m) / (double)(a - m);
            ww[a] = v;
        }
        o[ax] = lo;
    }
    if (o[0] < 0 || o[1] < 0 || o[0] + 3 >= d.nx || o[1] + 3 >= d.ny)
        return fail(LEE_E_PROBE, "probe stencil leaves the domain");
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a) {
            if (!H->fluid[(size_t)(o[1] + b) * d.nx + o[0] + a])
                return fail(LEE_E_PROBE, "probe stencil touches a non-fluid node");
            w[b * 4 + a] = wy[b] * wx[a];
        }
    *i0 = o[0];
    *j0 = o[1];
    return LEE_OK;
}

}  // namespace lee
