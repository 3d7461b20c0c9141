/*
 * FP64 time stepping of the oracle.  TEST INFRASTRUCTURE ONLY: loaded by the
 * oracle's Python driver through ctypes; never linked into the GPU library.
 *
 * One Runge-Kutta stage follows the six coupling steps of Sec. 3.2 literally,
 * ghost by ghost:
 *   1. least-squares read-out of p, u, v at P_0..P_4 (W from the Python side);
 *      p_BP = p(P_0);
 *   2. ADE derivative dPsi/dt = A Psi^(l-1) + f p_BP (Sec. 2.5 / eq. ADEgeneral;
 *      ns states per ghost, one dense system for every impedance kind);
 *   3. u_n,BP = c.Psi^(l-1) and du_n,BP/dt = c.dPsi/dt (eqs. ADE-un, ADE-dpdn);
 *   4. boundary data in the frame of the immersed-boundary normal n (wall to
 *      fluid): u.n = -u_n,BP (u_n counts positive into the wall) and
 *      dp/dn = +du_n,BP/dt (momentum eq. momentum-normal with the normal
 *      reversed); tangential velocity free;
 *   5. 1-D extrapolation to s = -r (eq. ns-ghost): Dirichlet for u.n, Neumann
 *      for p (Q'(0) = h dp/dn in the reduced coordinate), free for u.t;
 *   6. right-hand side of the LEE (eq. LEE, rho0 = c0 = 1) at every fluid node
 *      with the DRP first derivative (eq. DRP_s), plus the selective-filter
 *      damping term, the outer sponge and the monopole source, and the stage
 *      update q^(l) = q^n + alpha_l dt RHS(q^(l-1)).
 *
 * Filter rows (a reading: the paper has no filter): along each axis a fluid
 * node takes the widest centred filter row whose nodes are all fluid or
 * outside the domain (the zero frame): the 11-point selective filter where
 * five nodes on either side qualify, else the standard centred filter of
 * half-width w (damping function sin^{2w}(k/2)) for the w nodes that do, and
 * none next to the wall.  The filter so never reads a ghost value: the
 * extrapolated values made the damping term feed a wall mode that grew as
 * sigma_d / dt.  The half-widths come per node from the Python side.
 * The auxiliary states follow the same stage update,
 * Psi^(l) = Psi^n + alpha_l dt dPsi/dt.
 *
 * Fields are (ny + 2F) x (nx + 2F) row-major arrays: the domain plus a frame of
 * F = 5 nodes held at zero on every side.
 *
 * Parity: the interior scheme is pinned by the free-field pulse and monopole
 * closed forms, the walls by the image solution, the plane-wave reflection of
 * the impedance and the convergence orders (tests).  The outer sponge is a
 * reading (the paper truncates its domains with radiation conditions instead):
 * its profile sigma(d) = sigma_max ((W - d) / W)^2 is pinned through the
 * right-hand side of a uniform field, which is exactly -sigma(d) away from
 * the frame (tests).
 *
 * Radiation condition (optional; Sec. 2.2 names one-sided stencils at the
 * outer boundary, Sec. 4.1-4.2 the non-reflecting condition of Tam and Webb
 * on it): at the fluid nodes closer than rad_w nodes to an edge of the
 * domain, step 6 uses the far-field form of the LEE for outgoing waves
 * without mean flow, dq/dt = -(dq/dr + q/(2r)) for q = p, u, v, with r and
 * theta measured from a centre inside the domain and d/dr = cos(theta) d/dx
 * + sin(theta) d/dy; the derivatives take 7 nodes inside the domain
 * (central where possible, one-sided next to the edge) and no filter term.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the stepping loops (for timing the oracle at a stated thread
 * count); returns the count now in use. */
int oc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

typedef struct {
    int nx, ny, F, H;
    double h, dt, x0, y0;
    double a[5];            /* DRP a_1..a_H */
    double sigma_d;         /* filter strength, 0 = off */
    int sponge_w;
    double sponge_smax;
    int has_src;
    double src_x, src_y, src_a, src_b, src_omega;
    const unsigned char *fluid; /* ny*nx */
    int G;
    const long long *gidx;      /* G, linear j*nx+i */
    const double *gnx, *gny;    /* G */
    const long long *cptr;      /* G+1 */
    const long long *cidx;      /* nnz, linear */
    const double *W;            /* nnz*5 */
    const double *lag;          /* G*5  Lagrange l_i(-r) */
    const double *bir;          /* G*5  Birkhoff mu_i(-r) */
    int ade_ns;                 /* auxiliary states per ghost (1..8) */
    double ade_A[64];           /* dPsi/dt = A Psi + f p_BP, A row-major ns x ns in an 8 x 8 array */
    double ade_f[8];
    double ade_c[8];            /* u_n,BP = c . Psi */
    int watch_g;                /* ghost whose p_BP and u_n,BP are recorded (-1: none) */
    int rad_w;                  /* radiation band: nodes closer than rad_w to an edge (0 = none) */
    double rad_xc, rad_yc;      /* centre of the radiation condition */
    double rad_c[3];            /* central 7-point first derivative a_1..a_3 */
    double rad_b[3][7];         /* one-sided 7-point first derivative at point m of 0..6 */
    const unsigned char *fw;    /* per node, x then y: index of its filter row in frow */
    double frow[36][11];        /* filter rows: weights of nodes -5..5 */
    int filter_explicit;        /* the filter once per step instead of in the RHS */
} oc_case;

static const double RK_ALPHA[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};
static const double RK_C[4] = {0.0, 0.25, 1.0 / 3.0, 0.5};

static long long pad_index(const oc_case *c, long long lin)
{
    long long i = lin % c->nx, j = lin / c->nx;
    return (j + c->F) * (long long)(c->nx + 2 * c->F) + (i + c->F);
}

/* steps 1-5 for every ghost; writes ghost values into (p, u, v) and the
 * stage value of the auxiliary states into psi_out; when watch is given, the
 * watched ghost's p_BP, u_n,BP and fluid-side u_n go to watch[0..2]
 * (recording only) */
static void fill_ghosts(const oc_case *c, double *p, double *u, double *v,
                        const double *psi_in, const double *psi_n, double *psi_out,
                        double adt, double *watch)
{
    int g;
#pragma omp parallel for schedule(static)
    for (g = 0; g < c->G; ++g) {
        double fp[5] = {0}, fu[5] = {0}, fv[5] = {0}, un[5], ut[5];
        double nx = c->gnx[g], ny = c->gny[g];
        long long e;
        int i;
        /* step 1: least-squares read-out at P_0..P_4 */
        for (e = c->cptr[g]; e < c->cptr[g + 1]; ++e) {
            long long q = pad_index(c, c->cidx[e]);
            for (i = 0; i < 5; ++i) {
                double w = c->W[e * 5 + i];
                fp[i] += w * p[q];
                fu[i] += w * u[q];
                fv[i] += w * v[q];
            }
        }
        for (i = 0; i < 5; ++i) {
            un[i] = nx * fu[i] + ny * fv[i];
            ut[i] = -ny * fu[i] + nx * fv[i];
        }
        double pBP = fp[0];
        /* steps 2-3: ADE derivative, wall velocity and its time derivative */
        const int ns = c->ade_ns;
        const double *sg = psi_in + (long long)ns * g;
        double d[8], U = 0.0, Ud = 0.0;
        for (i = 0; i < ns; ++i) {
            double acc = c->ade_f[i] * pBP;
            int j;
            for (j = 0; j < ns; ++j) acc += c->ade_A[8 * i + j] * sg[j];
            d[i] = acc;
        }
        for (i = 0; i < ns; ++i) {
            U += c->ade_c[i] * sg[i];
            Ud += c->ade_c[i] * d[i];
        }
        /* steps 4-5: boundary data in the IBM frame and 1-D extrapolation */
        const double *L = c->lag + 5 * g, *B = c->bir + 5 * g;
        double pg = B[0] * (c->h * Ud);
        double ung = L[0] * (-U);
        double utg = L[0] * ut[0];
        for (i = 1; i < 5; ++i) {
            pg += B[i] * fp[i];
            ung += L[i] * un[i];
            utg += L[i] * ut[i];
        }
        if (watch && g == c->watch_g) {
            watch[0] = pBP;
            watch[1] = U;
            /* the fluid's own normal velocity at the boundary point: the
             * least-squares read-out of u.n at P_0, unconstrained by the wall
             * datum, counted positive into the wall like U (Sec. 4.3 compares
             * the two) */
            watch[2] = -un[0];
        }
        long long q = pad_index(c, c->gidx[g]);
        p[q] = pg;
        u[q] = nx * ung - ny * utg;
        v[q] = ny * ung + nx * utg;
        for (i = 0; i < ns; ++i)
            psi_out[(long long)ns * g + i] = psi_n[(long long)ns * g + i] + adt * d[i];
    }
}

static double sponge(const oc_case *c, int i, int j)
{
    if (c->sponge_w <= 0) return 0.0;
    int e = i;
    if (j < e) e = j;
    if (c->nx - 1 - i < e) e = c->nx - 1 - i;
    if (c->ny - 1 - j < e) e = c->ny - 1 - j;
    if (e >= c->sponge_w) return 0.0;
    double f = (double)(c->sponge_w - e) / (double)c->sponge_w;
    return c->sponge_smax * f * f;
}

/* First derivative along one axis at a node i of n (stride between
 * neighbours in the padded plane) from the 7 nearest nodes inside the
 * domain: the central 7-point stencil where three nodes lie on either side,
 * else the one-sided set with the node at place m of the seven (m nodes on
 * the near side), mirrored at the far edge. */
static double rad_deriv(const oc_case *c, const double *q, long long at, int i, int n, long long stride)
{
    int lo = i, hi = n - 1 - i, k;
    double s = 0.0;
    if (lo >= 3 && hi >= 3) {
        for (k = 1; k <= 3; ++k) s += c->rad_c[k - 1] * (q[at + k * stride] - q[at - k * stride]);
    } else if (lo < 3) {
        for (k = 0; k < 7; ++k) s += c->rad_b[lo][k] * q[at + (k - lo) * stride];
    } else {
        for (k = 0; k < 7; ++k) s -= c->rad_b[hi][k] * q[at - (k - hi) * stride];
    }
    return s / c->h;
}

/* step 6: RHS at fluid nodes of the stage input (ps, us, vs) and the update */
static void sweep(const oc_case *c, const double *p, const double *u, const double *v,
                  const double *ps, const double *us, const double *vs,
                  double *po, double *uo, double *vo, double adt, double t)
{
    const long long sy = c->nx + 2 * c->F;
    const double amp = c->has_src ? sin(c->src_omega * t) : 0.0;
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < c->ny; ++j) {
        int i, k;
        for (i = 0; i < c->nx; ++i) {
            long long q = (j + c->F) * sy + (i + c->F);
            if (!c->fluid[(long long)j * c->nx + i]) {
                po[q] = 0.0; uo[q] = 0.0; vo[q] = 0.0;
                continue;
            }
            double rp, ru, rv;
            int e = i;
            if (j < e) e = j;
            if (c->nx - 1 - i < e) e = c->nx - 1 - i;
            if (c->ny - 1 - j < e) e = c->ny - 1 - j;
            if (e < c->rad_w) {
                /* radiation condition: (d/dt + d/dr + 1/(2r)) q = 0 for each
                 * of p, u, v, r and theta about (rad_xc, rad_yc) */
                double x = c->x0 + (double)i * c->h - c->rad_xc, y = c->y0 + (double)j * c->h - c->rad_yc;
                double r = sqrt(x * x + y * y), ct = x / r, st = y / r, hr = 0.5 / r;
                rp = -(ct * rad_deriv(c, ps, q, i, c->nx, 1) + st * rad_deriv(c, ps, q, j, c->ny, sy) + hr * ps[q]);
                ru = -(ct * rad_deriv(c, us, q, i, c->nx, 1) + st * rad_deriv(c, us, q, j, c->ny, sy) + hr * us[q]);
                rv = -(ct * rad_deriv(c, vs, q, i, c->nx, 1) + st * rad_deriv(c, vs, q, j, c->ny, sy) + hr * vs[q]);
            } else {
            double dpdx = 0, dudx = 0, dpdy = 0, dvdy = 0;
            for (k = 1; k <= c->H; ++k) {
                dpdx += c->a[k - 1] * (ps[q + k] - ps[q - k]);
                dudx += c->a[k - 1] * (us[q + k] - us[q - k]);
                dpdy += c->a[k - 1] * (ps[q + k * sy] - ps[q - k * sy]);
                dvdy += c->a[k - 1] * (vs[q + k * sy] - vs[q - k * sy]);
            }
            dpdx /= c->h; dudx /= c->h; dpdy /= c->h; dvdy /= c->h;
            rp = -(dudx + dvdy);
            ru = -dpdx;
            rv = -dpdy;
            if (c->sigma_d > 0.0 && !c->filter_explicit) {
                /* selective-filter damping -(sigma_d/dt)(F_x + F_y)q, each
                 * axis with the row of this node's half-width along it */
                const long long lin = (long long)j * c->nx + i;
                const double *wx = c->frow[c->fw[2 * lin]];
                const double *wy = c->frow[c->fw[2 * lin + 1]];
                double fp = 0.0, fu = 0.0, fv = 0.0;
                for (k = -5; k <= 5; ++k) {
                    fp += wx[k + 5] * ps[q + k] + wy[k + 5] * ps[q + k * sy];
                    fu += wx[k + 5] * us[q + k] + wy[k + 5] * us[q + k * sy];
                    fv += wx[k + 5] * vs[q + k] + wy[k + 5] * vs[q + k * sy];
                }
                double s = c->sigma_d / c->dt;
                rp -= s * fp; ru -= s * fu; rv -= s * fv;
            }
            }
            double ss = sponge(c, i, j);
            if (ss != 0.0) {
                rp -= ss * ps[q]; ru -= ss * us[q]; rv -= ss * vs[q];
            }
            if (c->has_src) {
                double x = c->x0 + (double)i * c->h, y = c->y0 + (double)j * c->h;
                double r2 = (x - c->src_x) * (x - c->src_x) + (y - c->src_y) * (y - c->src_y);
                rp += c->src_a * exp(-c->src_b * r2) * amp;
            }
            po[q] = p[q] + adt * rp;
            uo[q] = u[q] + adt * ru;
            vo[q] = v[q] + adt * rv;
        }
    }
}

/*
 * The explicit form of the filter (the alternative to the damping term in
 * the right-hand side): after a full step, q <- q - sigma_d (F_x + F_y) q at
 * every fluid node outside the radiation band, each axis with the row of the
 * node's half-width along it (the rows of the damping term), from the step's
 * result; other nodes are left as they are (ghost values are filled again by
 * the next stage).
 */
static void filter_step(const oc_case *c, double *p, double *u, double *v, double *fp, double *fu, double *fv)
{
    const long long sy = c->nx + 2 * c->F;
    int j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < c->ny; ++j) {
        int i, k;
        for (i = 0; i < c->nx; ++i) {
            const long long lin = (long long)j * c->nx + i;
            if (!c->fluid[lin]) continue;
            const long long q = (j + c->F) * sy + (i + c->F);
            int e = i;
            if (j < e) e = j;
            if (c->nx - 1 - i < e) e = c->nx - 1 - i;
            if (c->ny - 1 - j < e) e = c->ny - 1 - j;
            if (e < c->rad_w) {                  /* the radiation band has no filter */
                fp[q] = p[q]; fu[q] = u[q]; fv[q] = v[q];
                continue;
            }
            const double *wx = c->frow[c->fw[2 * lin]];
            const double *wy = c->frow[c->fw[2 * lin + 1]];
            double a = 0.0, b = 0.0, d = 0.0;
            for (k = -5; k <= 5; ++k) {
                a += wx[k + 5] * p[q + k] + wy[k + 5] * p[q + k * sy];
                b += wx[k + 5] * u[q + k] + wy[k + 5] * u[q + k * sy];
                d += wx[k + 5] * v[q + k] + wy[k + 5] * v[q + k * sy];
            }
            fp[q] = p[q] - c->sigma_d * a;
            fu[q] = u[q] - c->sigma_d * b;
            fv[q] = v[q] - c->sigma_d * d;
        }
    }
#pragma omp parallel for schedule(static)
    for (j = 0; j < c->ny; ++j) {
        int i;
        for (i = 0; i < c->nx; ++i) {
            const long long lin = (long long)j * c->nx + i;
            if (!c->fluid[lin]) continue;
            const long long q = (j + c->F) * sy + (i + c->F);
            p[q] = fp[q];
            u[q] = fu[q];
            v[q] = fv[q];
        }
    }
}

/*
 * Advance nsteps full steps from step counter step0.  After every step the
 * probes are sampled from q^{n+1}: trace[(s*np + k)*3 + {0,1,2}] = p, u, v at
 * probe k, with 4x4 interpolation weights probe_w[k*16 + b*4 + a] applied to
 * node (probe_ij[2k] + a, probe_ij[2k+1] + b).  watch (3 per step, may be
 * NULL) receives the watched ghost's p_BP, u_n,BP of the ADE and u_n at the
 * boundary point read out of the fluid, all of the step's first stage.
 */
int oc_run(const oc_case *c, double *p, double *u, double *v, double *psi,
           long long step0, int nsteps, int np, const long long *probe_ij,
           const double *probe_w, double *trace, double *watch)
{
    const long long sy = c->nx + 2 * c->F;
    const long long n = sy * (long long)(c->ny + 2 * c->F);
    double *buf = (double *)calloc((size_t)(6 * n), sizeof(double));
    const long long npsi = (long long)c->ade_ns * (c->G > 0 ? c->G : 1);
    double *psb = (double *)calloc((size_t)(2 * npsi), sizeof(double));
    if (!buf || !psb) { free(buf); free(psb); return -1; }
    double *S[3] = {buf, buf + n, buf + 2 * n};      /* stage value q^(l-1) */
    double *T[3] = {buf + 3 * n, buf + 4 * n, buf + 5 * n}; /* stage output */
    double *psS = psb, *psT = psb + npsi;
    int s, l, k;
    for (s = 0; s < nsteps; ++s) {
        for (l = 0; l < 4; ++l) {
            double *ps = l == 0 ? p : S[0], *us = l == 0 ? u : S[1], *vs = l == 0 ? v : S[2];
            const double *psi_in = l == 0 ? psi : psS;
            double t = ((double)(step0 + s) + RK_C[l]) * c->dt;
            const double adt = RK_ALPHA[l] * c->dt;
            fill_ghosts(c, ps, us, vs, psi_in, psi, psT, adt, (watch && l == 0) ? watch + 3 * s : NULL);
            sweep(c, p, u, v, ps, us, vs, T[0], T[1], T[2], adt, t);
            for (k = 0; k < 3; ++k) { double *x = S[k]; S[k] = T[k]; T[k] = x; }
            { double *x = psS; psS = psT; psT = x; }
        }
        memcpy(p, S[0], (size_t)n * sizeof(double));
        memcpy(u, S[1], (size_t)n * sizeof(double));
        memcpy(v, S[2], (size_t)n * sizeof(double));
        if (c->filter_explicit && c->sigma_d > 0.0) filter_step(c, p, u, v, T[0], T[1], T[2]);
        if (c->G > 0) memcpy(psi, psS, (size_t)c->ade_ns * c->G * sizeof(double));
        for (k = 0; k < np; ++k) {
            double acc[3] = {0, 0, 0};
            int a, b;
            for (b = 0; b < 4; ++b)
                for (a = 0; a < 4; ++a) {
                    long long lin = (probe_ij[2 * k + 1] + b) * (long long)c->nx + probe_ij[2 * k] + a;
                    long long q = pad_index(c, lin);
                    double w = probe_w[k * 16 + b * 4 + a];
                    acc[0] += w * p[q]; acc[1] += w * u[q]; acc[2] += w * v[q];
                }
            trace[((long long)s * np + k) * 3 + 0] = acc[0];
            trace[((long long)s * np + k) * 3 + 1] = acc[1];
            trace[((long long)s * np + k) * 3 + 2] = acc[2];
        }
    }
    free(buf);
    free(psb);
    return 0;
}

/*
 * The semi-discrete operator at a state (the spectral analysis of the
 * abstract): with the ghosts filled from (p, u, v) and psi as every stage
 * fills them, (rp, ru, rv) receive the right-hand side of step 6 at the
 * fluid nodes (zero elsewhere) and rpsi the auxiliary states' derivative
 * dPsi/dt, at time t (the source, if any, at that time).  Each is the stage
 * update with q^n = 0 and a step of 1, so it is the same arithmetic as a
 * stage.  Arrays are (ny + 2F) x (nx + 2F); the inputs are not modified.
 */
int oc_rhs(const oc_case *c, const double *p, const double *u, const double *v, const double *psi, double t,
           double *rp, double *ru, double *rv, double *rpsi)
{
    const long long sy = c->nx + 2 * c->F;
    const long long n = sy * (long long)(c->ny + 2 * c->F);
    const long long npsi = (long long)c->ade_ns * (c->G > 0 ? c->G : 1);
    double *buf = (double *)calloc((size_t)(4 * n), sizeof(double));
    double *z = (double *)calloc((size_t)npsi, sizeof(double));
    if (!buf || !z) { free(buf); free(z); return -1; }
    double *ps = buf, *us = buf + n, *vs = buf + 2 * n, *zero = buf + 3 * n;
    memcpy(ps, p, (size_t)n * sizeof(double));
    memcpy(us, u, (size_t)n * sizeof(double));
    memcpy(vs, v, (size_t)n * sizeof(double));
    fill_ghosts(c, ps, us, vs, psi, z, rpsi, 1.0, NULL);
    sweep(c, zero, zero, zero, ps, us, vs, rp, ru, rv, 1.0, t);
    free(buf);
    free(z);
    return 0;
}
