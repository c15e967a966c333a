/*
 * Plain, slow FP64 CPU oracle for the explicit energy-conserving particle-in-cell step of
 * Ricketson & Hu, "An explicit, energy-conserving particle-in-cell scheme".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent check of the GPU library: only
 * the test suite, the package smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or constant with the GPU path.
 *
 * Everything is a direct transcription of the paper's definitions in one spatial
 * dimension, periodic in x on [0, L) with nodes x_i = i h, h = L / N_g:
 *   - shape functions are the cardinal B-splines of section 2.2 (degree 1 is the tent
 *     S(z) = max(0, 1 - |z|/h); degree 2 is the next member of the family), evaluated
 *     at every node that can lie in the support;
 *   - deposit  j_i = (1/h) sum_p w_p v_p S(x_i - x_p)       (section 2.2),
 *     gather   E_p = sum_i E_i S(x_p - x_i)                 (section 2.2);
 *   - ESEC2: the corrected scheme, eq. (good_translation) with (doublestardef);
 *   - ESEC1: the first scheme, eq. (naivetranslation) + eq. (PICmodification) with the
 *     closed-form root eq. (opt_solution);
 *   - EMEC(LI): eq. (EMbasic), Crank-Nicolson Maxwell on a staggered 1D grid;
 *   - EMEC(PSATD): eq. (EM_PSATD), the field update solved exactly in time per Fourier mode
 *     (eq. (PSATDformula) and its time average) with spectral staggered curls;
 *   - EMEC(LF): eq. (EMleapfrog), the Yee leapfrog: B lives at half steps (the state holds
 *     E^n and B^{n-1/2}) and the magnetic energy is the non-standard
 *     W_B^n = c^2/2 h sum B^{n+1/2} . B^{n-1/2} of section 4.1;
 *   - exact charge conservation (section 3.5, ocfg.cc = 1; ESEC2/ESEC1, electrostatic,
 *     tent shapes): E_x and the current on the half nodes, the charge density on the nodes
 *     with the quadratic B-spline, and each particle's path split at the tent's kinks;
 *   - the fallback Gamma := 1 when the root is imaginary (section 3.2), counted;
 *   - total energy of section 5.1.
 * The electrostatic Ampere update is E <- E - dt (j - mean j): in 1D, E = -d(phi)/dx
 * (section 3.2) makes the mean of E zero, so only the mean-free part of j drives E.
 * Sums over particles run in particle index order; energy sums are compensated.
 * No loop is blocked, fused or reordered beyond what the equations say.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nv;          /* 1 (1D-1V) or 3 (1D-3V)                                  */
    int32_t scheme;      /* 0 ESEC2, 1 ESEC1, 2 EMEC(LI), 4 EMEC(PSATD), 5 EMEC(LF)  */
    int32_t order;       /* B-spline degree: 1 or 2                                  */
    int32_t n_cells;     /* N_g                                                      */
    int64_t n_particles; /* N_p                                                      */
    double length;       /* L                                                        */
    double dt;
    double c;            /* speed of light in thermal-speed units (EM only)          */
    double b_ext[3];     /* uniform imposed magnetic field                           */
    int32_t cc;          /* 1: exact charge conservation (section 3.5), see below    */
    int32_t pad;
} ocfg;

typedef struct {
    double kinetic, field_e, field_b, total, max_gamma_dev;
    int64_t fallbacks;
    int32_t nonfinite;
    int32_t pad;
} odiag;

/* ---------------------------------------------------------------- shape functions */

/* Cardinal B-spline of degree `order` in units of h, centred at 0 (section 2.2). */
static double bspline(int order, double t)
{
    t = fabs(t);
    if (order == 1)
        return t < 1.0 ? 1.0 - t : 0.0;
    /* degree 2: 3/4 - t^2 on |t| < 1/2, (3/2 - |t|)^2 / 2 on 1/2 <= |t| < 3/2 */
    if (t < 0.5)
        return 0.75 - t * t;
    if (t < 1.5)
        return 0.5 * (1.5 - t) * (1.5 - t);
    return 0.0;
}

static int64_t pmod(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

/* Nodes whose shape value at position xi (in units of h, grid offset `shift`) may be
 * non-zero: j = floor(xi) - 1 .. floor(xi) + 2 covers support radius <= 3/2. */
static int stencil(int order, double pos, double h, double shift, int ng, int64_t *idx,
                   double *wt)
{
    double xi = pos / h - shift;
    int64_t j0 = (int64_t)floor(xi);
    int n = 0;
    for (int64_t j = j0 - 1; j <= j0 + 2; ++j) {
        double s = bspline(order, (double)j - xi);
        if (s != 0.0) {
            idx[n] = pmod(j, ng);
            wt[n] = s;
            ++n;
        }
    }
    return n;
}

int oracle_stencil(int order, double pos, double h, double shift, int ng, int64_t *idx,
                   double *wt)
{
    return stencil(order, pos, h, shift, ng, idx, wt);
}

/* j_i = (1/h) sum_p q_p S(x_i - x_p);  q_p = w_p u_p.  out is zeroed first. */
void oracle_deposit(int order, int64_t np, const double *x, const double *w,
                    const double *u, int ng, double h, double shift, double *out)
{
    int64_t idx[4];
    double wt[4];
    memset(out, 0, sizeof(double) * (size_t)ng);
    for (int64_t p = 0; p < np; ++p) {
        int n = stencil(order, x[p], h, shift, ng, idx, wt);
        for (int k = 0; k < n; ++k)
            out[idx[k]] += w[p] * u[p] * wt[k] / h;
    }
}

/* E_p = sum_i E_i S(x_p - x_i) */
void oracle_gather(int order, int64_t np, const double *x, const double *field, int ng,
                   double h, double shift, double *out)
{
    int64_t idx[4];
    double wt[4];
    for (int64_t p = 0; p < np; ++p) {
        int n = stencil(order, x[p], h, shift, ng, idx, wt);
        double acc = 0.0;
        for (int k = 0; k < n; ++k)
            acc += field[idx[k]] * wt[k];
        out[p] = acc;
    }
}

/* ------------------------------------------------------------------- small helpers */

typedef struct { double s, c; } nsum;   /* Neumaier compensated sum */

static void nadd(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double wrap(double x, double L)
{
    x = x - L * floor(x / L);
    if (x < 0.0)
        x += L;
    if (x >= L)
        x = 0.0;
    return x;
}

static double mean(const double *a, int n)
{
    nsum s = {0.0, 0.0};
    for (int i = 0; i < n; ++i)
        nadd(&s, a[i]);
    return (s.s + s.c) / n;
}

/* ----------------------------------------------------------- initial Gauss solve */

/* dE/dx = rho - 1 solved spectrally on the nodes (Poisson form, section 2.1): with
 * DFT coefficients rho_m, E_m = rho_m / (i k_m), k_m = 2 pi m / L for 0 < |m| < N/2;
 * the mean mode and (even N) the Nyquist mode of E are zero.  The map rho -> E is
 * linear (the constant background only enters the mean mode). */
void oracle_gauss_rho(int ng, double L, const double *rho, double *E)
{
    double *ere = (double *)calloc((size_t)ng, sizeof(double));
    double *eim = (double *)calloc((size_t)ng, sizeof(double));
    for (int m = 1; m < ng; ++m) {
        if (2 * m == ng)
            continue;                               /* Nyquist mode stays zero */
        int ms = m <= ng / 2 ? m : m - ng;          /* signed mode number */
        double re = 0.0, im = 0.0;                  /* rho_hat_m */
        for (int l = 0; l < ng; ++l) {
            double th = 2.0 * M_PI * (double)(((int64_t)m * l) % ng) / ng;
            re += rho[l] * cos(th);
            im -= rho[l] * sin(th);
        }
        double k = 2.0 * M_PI * ms / L;
        ere[m] = im / k;                            /* rho_hat / (i k) */
        eim[m] = -re / k;
    }
    for (int i = 0; i < ng; ++i) {
        double acc = 0.0;
        for (int m = 1; m < ng; ++m) {
            double th = 2.0 * M_PI * (double)(((int64_t)m * i) % ng) / ng;
            acc += ere[m] * cos(th) - eim[m] * sin(th);
        }
        E[i] = acc / ng;
    }
    free(ere);
    free(eim);
}

void oracle_gauss(int order, int64_t np, const double *x, const double *w, int ng,
                  double L, double *E)
{
    double h = L / ng;
    double *rho = (double *)malloc(sizeof(double) * (size_t)ng);
    double *ones = (double *)malloc(sizeof(double) * (size_t)np);
    for (int64_t p = 0; p < np; ++p)
        ones[p] = 1.0;
    oracle_deposit(order, np, x, w, ones, ng, h, 0.0, rho);
    oracle_gauss_rho(ng, L, rho, E);
    free(ones);
    free(rho);
}

/* ------------------------------------------ exact charge conservation (section 3.5) */

/* Section 3.5 asks for a shape pair (S, S') with
 *   S'(x_i - x^{n+1}) - S'(x_i - x^n) = -(x^{n+1} - x^n) . grad_h S(x_i - x^{n+1/2})
 * (eq. (detbal)), so that rho^n_i = (1/h) sum_p w_p S'(x_i - x_p^n) and the centred current
 * satisfy the discrete continuity equation (eq. (discCont)).  In 1D with second-order
 * differences the pair is S = the tent (degree 1) and S' = the quadratic B-spline (degree 2):
 * the derivative of the quadratic B-spline centred at a node is the difference of the two
 * tents centred at the neighbouring half nodes, divided by h.  So here the current (and E_x,
 * which Ampere's law updates from it) lives on the half nodes x_{i+1/2} = (i + 1/2) h with
 * the tent S, and the divergence of a half-node field at node i is (f_{i+1/2} - f_{i-1/2})/h.
 * Eq. (detbal) needs S' quadratic along the particle's path, i.e. S linear there: the
 * path [x^n, x^{n+1}] is cut where S has its kinks (at the half nodes), and on each piece
 * [a, b] the tent's time average is its value at the piece's midpoint.  The piece carries
 * the fraction (b - a)/(x^{n+1} - x^n) of the particle's current w v*.  Coordinates below
 * are u = x / h - 1/2, in which the half nodes are the integers and the tent centred at
 * half node i is max(0, 1 - |u - i|). */

/* Tent weights at the half nodes around u: (i0, 1 - d) and (i0 + 1, d), d = u - floor(u). */
static void tent_u(double u, int ng, int64_t *idx, double *wt)
{
    double f = floor(u);
    double d = u - f;
    idx[0] = pmod((int64_t)f, ng);
    idx[1] = pmod((int64_t)f + 1, ng);
    wt[0] = 1.0 - d;
    wt[1] = d;
}

/* The pieces of the path from x0 to x1 (unwrapped): for each, call visit(mid_u, frac). */
typedef void (*piece_fn)(double mid_u, double frac, void *ctx);

static void cc_pieces(double x0, double x1, double h, piece_fn visit, void *ctx)
{
    double ua = x0 / h - 0.5, ub = x1 / h - 0.5;
    double lo = ua < ub ? ua : ub, hi = ua < ub ? ub : ua, len = hi - lo;
    if (!(len > 0.0) || !isfinite(len)) {          /* no motion (or no finite path) */
        visit(0.5 * (ua + ub), 1.0, ctx);
        return;
    }
    double s = lo;
    for (;;) {
        double e = floor(s) + 1.0;                  /* next kink after s */
        if (e > hi)
            e = hi;
        visit(0.5 * (s + e), (e - s) / len, ctx);
        if (e >= hi)
            break;
        s = e;
    }
}

typedef struct {
    int ng;
    double q, scale;      /* deposit: q = w u / h */
    double *out;          /* deposit target or NULL */
    const double *field;  /* gather source or NULL */
    double acc;
} piece_ctx;

static void piece_visit(double mid_u, double frac, void *vctx)
{
    piece_ctx *c = (piece_ctx *)vctx;
    int64_t idx[2];
    double wt[2];
    tent_u(mid_u, c->ng, idx, wt);
    for (int k = 0; k < 2; ++k) {
        if (c->out)
            c->out[idx[k]] += c->q * frac * wt[k];
        if (c->field)
            c->acc += frac * wt[k] * c->field[idx[k]];
    }
}

/* j_{i+1/2} = (1/h) sum_p w_p u_p sum_pieces frac S(x_{i+1/2} - mid), paths x0 -> x1. */
void oracle_deposit_cc(int64_t np, const double *x0, const double *x1, const double *w,
                       const double *u, int ng, double h, double *out)
{
    memset(out, 0, sizeof(double) * (size_t)ng);
    for (int64_t p = 0; p < np; ++p) {
        piece_ctx c = {ng, w[p] * u[p] / h, 1.0, out, NULL, 0.0};
        cc_pieces(x0[p], x1[p], h, piece_visit, &c);
    }
}

/* E_p = sum_pieces frac sum_i E_{i+1/2} S(x_{i+1/2} - mid), paths x0 -> x1. */
void oracle_gather_cc(int64_t np, const double *x0, const double *x1, const double *field,
                      int ng, double h, double *out)
{
    for (int64_t p = 0; p < np; ++p) {
        piece_ctx c = {ng, 0.0, 1.0, NULL, field, 0.0};
        cc_pieces(x0[p], x1[p], h, piece_visit, &c);
        out[p] = c.acc;
    }
}

/* Charge density on the nodes with the quadratic B-spline (the S' of the pair above). */
void oracle_rho_cc(int64_t np, const double *x, const double *w, int ng, double h, double *rho)
{
    double *ones = (double *)malloc(sizeof(double) * (size_t)np);
    for (int64_t p = 0; p < np; ++p)
        ones[p] = 1.0;
    oracle_deposit(2, np, x, w, ones, ng, h, 0.0, rho);
    free(ones);
}

/* Gauss' law on the half-node E: (E_{i+1/2} - E_{i-1/2}) / h = rho_i - mean(rho), E with
 * zero mean (E = -d(phi)/dx); E[i] holds E_{i+1/2}. */
void oracle_gauss_cc(int64_t np, const double *x, const double *w, int ng, double L, double *E)
{
    double h = L / ng;
    double *rho = (double *)malloc(sizeof(double) * (size_t)ng);
    oracle_rho_cc(np, x, w, ng, h, rho);
    double m = mean(rho, ng);
    E[0] = 0.0;
    for (int i = 1; i < ng; ++i)
        E[i] = E[i - 1] + h * (rho[i] - m);
    double me = mean(E, ng);
    for (int i = 0; i < ng; ++i)
        E[i] -= me;
    free(rho);
}

/* -------------------------------------------- Crank-Nicolson circulant solve (EM) */

/* Solve (I - s L_h) y = r with L_h the periodic 3-point Laplacian (f_{i+1} - 2 f_i +
 * f_{i-1}) / h^2 and s = (dt/2)^2 c^2: the matrix is circulant, diagonal in the DFT
 * basis with eigenvalues 1 + s (4/h^2) sin^2(pi m / N). */
void oracle_cn_solve(int ng, double h, double s, const double *r, double *y)
{
    double *re = (double *)malloc(sizeof(double) * (size_t)ng);
    double *im = (double *)malloc(sizeof(double) * (size_t)ng);
    for (int m = 0; m < ng; ++m) {
        double a = 0.0, b = 0.0;
        for (int l = 0; l < ng; ++l) {
            double th = 2.0 * M_PI * (double)(((int64_t)m * l) % ng) / ng;
            a += r[l] * cos(th);
            b -= r[l] * sin(th);
        }
        double sn = sin(M_PI * m / ng);
        double lam = 1.0 + s * 4.0 / (h * h) * sn * sn;
        re[m] = a / lam;
        im[m] = b / lam;
    }
    for (int i = 0; i < ng; ++i) {
        double acc = 0.0;
        for (int m = 0; m < ng; ++m) {
            double th = 2.0 * M_PI * (double)(((int64_t)m * i) % ng) / ng;
            acc += re[m] * cos(th) - im[m] * sin(th);
        }
        y[i] = acc / ng;
    }
    free(re);
    free(im);
}

/* ---------------------------------------------- PSATD field solve (EMEC(PSATD) only) */

/* Exact solution over a time tau of the semi-discrete Maxwell system with the current j held
 * fixed (eq. (PSATDconstruction)), by Fourier mode (eq. (PSATDformula)), and its time
 * average over [0, tau] (the formula at the end of section 4.2).  In 1D along x the
 * transverse pairs (E_y, B_z) and (E_z, -B_y) both obey dE/dt = -c^2 D- B - j, dB/dt = -D+ E,
 * with E, j on the nodes x_i and B on the half nodes x_{i+1/2}; the curls are spectral on the
 * staggered grid: D+ (nodes -> half nodes) multiplies mode m by a = i k e^{i k h/2}, D- (half
 * nodes -> nodes) by b = i k e^{-i k h/2}, k = 2 pi m / L with m signed (|m| <= N/2), so that
 * a b = -k^2.  With w = c |k|, C = cos(w tau), S = sin(w tau):
 *   E(tau) = C E - c^2 b S/w B - S/w j,
 *   B(tau) = C B - a S/w E + a (1 - C)/w^2 j,
 *   <E>    = S/(w tau) E - c^2 b (1 - C)/(w^2 tau) B - (1 - C)/(w^2 tau) j,
 * and for k = 0: E - tau j, B, E - tau/2 j.  E_x (no curl): E_x - tau j_x, average
 * E_x - tau/2 j_x.  E, J: [3][ng]; B: [2][ng] (B_y, B_z).  Outputs Eo [3][ng], Bo [2][ng]
 * and Ea [3][ng] (may be NULL).  Direct O(N^2) transforms. */
static void dft(int ng, const double *f, double complex *F)
{
    for (int m = 0; m < ng; ++m) {
        double complex acc = 0.0;
        for (int i = 0; i < ng; ++i) {
            double th = 2.0 * M_PI * (double)(((int64_t)m * i) % ng) / ng;
            acc += f[i] * cexp(-I * th);
        }
        F[m] = acc;
    }
}

static void idft(int ng, const double complex *F, double *f)
{
    for (int i = 0; i < ng; ++i) {
        double complex acc = 0.0;
        for (int m = 0; m < ng; ++m) {
            double th = 2.0 * M_PI * (double)(((int64_t)m * i) % ng) / ng;
            acc += F[m] * cexp(I * th);
        }
        f[i] = creal(acc) / ng;
    }
}

void oracle_psatd(int ng, double L, double c, double tau, const double *E, const double *B,
                  const double *J, double *Eo, double *Bo, double *Ea)
{
    const double h = L / ng, c2 = c * c;
    double complex *Ef = malloc(sizeof(double complex) * (size_t)ng);
    double complex *Bf = malloc(sizeof(double complex) * (size_t)ng);
    double complex *Jf = malloc(sizeof(double complex) * (size_t)ng);
    double complex *E1 = malloc(sizeof(double complex) * (size_t)ng);
    double complex *B1 = malloc(sizeof(double complex) * (size_t)ng);
    double complex *A1 = malloc(sizeof(double complex) * (size_t)ng);
    double *bneg = malloc(sizeof(double) * (size_t)ng), *tmp = malloc(sizeof(double) * (size_t)ng);
    for (int i = 0; i < ng; ++i) {
        Eo[i] = E[i] - tau * J[i];                              /* E_x */
        if (Ea)
            Ea[i] = E[i] - 0.5 * tau * J[i];
    }
    for (int pair = 0; pair < 2; ++pair) {
        /* pair 0: (E_y, B_z, j_y); pair 1: (E_z, -B_y, j_z) */
        const double *e = E + (1 + pair) * ng, *j = J + (1 + pair) * ng;
        const double *bb = pair == 0 ? B + ng : B;
        const double sg = pair == 0 ? 1.0 : -1.0;
        for (int i = 0; i < ng; ++i)
            bneg[i] = sg * bb[i];
        dft(ng, e, Ef);
        dft(ng, bneg, Bf);
        dft(ng, j, Jf);
        for (int m = 0; m < ng; ++m) {
            const int ms = 2 * m <= ng ? m : m - ng;             /* signed mode number */
            if (ms == 0) {
                E1[m] = Ef[m] - tau * Jf[m];
                B1[m] = Bf[m];
                A1[m] = Ef[m] - 0.5 * tau * Jf[m];
                continue;
            }
            const double k = 2.0 * M_PI * ms / L, w = c * fabs(k);
            const double complex a = I * k * cexp(I * 0.5 * k * h);
            const double complex b = I * k * cexp(-I * 0.5 * k * h);
            const double C = cos(w * tau), S = sin(w * tau);
            E1[m] = C * Ef[m] - c2 * b * S / w * Bf[m] - S / w * Jf[m];
            B1[m] = C * Bf[m] - a * S / w * Ef[m] + a * (1.0 - C) / (w * w) * Jf[m];
            A1[m] = S / (w * tau) * Ef[m] - c2 * b * (1.0 - C) / (w * w * tau) * Bf[m]
                    - (1.0 - C) / (w * w * tau) * Jf[m];
        }
        idft(ng, E1, Eo + (1 + pair) * ng);
        idft(ng, B1, tmp);
        for (int i = 0; i < ng; ++i)
            (pair == 0 ? Bo + ng : Bo)[i] = sg * tmp[i];
        if (Ea)
            idft(ng, A1, Ea + (1 + pair) * ng);
    }
    free(Ef); free(Bf); free(Jf); free(E1); free(B1); free(A1); free(bneg); free(tmp);
}

/* Staggered differences: node arrays f[i] at i h, half-node arrays g[i] at (i + 1/2) h.
 * D+ f at half node i: (f[i+1] - f[i]) / h;  D- g at node i: (g[i] - g[i-1]) / h. */
static double dplus(const double *f, int i, int ng, double h)
{
    return (f[(i + 1) % ng] - f[i]) / h;
}

static double dminus(const double *g, int i, int ng, double h)
{
    return (g[i] - g[(i + ng - 1) % ng]) / h;
}

/* Yee leapfrog magnetic half step (eq. (EMleapfrog), second line):
 * B^{n+1/2} = B^{n-1/2} - dt curl E^n, (curl E)_y = -D+E_z, (curl E)_z = D+E_y.
 * E [3][ng] on the nodes, B and Bo [2][ng] (B_y, B_z) on the half nodes. */
static void leapfrog_b(int ng, double h, double dt, const double *E, const double *B, double *Bo)
{
    const double *Ey = E + ng, *Ez = E + 2 * ng;
    for (int i = 0; i < ng; ++i) {
        Bo[i] = B[i] + dt * dplus(Ez, i, ng, h);
        Bo[ng + i] = B[ng + i] - dt * dplus(Ey, i, ng, h);
    }
}

/* ------------------------------------------------------------------------ energy */

void oracle_energy(const ocfg *cfg, const double *v, const double *w, const double *E,
                   const double *B, odiag *d)
{
    int64_t np = cfg->n_particles;
    int ng = cfg->n_cells, nv = cfg->nv;
    double h = cfg->length / ng, wu = cfg->length / (double)np;
    nsum ke = {0, 0}, we = {0, 0}, wb = {0, 0};
    for (int64_t p = 0; p < np; ++p) {
        double v2 = 0.0;
        for (int c = 0; c < nv; ++c)
            v2 += v[c * np + p] * v[c * np + p];
        nadd(&ke, 0.5 * (w ? w[p] : wu) * v2);
    }
    const int emf = cfg->scheme == 2 || cfg->scheme == 4 || cfg->scheme == 5;
    int ne = emf ? 3 : 1;
    for (int c = 0; c < ne; ++c)
        for (int i = 0; i < ng; ++i)
            nadd(&we, 0.5 * h * E[c * ng + i] * E[c * ng + i]);
    if (emf && B && cfg->scheme == 5) {
        /* leapfrog (section 4.1): the state holds E^n and B^{n-1/2};
         * W_B^n = c^2/2 h sum B^{n+1/2} . B^{n-1/2} with B^{n+1/2} = B^{n-1/2} - dt curl E^n */
        double *bh = malloc(sizeof(double) * 2 * (size_t)ng);
        leapfrog_b(ng, h, cfg->dt, E, B, bh);
        for (int c = 0; c < 2; ++c)
            for (int i = 0; i < ng; ++i)
                nadd(&wb, 0.5 * cfg->c * cfg->c * h * bh[c * ng + i] * B[c * ng + i]);
        free(bh);
    } else if (emf && B) {
        for (int c = 0; c < 2; ++c)
            for (int i = 0; i < ng; ++i)
                nadd(&wb, 0.5 * cfg->c * cfg->c * h * B[c * ng + i] * B[c * ng + i]);
    }
    d->kinetic = ke.s + ke.c;
    d->field_e = we.s + we.c;
    d->field_b = wb.s + wb.c;
    d->total = d->kinetic + d->field_e + d->field_b;
}

/* --------------------------------------------------------------------- the step */

typedef struct {
    double *xs, *x1, *xh, *vs, *wv, *gE, *gB;
    double *J1, *J2, *Es, *Bs, *En, *Bn, *Eb, *Bb, *R;
} owork;

static void cross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Solve v = u + v x t for v (the implicit half-step velocity of eq. (EMbasic), also the
 * rotation of the symmetric Boris push): v = (u + u x t + (u.t) t) / (1 + |t|^2). */
static void solve_vstar(const double *u, const double *t, double *v)
{
    double uxt[3];
    cross(u, t, uxt);
    double ut = u[0] * t[0] + u[1] * t[1] + u[2] * t[2];
    double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int c = 0; c < 3; ++c)
        v[c] = (u[c] + uxt[c] + ut * t[c]) / (1.0 + tt);
}

static int step(const ocfg *cfg, double *x, double *v, const double *w, double *E,
                double *B, owork *o, odiag *d, double *gamma_out)
{
    const int64_t np = cfg->n_particles;
    const int ng = cfg->n_cells, nv = cfg->nv, ord = cfg->order, sch = cfg->scheme;
    const double L = cfg->length, h = L / ng, dt = cfg->dt, c2 = cfg->c * cfg->c;
    const double wu = L / (double)np;
    const int psatd = sch == 4, lf = sch == 5;
    const int em = sch == 2 || psatd || lf;
    const double gs = cfg->cc ? 0.5 : 0.0;       /* E_x, j on the half nodes (cc) */
    const int ncur = em ? 3 : 1;                 /* current components that matter */
    double *vx = v;

    for (int64_t p = 0; p < np; ++p)
        o->wv[p] = w ? w[p] : wu;

    /* S1: x* = x^n + dt/2 v^n */
    for (int64_t p = 0; p < np; ++p)
        o->xs[p] = x[p] + 0.5 * dt * vx[p];

    /* S2-S3: predictor deposit j^{n,*} (velocity v^n at x*) and predictor fields */
    if (sch == 1) {
        memcpy(o->Es, E, sizeof(double) * (size_t)ng);
    } else {
        for (int c = 0; c < ncur; ++c)
            oracle_deposit(ord, np, o->xs, o->wv, v + c * np, ng, h, gs, o->J1 + c * ng);
        if (!em) {
            double m = mean(o->J1, ng);
            for (int i = 0; i < ng; ++i)
                o->Es[i] = E[i] - 0.5 * dt * (o->J1[i] - m);
        } else if (psatd) {
            /* (E*, B*) = PSATD(E^n, B^n, j^{n,*}, dt/2) */
            oracle_psatd(ng, L, cfg->c, 0.5 * dt, E, B, o->J1, o->Es, o->Bs, NULL);
        } else if (lf) {
            /* B^{n+1/2} = B^{n-1/2} - dt curl E^n into Bs (gathered at x* for v* and at
             * x^{n+1/2} for v-dagger);  E* = E^n + dt/2 (c^2 curl B^{n+1/2} - j^{n,*}) */
            leapfrog_b(ng, h, dt, E, B, o->Bs);
            const double *By = o->Bs, *Bz = o->Bs + ng;
            for (int i = 0; i < ng; ++i) {
                o->Es[i] = E[i] - 0.5 * dt * o->J1[i];
                o->Es[ng + i] = E[ng + i] + 0.5 * dt * (-c2 * dminus(Bz, i, ng, h) - o->J1[ng + i]);
                o->Es[2 * ng + i] = E[2 * ng + i] + 0.5 * dt * (c2 * dminus(By, i, ng, h) - o->J1[2 * ng + i]);
            }
        } else {
            const double *Ex = E, *Ey = E + ng, *Ez = E + 2 * ng;
            const double *By = B, *Bz = B + ng;
            for (int i = 0; i < ng; ++i) {
                /* E* = E + dt/2 (c^2 curl B - j):  (curl B)_y = -D-Bz, (curl B)_z = D-By */
                o->Es[i] = Ex[i] - 0.5 * dt * o->J1[i];
                o->Es[ng + i] = Ey[i] + 0.5 * dt * (-c2 * dminus(Bz, i, ng, h) - o->J1[ng + i]);
                o->Es[2 * ng + i] = Ez[i] + 0.5 * dt * (c2 * dminus(By, i, ng, h) - o->J1[2 * ng + i]);
                /* B* = B - dt/2 curl E:  (curl E)_y = -D+Ez, (curl E)_z = D+Ey */
                o->Bs[i] = By[i] + 0.5 * dt * dplus(Ez, i, ng, h);
                o->Bs[ng + i] = Bz[i] - 0.5 * dt * dplus(Ey, i, ng, h);
            }
        }
    }

    /* S4-S5: gather at x* and the half-step velocity v* */
    if (nv == 1) {
        oracle_gather(ord, np, o->xs, o->Es, ng, h, gs, o->gE);
        for (int64_t p = 0; p < np; ++p)
            o->vs[p] = v[p] + 0.5 * dt * o->gE[p];
    } else {
        int ne = em ? 3 : 1;
        double *gE = o->gE;                        /* [3][np] */
        for (int c = 0; c < 3; ++c) {
            if (c < ne)
                oracle_gather(ord, np, o->xs, o->Es + c * ng, ng, h, gs, gE + c * np);
            else
                memset(gE + c * np, 0, sizeof(double) * (size_t)np);
        }
        if (em) {   /* B_y, B_z live on the half nodes */
            oracle_gather(ord, np, o->xs, o->Bs, ng, h, 0.5, o->gB);
            oracle_gather(ord, np, o->xs, o->Bs + ng, ng, h, 0.5, o->gB + np);
        }
        for (int64_t p = 0; p < np; ++p) {
            double u[3], t[3], vs[3];
            double bb[3] = {cfg->b_ext[0], cfg->b_ext[1], cfg->b_ext[2]};
            if (em) {
                bb[1] += o->gB[p];
                bb[2] += o->gB[np + p];
            }
            for (int c = 0; c < 3; ++c) {
                u[c] = v[c * np + p] + 0.5 * dt * gE[c * np + p];
                t[c] = 0.5 * dt * bb[c];
            }
            solve_vstar(u, t, vs);
            for (int c = 0; c < 3; ++c)
                o->vs[c * np + p] = vs[c];
        }
    }

    /* S6: x^{n+1} = x^n + dt v*_x (unwrapped) and x^{n+1/2} = (x^n + x^{n+1}) / 2 */
    for (int64_t p = 0; p < np; ++p) {
        o->x1[p] = x[p] + dt * o->vs[p];
        o->xh[p] = 0.5 * (x[p] + o->x1[p]);
    }

    /* S7: centred deposit j^{*,n+1/2} (velocity v* at x^{n+1/2}); with exact charge
     * conservation, through the pieces of the path x^n -> x^{n+1} (their midpoints replace
     * x^{n+1/2}) */
    if (cfg->cc)
        oracle_deposit_cc(np, x, o->x1, o->wv, o->vs, ng, h, o->J2);
    else
        for (int c = 0; c < ncur; ++c)
            oracle_deposit(ord, np, o->xh, o->wv, o->vs + c * np, ng, h, 0.0, o->J2 + c * ng);

    /* S8: field update */
    if (lf) {
        /* E^{n+1} = E^n + dt (c^2 curl B^{n+1/2} - j^{*,n+1/2}); v-dagger gathers
         * E^{n+1/2} = (E^n + E^{n+1})/2 and B^{n+1/2}, which the state carries on */
        const double *By = o->Bs, *Bz = o->Bs + ng;
        for (int i = 0; i < ng; ++i) {
            o->En[i] = E[i] - dt * o->J2[i];
            o->En[ng + i] = E[ng + i] + dt * (-c2 * dminus(Bz, i, ng, h) - o->J2[ng + i]);
            o->En[2 * ng + i] = E[2 * ng + i] + dt * (c2 * dminus(By, i, ng, h) - o->J2[2 * ng + i]);
        }
        for (int i = 0; i < 3 * ng; ++i)
            o->Eb[i] = 0.5 * (E[i] + o->En[i]);
        memcpy(o->Bb, o->Bs, sizeof(double) * 2 * (size_t)ng);
        memcpy(o->Bn, o->Bs, sizeof(double) * 2 * (size_t)ng);
    } else if (psatd) {
        /* (E^{n+1}, B^{n+1}) = PSATD(E^n, B^n, j^{*,n+1/2}, dt); the gather for v-dagger takes
         * the time average <E> over the step; B at n + 1/2 is the mean of B^n and B^{n+1} */
        oracle_psatd(ng, L, cfg->c, dt, E, B, o->J2, o->En, o->Bn, o->Eb);
        for (int i = 0; i < 2 * ng; ++i)
            o->Bb[i] = 0.5 * (B[i] + o->Bn[i]);
    } else if (!em) {
        double m = mean(o->J2, ng);
        for (int i = 0; i < ng; ++i)
            o->En[i] = E[i] - dt * (o->J2[i] - m);
        for (int i = 0; i < ng; ++i)
            o->Eb[i] = 0.5 * (E[i] + o->En[i]);
    } else {
        const double a = 0.5 * dt, s = a * a * c2;
        const double *Ex = E, *Ey = E + ng, *Ez = E + 2 * ng;
        const double *By = B, *Bz = B + ng;
        double *Lf = o->R + ng;
        /* E_x: no curl term in 1D */
        for (int i = 0; i < ng; ++i)
            o->En[i] = Ex[i] - dt * o->J2[i];
        /* (I - s L) Ey' = (I + s L) Ey - dt c^2 D-Bz - dt jy */
        for (int i = 0; i < ng; ++i) {
            double lap = (Ey[(i + 1) % ng] - 2.0 * Ey[i] + Ey[(i + ng - 1) % ng]) / (h * h);
            o->R[i] = Ey[i] + s * lap - dt * c2 * dminus(Bz, i, ng, h) - dt * o->J2[ng + i];
        }
        oracle_cn_solve(ng, h, s, o->R, o->En + ng);
        /* (I - s L) Ez' = (I + s L) Ez + dt c^2 D-By - dt jz */
        for (int i = 0; i < ng; ++i) {
            double lap = (Ez[(i + 1) % ng] - 2.0 * Ez[i] + Ez[(i + ng - 1) % ng]) / (h * h);
            o->R[i] = Ez[i] + s * lap + dt * c2 * dminus(By, i, ng, h) - dt * o->J2[2 * ng + i];
        }
        oracle_cn_solve(ng, h, s, o->R, o->En + 2 * ng);
        /* Bz' = Bz - a D+(Ey + Ey'),  By' = By + a D+(Ez + Ez') */
        for (int i = 0; i < ng; ++i)
            Lf[i] = Ey[i] + o->En[ng + i];
        for (int i = 0; i < ng; ++i)
            o->Bn[ng + i] = Bz[i] - a * dplus(Lf, i, ng, h);
        for (int i = 0; i < ng; ++i)
            Lf[i] = Ez[i] + o->En[2 * ng + i];
        for (int i = 0; i < ng; ++i)
            o->Bn[i] = By[i] + a * dplus(Lf, i, ng, h);
        for (int i = 0; i < 3 * ng; ++i)
            o->Eb[i] = 0.5 * (E[i] + o->En[i]);
        for (int i = 0; i < 2 * ng; ++i)
            o->Bb[i] = 0.5 * (B[i] + o->Bn[i]);
    }

    /* S9-S13: gather at x^{n+1/2}, provisional v-dagger, energy-restoring Gamma */
    int64_t fb = 0;
    double gmax = 0.0;
    int nonfinite = 0;
    int ne = em ? 3 : 1;
    double *gE = o->gE, *gBy = o->gB, *gBz = o->gB + np;
    for (int c = 0; c < nv; ++c) {
        if (c < ne && cfg->cc)
            oracle_gather_cc(np, x, o->x1, o->Eb, ng, h, gE);   /* E_x through the pieces */
        else if (c < ne)
            oracle_gather(ord, np, o->xh, o->Eb + c * ng, ng, h, 0.0, gE + c * np);
        else
            memset(gE + c * np, 0, sizeof(double) * (size_t)np);
    }
    if (em) {
        oracle_gather(ord, np, o->xh, o->Bb, ng, h, 0.5, gBy);
        oracle_gather(ord, np, o->xh, o->Bb + ng, ng, h, 0.5, gBz);
    }
    for (int64_t p = 0; p < np; ++p) {
        double vn[3] = {0, 0, 0}, vs[3] = {0, 0, 0}, vd[3] = {0, 0, 0};
        for (int c = 0; c < nv; ++c) {
            vn[c] = v[c * np + p];
            vs[c] = o->vs[c * np + p];
        }
        if (nv == 1) {
            vd[0] = vn[0] + dt * gE[p];
        } else {
            double bb[3] = {cfg->b_ext[0], cfg->b_ext[1], cfg->b_ext[2]}, vxb[3];
            if (em) {
                bb[1] += gBy[p];
                bb[2] += gBz[p];
            }
            cross(vs, bb, vxb);
            for (int c = 0; c < 3; ++c)
                vd[c] = vn[c] + dt * (gE[c * np + p] + vxb[c]);
        }
        /* S11: r = 1 + 2 (v* - (v-dagger + v^n)/2) . (v-dagger - v^n) / |v-dagger|^2 */
        double num = 0.0, den = 0.0;
        for (int c = 0; c < nv; ++c) {
            num += (vs[c] - 0.5 * (vd[c] + vn[c])) * (vd[c] - vn[c]);
            den += vd[c] * vd[c];
        }
        double r = 1.0 + 2.0 * num / den;
        double g;
        /* S12: the root is real iff r >= 0; otherwise (or if r is not finite) Gamma := 1 */
        if (r >= 0.0 && isfinite(r)) {
            g = sqrt(r);
        } else {
            g = 1.0;
            ++fb;
        }
        if (fabs(g - 1.0) > gmax)
            gmax = fabs(g - 1.0);
        if (gamma_out)
            gamma_out[p] = (r >= 0.0 && isfinite(r)) ? g : NAN;
        /* S13 */
        for (int c = 0; c < nv; ++c) {
            v[c * np + p] = g * vd[c];
            if (!isfinite(v[c * np + p]))
                nonfinite = 1;
        }
        if (!isfinite(o->x1[p]))
            nonfinite = 1;
        x[p] = wrap(o->x1[p], L);
    }
    memcpy(E, o->En, sizeof(double) * (size_t)(ne * ng));
    if (em)
        memcpy(B, o->Bn, sizeof(double) * (size_t)(2 * ng));

    oracle_energy(cfg, v, w, E, B, d);
    d->fallbacks = fb;
    d->max_gamma_dev = gmax;
    d->nonfinite = nonfinite;
    return 0;
}

/* Validate the configuration: 0 if usable, -1 otherwise. */
int oracle_check(const ocfg *cfg)
{
    if (!cfg || (cfg->nv != 1 && cfg->nv != 3) || cfg->scheme < 0 || cfg->scheme > 5)
        return -1;
    if (cfg->order < 1 || cfg->order > 2 || cfg->n_particles < 1)
        return -1;
    if (cfg->n_cells < 2 * cfg->order + 1 || !(cfg->length > 0.0) || !(cfg->dt > 0.0))
        return -1;
    if (cfg->scheme == 3 || cfg->scheme > 5)
        return -1;
    if ((cfg->scheme == 2 || cfg->scheme >= 4) && (cfg->nv != 3 || !(cfg->c > 0.0)))
        return -1;
    if (cfg->cc && (cfg->scheme > 1 || cfg->order != 1))
        return -1;                      /* charge conservation: ESEC2/ESEC1, tent shapes */
    return 0;
}

/* Run n steps.  rec[0] holds the diagnostics of the initial state, rec[k] those after
 * step k.  If init_gauss, E_x is first set from the particles by oracle_gauss.
 * x is wrapped into [0, L) before the first step.  If gamma_out is not NULL it
 * receives Gamma_p of the last step, NaN where the fallback was taken. */
int oracle_run_gamma(const ocfg *cfg, double *x, double *v, const double *w, double *E,
                     double *B, int64_t nsteps, int init_gauss, odiag *rec, double *gamma_out)
{
    if (oracle_check(cfg))
        return -1;
    const int64_t np = cfg->n_particles;
    const int ng = cfg->n_cells;
    for (int64_t p = 0; p < np; ++p)
        x[p] = wrap(x[p], cfg->length);
    if (init_gauss) {
        const double wu = cfg->length / (double)np;
        double *wv = (double *)malloc(sizeof(double) * (size_t)np);
        for (int64_t p = 0; p < np; ++p)
            wv[p] = w ? w[p] : wu;
        if (cfg->cc)
            oracle_gauss_cc(np, x, wv, ng, cfg->length, E);
        else
            oracle_gauss(cfg->order, np, x, wv, ng, cfg->length, E);
        free(wv);
    }
    owork o;
    size_t P = sizeof(double) * (size_t)np, G = sizeof(double) * (size_t)ng;
    o.xs = malloc(P); o.x1 = malloc(P); o.xh = malloc(P); o.wv = malloc(P);
    o.vs = malloc(3 * P); o.gE = malloc(3 * P); o.gB = malloc(2 * P);
    o.J1 = malloc(3 * G); o.J2 = malloc(3 * G); o.Es = malloc(3 * G); o.Bs = malloc(2 * G);
    o.En = malloc(3 * G); o.Bn = malloc(2 * G); o.Eb = malloc(3 * G); o.Bb = malloc(2 * G);
    o.R = malloc(2 * G);
    memset(&rec[0], 0, sizeof(odiag));
    oracle_energy(cfg, v, w, E, B, &rec[0]);
    for (int64_t n = 0; n < nsteps; ++n) {
        memset(&rec[n + 1], 0, sizeof(odiag));
        step(cfg, x, v, w, E, B, &o, &rec[n + 1], n + 1 == nsteps ? gamma_out : NULL);
    }
    free(o.xs); free(o.x1); free(o.xh); free(o.wv); free(o.vs); free(o.gE); free(o.gB);
    free(o.J1); free(o.J2); free(o.Es); free(o.Bs); free(o.En); free(o.Bn);
    free(o.Eb); free(o.Bb); free(o.R);
    return 0;
}

int oracle_run(const ocfg *cfg, double *x, double *v, const double *w, double *E,
               double *B, int64_t nsteps, int init_gauss, odiag *rec)
{
    return oracle_run_gamma(cfg, x, v, w, E, B, nsteps, init_gauss, rec, NULL);
}

/* ====================================================================================
 * Standard explicit PIC, the comparison scheme of section 5: the Vlasov-Poisson system
 * with the leapfrog/Boris push in its symmetric form, eq. (symm_Boris):
 *   x* = x^n + dt/2 v^n,
 *   v^{n+1} = v^n + dt (E(x*, t^{n+1/2}) + v^{n+1/2} x B),  v^{n+1/2} = (v^n + v^{n+1}) / 2,
 *   x^{n+1} = x* + dt/2 v^{n+1}.
 * E(., t^{n+1/2}) is the Poisson (Gauss) field of the charge density deposited at the
 * positions x* (section 2.2), solved spectrally as in oracle_gauss_rho; optionally the
 * density first passes once through the binomial filter (1/4, 1/2, 1/4), which section 5
 * applies to the standard scheme.  B is the uniform imposed field (1D-3V); with nv = 1
 * there is no B.  The velocity update is linear in v^{n+1}: v^{n+1/2} = u + v^{n+1/2} x t
 * with u = v^n + dt/2 E, t = dt/2 B, solved in closed form (solve_vstar).
 *
 * Energy records (section 5.1's TE, with the leapfrog's fields at half steps):
 *   rec[0]     = KE(v^0) + W_E(E^0), E^0 the Gauss field of the density at x^0;
 *   rec[n + 1] = (KE(v^n) + KE(v^{n+1})) / 2 + W_E(E^{n+1/2})   (time (n + 1/2) dt).
 * Fallbacks and max |Gamma - 1| are zero (there is no Gamma).
 * ==================================================================================== */

/* One pass of the periodic binomial filter: out_i = (f_{i-1} + 2 f_i + f_{i+1}) / 4. */
void oracle_binomial(int ng, const double *f, double *out)
{
    for (int i = 0; i < ng; ++i)
        out[i] = 0.25 * f[(i + ng - 1) % ng] + 0.5 * f[i] + 0.25 * f[(i + 1) % ng];
}

/* Field of the particles at positions pos: deposit, optional filter, Gauss solve. */
static void std_field(const ocfg *cfg, const double *pos, const double *wv, const double *ones,
                      int filter, double *rho, double *tmp, double *E)
{
    const int ng = cfg->n_cells;
    const double h = cfg->length / ng;
    oracle_deposit(cfg->order, cfg->n_particles, pos, wv, ones, ng, h, 0.0, rho);
    if (filter) {
        oracle_binomial(ng, rho, tmp);
        memcpy(rho, tmp, sizeof(double) * (size_t)ng);
    }
    oracle_gauss_rho(ng, cfg->length, rho, E);
}

static double kinetic(const ocfg *cfg, const double *v, const double *wv)
{
    const int64_t np = cfg->n_particles;
    nsum ke = {0.0, 0.0};
    for (int64_t p = 0; p < np; ++p) {
        double v2 = 0.0;
        for (int c = 0; c < cfg->nv; ++c)
            v2 += v[c * np + p] * v[c * np + p];
        nadd(&ke, 0.5 * wv[p] * v2);
    }
    return ke.s + ke.c;
}

static double field_energy(const ocfg *cfg, const double *E)
{
    const double h = cfg->length / cfg->n_cells;
    nsum we = {0.0, 0.0};
    for (int i = 0; i < cfg->n_cells; ++i)
        nadd(&we, 0.5 * h * E[i] * E[i]);
    return we.s + we.c;
}

/* Run n steps of the standard scheme (nv = 1, or 3 with the uniform B of cfg->b_ext).
 * x, v: the state in, the state n steps later out.  E: the newest field out (E^{n-1/2},
 * or E^0 after a first call with n = 0).  first != 0: the state is the initial one (x is
 * wrapped, rec[0] is the initial record); otherwise the run continues and rec[0] is not
 * written.  rec[1..n] as described above.  Returns 0, or -1 for a bad configuration. */
int oracle_std_run(const ocfg *cfg, double *x, double *v, const double *w, double *E,
                   int64_t nsteps, int filter, int first, odiag *rec)
{
    if (oracle_check(cfg) || cfg->scheme == 2 || cfg->scheme >= 4 || cfg->cc)
        return -1;
    const int64_t np = cfg->n_particles;
    const int ng = cfg->n_cells, nv = cfg->nv;
    const double L = cfg->length, h = L / ng, dt = cfg->dt;
    const size_t P = sizeof(double) * (size_t)np, G = sizeof(double) * (size_t)ng;
    double *wv = malloc(P), *ones = malloc(P), *xs = malloc(P), *gE = malloc(P);
    double *rho = malloc(G), *tmp = malloc(G);
    const double wu = L / (double)np;
    for (int64_t p = 0; p < np; ++p) {
        wv[p] = w ? w[p] : wu;
        ones[p] = 1.0;
        if (first)
            x[p] = wrap(x[p], L);
    }
    double ke_old = kinetic(cfg, v, wv);
    if (first) {
        /* record 0: the field of the initial positions */
        std_field(cfg, x, wv, ones, filter, rho, tmp, E);
        memset(&rec[0], 0, sizeof(odiag));
        rec[0].kinetic = ke_old;
        rec[0].field_e = field_energy(cfg, E);
        rec[0].total = rec[0].kinetic + rec[0].field_e;
    }
    for (int64_t n = 0; n < nsteps; ++n) {
        /* x* = x^n + dt/2 v^n and the field E^{n+1/2} of the density there */
        for (int64_t p = 0; p < np; ++p)
            xs[p] = x[p] + 0.5 * dt * v[p];
        std_field(cfg, xs, wv, ones, filter, rho, tmp, E);
        oracle_gather(cfg->order, np, xs, E, ng, h, 0.0, gE);
        int nonfinite = 0;
        for (int64_t p = 0; p < np; ++p) {
            if (nv == 1) {
                v[p] = v[p] + dt * gE[p];
            } else {
                double u[3], t[3], vh[3];
                for (int c = 0; c < 3; ++c) {
                    u[c] = v[c * np + p] + (c == 0 ? 0.5 * dt * gE[p] : 0.0);
                    t[c] = 0.5 * dt * cfg->b_ext[c];
                }
                solve_vstar(u, t, vh);                      /* v^{n+1/2} */
                for (int c = 0; c < 3; ++c)
                    v[c * np + p] = 2.0 * vh[c] - v[c * np + p];
            }
            const double x1 = xs[p] + 0.5 * dt * v[p];
            for (int c = 0; c < nv; ++c)
                if (!isfinite(v[c * np + p]))
                    nonfinite = 1;
            if (!isfinite(x1))
                nonfinite = 1;
            x[p] = wrap(x1, L);
        }
        const double ke_new = kinetic(cfg, v, wv);
        odiag *d = &rec[n + 1];
        memset(d, 0, sizeof(odiag));
        d->kinetic = 0.5 * (ke_old + ke_new);
        d->field_e = field_energy(cfg, E);
        d->total = d->kinetic + d->field_e;
        d->nonfinite = nonfinite;
        ke_old = ke_new;
    }
    free(wv); free(ones); free(xs); free(gE); free(rho); free(tmp);
    return 0;
}

/* ====================================================================================
 * Tangent-linear (forward-mode) derivative of an ESEC2 run, 1D-1V electrostatic.
 *
 * The run is the map (x^0, v^0) -> (x^n, v^n, E^n), n = 1..N, of eq. (good_translation)
 * with (doublestardef), with E^0 from the Gauss solve of the initial particles, and the
 * loss J = lw * sum_{n=1..N} W_E^n with W_E = (h/2) sum_i E_i^2 (section 5.1).  This
 * function propagates K tangent directions (dx^0, dv^0) alongside the state by the
 * chain rule applied to each of S0-S13 in turn, and accumulates dJ for each direction.
 * It is the plain definition of the derivative written out; the fallback branch Gamma
 * := 1 (section 3.2) is a constant, so its derivative is zero.
 * ==================================================================================== */

/* Derivative of bspline(order, t) with respect to t (zero at the tent's kinks). */
static double dbspline(int order, double t)
{
    double a = fabs(t), sg = t > 0.0 ? 1.0 : (t < 0.0 ? -1.0 : 0.0);
    if (order == 1)
        return a < 1.0 ? -sg : 0.0;
    if (a < 0.5)
        return -2.0 * t;
    if (a < 1.5)
        return -(1.5 - a) * sg;
    return 0.0;
}

/* Nodes of a particle at position pos with the weight S(x_j - pos) and its derivative
 * with respect to pos: d/dpos bspline(j - pos/h) = -bspline'(j - pos/h) / h. */
static int stencil_d(int order, double pos, double h, int ng, int64_t *idx, double *wt,
                     double *dwt)
{
    double xi = pos / h;
    int64_t j0 = (int64_t)floor(xi);
    int n = 0;
    for (int64_t j = j0 - 1; j <= j0 + 2; ++j) {
        double s = bspline(order, (double)j - xi);
        double ds = -dbspline(order, (double)j - xi) / h;
        if (s != 0.0 || ds != 0.0) {
            idx[n] = pmod(j, ng);
            wt[n] = s;
            dwt[n] = ds;
            ++n;
        }
    }
    return n;
}

/* d j_i = (1/h) sum_p w_p [du_p S(x_i - x_p) + u_p dS/dx_p dx_p]; out zeroed first. */
static void tlm_deposit(int order, int64_t np, const double *x, const double *dx,
                        const double *w, const double *u, const double *du, int ng, double h,
                        double *out)
{
    int64_t idx[4];
    double wt[4], dwt[4];
    memset(out, 0, sizeof(double) * (size_t)ng);
    for (int64_t p = 0; p < np; ++p) {
        int n = stencil_d(order, x[p], h, ng, idx, wt, dwt);
        for (int k = 0; k < n; ++k)
            out[idx[k]] += w[p] * (du[p] * wt[k] + u[p] * dwt[k] * dx[p]) / h;
    }
}

/* d G_p = sum_i [dF_i S(x_i - x_p) + F_i dS/dx_p dx_p]. */
static void tlm_gather(int order, int64_t np, const double *x, const double *dx,
                       const double *F, const double *dF, int ng, double h, double *out)
{
    int64_t idx[4];
    double wt[4], dwt[4];
    for (int64_t p = 0; p < np; ++p) {
        int n = stencil_d(order, x[p], h, ng, idx, wt, dwt);
        double acc = 0.0;
        for (int k = 0; k < n; ++k)
            acc += dF[idx[k]] * wt[k] + F[idx[k]] * dwt[k] * dx[p];
        out[p] = acc;
    }
}

/* Run N steps of ESEC2 (cfg: nv 1, scheme 0) from (x, v) with K tangent directions.
 *   x, v      [np]: initial state in, final state out (x wrapped first)
 *   E         [ng]: E^0 in when !init_gauss (else computed), E^N out
 *   dx, dv  [K][np]: initial tangents in, final tangents out
 *   dE      [K][ng]: tangent of E^0 in when !init_gauss (else computed), of E^N out
 *   loss, dloss[K]: J and dJ for each direction
 *   rec     [N+1] : diagnostics (as oracle_run), or NULL
 * Returns 0, or -1 for an unsupported configuration. */
int oracle_tlm_run(const ocfg *cfg, double *x, double *v, const double *w, double *E,
                   int64_t nsteps, int init_gauss, double lw, int K, double *dx, double *dv,
                   double *dE, double *loss, double *dloss, odiag *rec)
{
    if (oracle_check(cfg) || cfg->nv != 1 || cfg->scheme != 0 || K < 0 || cfg->cc)
        return -1;
    const int64_t np = cfg->n_particles;
    const int ng = cfg->n_cells, ord = cfg->order;
    const double L = cfg->length, h = L / ng, dt = cfg->dt;
    const size_t P = sizeof(double) * (size_t)np, G = sizeof(double) * (size_t)ng;
    double *wv = malloc(P), *xs = malloc(P), *x1 = malloc(P), *xh = malloc(P);
    double *vs = malloc(P), *gs = malloc(P), *gb = malloc(P);
    double *J1 = malloc(G), *J2 = malloc(G), *Es = malloc(G), *En = malloc(G), *Eb = malloc(G);
    double *dxs = malloc(P), *dx1 = malloc(P), *dxh = malloc(P), *dvs = malloc(P);
    double *dgs = malloc(P), *dgb = malloc(P), *zero = calloc((size_t)np, sizeof(double));
    double *ones = malloc(P);
    double *dJ1 = malloc(G), *dJ2 = malloc(G), *dEs = malloc(G), *dEn = malloc(G), *dEb = malloc(G);
    double *vd = malloc(P), *num = malloc(P), *den = malloc(P), *gam = malloc(P);
    int *ok = malloc(sizeof(int) * (size_t)np);
    const double wu = L / (double)np;
    for (int64_t p = 0; p < np; ++p) {
        wv[p] = w ? w[p] : wu;
        ones[p] = 1.0;
        x[p] = wrap(x[p], L);
    }
    /* S0: E^0 from rho(x^0); its tangent from d rho = (1/h) sum w dS/dx dx */
    if (init_gauss) {
        double *rho = malloc(G);
        oracle_deposit(ord, np, x, wv, ones, ng, h, 0.0, rho);
        oracle_gauss_rho(ng, L, rho, E);
        for (int k = 0; k < K; ++k) {
            tlm_deposit(ord, np, x, dx + (size_t)k * np, wv, ones, zero, ng, h, rho);
            oracle_gauss_rho(ng, L, rho, dE + (size_t)k * ng);
        }
        free(rho);
    }
    nsum J = {0.0, 0.0};
    nsum *dJ = calloc((size_t)(K > 0 ? K : 1), sizeof(nsum));
    if (rec) {
        memset(&rec[0], 0, sizeof(odiag));
        oracle_energy(cfg, v, w, E, NULL, &rec[0]);
    }
    for (int64_t n = 0; n < nsteps; ++n) {
        /* ---- the step itself (as in step(), kept for the tangents) ---- */
        for (int64_t p = 0; p < np; ++p)
            xs[p] = x[p] + 0.5 * dt * v[p];                                     /* S1 */
        oracle_deposit(ord, np, xs, wv, v, ng, h, 0.0, J1);                     /* S2 */
        double m1 = mean(J1, ng);
        for (int i = 0; i < ng; ++i)
            Es[i] = E[i] - 0.5 * dt * (J1[i] - m1);                             /* S3 */
        oracle_gather(ord, np, xs, Es, ng, h, 0.0, gs);                         /* S4 */
        for (int64_t p = 0; p < np; ++p) {
            vs[p] = v[p] + 0.5 * dt * gs[p];                                    /* S5 */
            x1[p] = x[p] + dt * vs[p];                                          /* S6 */
            xh[p] = 0.5 * (x[p] + x1[p]);
        }
        oracle_deposit(ord, np, xh, wv, vs, ng, h, 0.0, J2);                    /* S7 */
        double m2 = mean(J2, ng);
        for (int i = 0; i < ng; ++i) {
            En[i] = E[i] - dt * (J2[i] - m2);                                   /* S8 */
            Eb[i] = 0.5 * (E[i] + En[i]);
        }
        oracle_gather(ord, np, xh, Eb, ng, h, 0.0, gb);                         /* S9 */
        int64_t fb = 0;
        double gmax = 0.0;
        for (int64_t p = 0; p < np; ++p) {
            vd[p] = v[p] + dt * gb[p];                                          /* S10 */
            num[p] = (vs[p] - 0.5 * (vd[p] + v[p])) * (vd[p] - v[p]);           /* S11 */
            den[p] = vd[p] * vd[p];
            double r = 1.0 + 2.0 * num[p] / den[p];
            ok[p] = r >= 0.0 && isfinite(r);                                    /* S12 */
            gam[p] = ok[p] ? sqrt(r) : 1.0;
            if (!ok[p])
                ++fb;
            if (fabs(gam[p] - 1.0) > gmax)
                gmax = fabs(gam[p] - 1.0);
        }
        /* ---- tangents, direction by direction ---- */
        for (int k = 0; k < K; ++k) {
            double *tx = dx + (size_t)k * np, *tv = dv + (size_t)k * np;
            double *tE = dE + (size_t)k * ng;
            for (int64_t p = 0; p < np; ++p)
                dxs[p] = tx[p] + 0.5 * dt * tv[p];
            tlm_deposit(ord, np, xs, dxs, wv, v, tv, ng, h, dJ1);
            double dm1 = mean(dJ1, ng);
            for (int i = 0; i < ng; ++i)
                dEs[i] = tE[i] - 0.5 * dt * (dJ1[i] - dm1);
            tlm_gather(ord, np, xs, dxs, Es, dEs, ng, h, dgs);
            for (int64_t p = 0; p < np; ++p) {
                dvs[p] = tv[p] + 0.5 * dt * dgs[p];
                dx1[p] = tx[p] + dt * dvs[p];
                dxh[p] = 0.5 * (tx[p] + dx1[p]);
            }
            tlm_deposit(ord, np, xh, dxh, wv, vs, dvs, ng, h, dJ2);
            double dm2 = mean(dJ2, ng);
            for (int i = 0; i < ng; ++i) {
                dEn[i] = tE[i] - dt * (dJ2[i] - dm2);
                dEb[i] = 0.5 * (tE[i] + dEn[i]);
            }
            tlm_gather(ord, np, xh, dxh, Eb, dEb, ng, h, dgb);
            for (int64_t p = 0; p < np; ++p) {
                double dvd = tv[p] + dt * dgb[p];
                double a = vs[p] - 0.5 * (vd[p] + v[p]), b = vd[p] - v[p];
                double dnum = (dvs[p] - 0.5 * (dvd + tv[p])) * b + a * (dvd - tv[p]);
                double dden = 2.0 * vd[p] * dvd;
                double dg = 0.0;
                if (ok[p]) {
                    /* Gamma = sqrt(1 + 2 num / den) */
                    double drho = 2.0 * dnum / den[p] - 2.0 * num[p] * dden / (den[p] * den[p]);
                    dg = drho / (2.0 * gam[p]);
                }
                tv[p] = dg * vd[p] + gam[p] * dvd;                                 /* S13 */
                tx[p] = dx1[p];                                  /* wrap: a translation */
            }
            memcpy(tE, dEn, G);
        }
        /* ---- state update and loss ---- */
        for (int64_t p = 0; p < np; ++p) {
            v[p] = gam[p] * vd[p];
            x[p] = wrap(x1[p], L);
        }
        memcpy(E, En, G);
        nsum we = {0.0, 0.0};
        for (int i = 0; i < ng; ++i)
            nadd(&we, 0.5 * h * E[i] * E[i]);
        nadd(&J, lw * (we.s + we.c));
        for (int k = 0; k < K; ++k) {
            const double *tE = dE + (size_t)k * ng;
            nsum d = {0.0, 0.0};
            for (int i = 0; i < ng; ++i)
                nadd(&d, h * E[i] * tE[i]);
            nadd(&dJ[k], lw * (d.s + d.c));
        }
        if (rec) {
            memset(&rec[n + 1], 0, sizeof(odiag));
            oracle_energy(cfg, v, w, E, NULL, &rec[n + 1]);
            rec[n + 1].fallbacks = fb;
            rec[n + 1].max_gamma_dev = gmax;
        }
    }
    *loss = J.s + J.c;
    for (int k = 0; k < K; ++k)
        dloss[k] = dJ[k].s + dJ[k].c;
    free(dJ);
    free(wv); free(xs); free(x1); free(xh); free(vs); free(gs); free(gb);
    free(J1); free(J2); free(Es); free(En); free(Eb);
    free(dxs); free(dx1); free(dxh); free(dvs); free(dgs); free(dgb); free(zero); free(ones);
    free(dJ1); free(dJ2); free(dEs); free(dEn); free(dEb);
    free(vd); free(num); free(den); free(gam); free(ok);
    return 0;
}
