/*
 * Reference oracle for the explicit finite-difference phase-field /
 * reaction-diffusion step (SymPhas 2.0, arXiv 2511.10508).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct
 * CPU implementation in FP64 that the GPU library is checked against.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code with the GPU library.
 *
 * Conventions
 *   - Fields are stored x fastest, then y, then z: site (x,y,z) has linear
 *     index x + nx*(y + ny*z).  A 2D grid has nz = 1, a 1D grid ny = nz = 1.
 *   - Boundaries are periodic (the paper's benchmarks and figures all use
 *     periodic boundaries, Sec. "Benchmarks").  Neighbour indices wrap with
 *     a true modulo, so a stencil wider than the grid is still defined.
 *   - The centred second-derivative weights w[1..r] (accuracy order p = 2r)
 *     are an input: the oracle's own generator (exact rationals) lives in
 *     oracle/weights.py.  w[0] is not used: the Laplacian is evaluated in
 *     difference form (below), which needs only w[1..r].
 *   - Everything is FP64 and compiled with -ffp-contract=off, so every
 *     operation is rounded exactly as written.
 *
 * Model equations (Sec. "Implementations"):
 *   Model A / Allen-Cahn, Eq. (model-a):   dphi/dt = lap(phi) + c1 phi - c2 phi^3
 *   Model B / Cahn-Hilliard, Eq. (model-b): drho/dt = lap(-lap(rho) - c1 rho + c2 rho^3)
 *   Gray-Scott (named in the Introduction; equations and constants are the
 *   standard reaction-diffusion pair, parameters Du, Dv, F, k):
 *       du/dt = Du lap(u) - u v^2 + F (1 - u)
 *       dv/dt = Dv lap(v) + u v^2 - (F + k) v
 *   Model C, Eq. (model-c):  dphi/dt = lap(phi) + c1 phi - c2 phi^3 - 2 phi rho
 *                            drho/dt = lap(rho + c3 phi^2)
 *   Model H, Eq. (model-h), transverse projector one: orc_rhs_mh below.
 * Cahn-Hilliard also comes with a direct biharmonic stencil in place of the
 * Laplacian applied twice (orc_rhs_chd below).
 * The time integrator is forward Euler, Jacobi style: every right-hand side
 * is evaluated from the state at the start of the step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_AC 1
#define ORC_CH 2
#define ORC_GS 3
#define ORC_MC 4

static int64_t wrap(int64_t i, int64_t n)
{
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

static int64_t site(const int64_t n[3], int64_t x, int64_t y, int64_t z)
{
    return wrap(x, n[0]) + n[0] * (wrap(y, n[1]) + n[1] * wrap(z, n[2]));
}

/*
 * Star-shaped discrete Laplacian (sum of 1D centred second-derivative
 * stencils along each active axis), in difference form:
 *
 *   (L u)_i = sum over axes a (x, then y, then z)
 *               sum over j = 1..r
 *                 (w_j / dx^2) * ((u_{i + j e_a} - u_i) + (u_{i - j e_a} - u_i))
 *
 * This equals w_0 u_i + sum_j w_j (u_{i+j} + u_{i-j}) per axis because
 * w_0 = -2 sum_j w_j, but keeps a constant field an exact zero of L.  The
 * paper maps the canonical form div(grad phi) to this one Laplacian stencil
 * (Sec. "Advanced Derivative Support").  Axes beyond ndim are skipped.
 */
void orc_laplacian(int ndim, const int64_t n[3], double dx, int r,
                   const double *w, const double *u, double *out)
{
    const double inv_dx2 = 1.0 / (dx * dx);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < n[2]; ++z)
        for (int64_t y = 0; y < n[1]; ++y)
            for (int64_t x = 0; x < n[0]; ++x) {
                const int64_t i = site(n, x, y, z);
                const double u0 = u[i];
                double acc = 0.0;
                for (int a = 0; a < ndim; ++a) {
                    for (int j = 1; j <= r; ++j) {
                        int64_t dp[3] = {0, 0, 0};
                        dp[a] = j;
                        const double up = u[site(n, x + dp[0], y + dp[1], z + dp[2])];
                        const double um = u[site(n, x - dp[0], y - dp[1], z - dp[2])];
                        acc = acc + (w[j] * inv_dx2) * ((up - u0) + (um - u0));
                    }
                }
                out[i] = acc;
            }
}

static int64_t nsites(const int64_t n[3]) { return n[0] * n[1] * n[2]; }

/*
 * One axis a of a centred even-derivative stencil, in difference form:
 *
 *   (D_a u)_i = sum over j = 1..r  (w_j / h) ((u_{i + j e_a} - u_i) + (u_{i - j e_a} - u_i))
 *
 * with h = dx^2 for the second derivative and dx^4 for the fourth (the
 * caller passes 1/h).  A centred stencil of an even derivative of order >= 2
 * has w_0 = -2 sum_j w_j, so this is the stencil itself.
 */
static void orc_axis(int a, const int64_t n[3], double inv_h, int r, const double *w,
                     const double *u, double *out)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < n[2]; ++z)
        for (int64_t y = 0; y < n[1]; ++y)
            for (int64_t x = 0; x < n[0]; ++x) {
                const int64_t i = site(n, x, y, z);
                const double u0 = u[i];
                double acc = 0.0;
                for (int j = 1; j <= r; ++j) {
                    int64_t dp[3] = {0, 0, 0};
                    dp[a] = j;
                    const double up = u[site(n, x + dp[0], y + dp[1], z + dp[2])];
                    const double um = u[site(n, x - dp[0], y - dp[1], z - dp[2])];
                    acc = acc + (w[j] * inv_h) * ((up - u0) + (um - u0));
                }
                out[i] = acc;
            }
}

/*
 * Direct discrete biharmonic (the paper derives stencils for any derivative
 * order from polynomial interpolation, Secs. "Advanced Derivative Support"
 * and "Compile-Time Stencil Generation"; this is the stencil of the
 * biharmonic itself rather than the Laplacian applied twice):
 *
 *   (B u) = sum over axes a of D4_a u  +  2 sum over axis pairs a < b of D2_a (D2_b u)
 *
 * D4_a: centred fourth-derivative stencil along a, accuracy p, radius
 * r4 = p/2 + 1, weights w4[0..r4];  D2_a: the second-derivative stencil of
 * the Laplacian (radius r = p/2, weights w), so the mixed terms are tensor
 * products of one-axis second derivatives.
 */
void orc_biharmonic_direct(int ndim, const int64_t n[3], double dx, int r, const double *w,
                           int r4, const double *w4, const double *u, double *out)
{
    const int64_t N = nsites(n);
    const double inv_dx2 = 1.0 / (dx * dx);
    const double inv_dx4 = 1.0 / (dx * dx * dx * dx);
    double *t = (double *)malloc(sizeof(double) * (size_t)N);
    double *tt = (double *)malloc(sizeof(double) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) out[i] = 0.0;
    for (int a = 0; a < ndim; ++a) {
        orc_axis(a, n, inv_dx4, r4, w4, u, t);
        for (int64_t i = 0; i < N; ++i) out[i] = out[i] + t[i];
    }
    for (int a = 0; a < ndim; ++a)
        for (int b = a + 1; b < ndim; ++b) {
            orc_axis(b, n, inv_dx2, r, w, u, t);
            orc_axis(a, n, inv_dx2, r, w, t, tt);
            for (int64_t i = 0; i < N; ++i) out[i] = out[i] + 2.0 * tt[i];
        }
    free(t);
    free(tt);
}

/*
 * Right-hand sides of the four models at the current state.
 *   AC: rhs = L phi + c1 phi - c2 phi^3                    (Eq. model-a)
 *   CH: mu  = c2 rho^3 - c1 rho - L rho;  rhs = L mu       (Eq. model-b)
 *   GS: ru  = Du L u - u v^2 + F (1 - u)
 *       rv  = Dv L v + u v^2 - (F + k) v
 *   MC: rphi = L phi + c1 phi - c2 phi^3 - 2 phi rho        (Eq. model-c)
 *       rrho = L (rho + c3 phi^2)
 * params: AC, CH: {c1, c2};  GS: {Du, Dv, F, k};  MC: {c1, c2, c3}.
 * in/rhs hold nfields arrays of nsites each (AC, CH: 1 field; GS: u then v;
 * MC: phi then rho).
 */
void orc_rhs(int kind, int ndim, const int64_t n[3], double dx, int r,
             const double *w, const double *params,
             const double *in, double *rhs)
{
    const int64_t N = nsites(n);
    double *lap = (double *)malloc(sizeof(double) * (size_t)N);
    if (kind == ORC_AC) {
        const double c1 = params[0], c2 = params[1];
        orc_laplacian(ndim, n, dx, r, w, in, lap);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            const double p = in[i];
            rhs[i] = (lap[i] + c1 * p) - c2 * (p * p * p);
        }
    } else if (kind == ORC_CH) {
        const double c1 = params[0], c2 = params[1];
        double *mu = (double *)malloc(sizeof(double) * (size_t)N);
        orc_laplacian(ndim, n, dx, r, w, in, lap);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            const double c = in[i];
            mu[i] = (c2 * (c * c * c) - c1 * c) - lap[i];
        }
        orc_laplacian(ndim, n, dx, r, w, mu, rhs);
        free(mu);
    } else if (kind == ORC_GS) {
        const double Du = params[0], Dv = params[1], F = params[2], k = params[3];
        const double *u = in, *v = in + N;
        double *lapv = (double *)malloc(sizeof(double) * (size_t)N);
        orc_laplacian(ndim, n, dx, r, w, u, lap);
        orc_laplacian(ndim, n, dx, r, w, v, lapv);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            const double uvv = u[i] * v[i] * v[i];
            rhs[i] = (Du * lap[i] - uvv) + F * (1.0 - u[i]);
            rhs[N + i] = (Dv * lapv[i] + uvv) - (F + k) * v[i];
        }
        free(lapv);
    } else if (kind == ORC_MC) {
        const double c1 = params[0], c2 = params[1], c3 = params[2];
        const double *phi = in, *rho = in + N;
        double *g = (double *)malloc(sizeof(double) * (size_t)N);
        orc_laplacian(ndim, n, dx, r, w, phi, lap);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) g[i] = rho[i] + c3 * (phi[i] * phi[i]);
        orc_laplacian(ndim, n, dx, r, w, g, rhs + N);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            const double p = phi[i];
            rhs[i] = ((lap[i] + c1 * p) - c2 * (p * p * p)) - 2.0 * p * rho[i];
        }
        free(g);
    }
    free(lap);
}

static int nfields_of(int kind) { return (kind == ORC_GS || kind == ORC_MC) ? 2 : 1; }

/*
 * Cahn-Hilliard (Eq. model-b) with the direct biharmonic: the right-hand side
 * L mu with mu = c2 rho^3 - c1 rho - L rho expands to L g - L(L rho) with
 * g = c2 rho^3 - c1 rho, and the composed L(L rho) is replaced by B rho:
 *   rhs = L g - B rho.
 */
void orc_rhs_chd(int ndim, const int64_t n[3], double dx, int r, const double *w,
                 int r4, const double *w4, const double *params,
                 const double *in, double *rhs)
{
    const int64_t N = nsites(n);
    const double c1 = params[0], c2 = params[1];
    double *g = (double *)malloc(sizeof(double) * (size_t)N);
    double *b = (double *)malloc(sizeof(double) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        const double c = in[i];
        g[i] = c2 * (c * c * c) - c1 * c;
    }
    orc_laplacian(ndim, n, dx, r, w, g, rhs);
    orc_biharmonic_direct(ndim, n, dx, r, w, r4, w4, in, b);
    for (int64_t i = 0; i < N; ++i) rhs[i] = rhs[i] - b[i];
    free(g);
    free(b);
}

/*
 * Model H (Eq. model-h) with the transverse projector set to one, as the
 * paper does: a conserved scalar m and a vector field j of ndim components,
 *   dm/dt = L mu - c3 div(m j),         mu = c2 m^3 - c1 m - L m
 *   dj/dt = L j - c3 m grad(L m + c1 m - c2 m^3) = L j + c3 m grad(mu)
 * (Sec. "Model H": the equation as printed).  grad and div use the centred
 * first-derivative stencil of accuracy p (radius r, antisymmetric weights
 * w1[1..r]):  (D1_a u)_i = sum_k (w1_k / dx) (u_{i + k e_a} - u_{i - k e_a}).
 * params {c1, c2, c3}; in/rhs hold 1 + ndim arrays (m, then j_x, j_y, j_z).
 */
static void orc_d1(int a, const int64_t n[3], double dx, int r, const double *w1,
                   const double *u, double *out)
{
    const double inv_dx = 1.0 / dx;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < n[2]; ++z)
        for (int64_t y = 0; y < n[1]; ++y)
            for (int64_t x = 0; x < n[0]; ++x) {
                double acc = 0.0;
                for (int k = 1; k <= r; ++k) {
                    int64_t dp[3] = {0, 0, 0};
                    dp[a] = k;
                    const double up = u[site(n, x + dp[0], y + dp[1], z + dp[2])];
                    const double um = u[site(n, x - dp[0], y - dp[1], z - dp[2])];
                    acc = acc + (w1[k] * inv_dx) * (up - um);
                }
                out[site(n, x, y, z)] = acc;
            }
}

void orc_rhs_mh(int ndim, const int64_t n[3], double dx, int r, const double *w,
                const double *w1, const double *params, const double *in, double *rhs)
{
    const int64_t N = nsites(n);
    const double c1 = params[0], c2 = params[1], c3 = params[2];
    const double *m = in;
    double *lap = (double *)malloc(sizeof(double) * (size_t)N);
    double *mu = (double *)malloc(sizeof(double) * (size_t)N);
    double *t = (double *)malloc(sizeof(double) * (size_t)N);
    double *d = (double *)malloc(sizeof(double) * (size_t)N);
    orc_laplacian(ndim, n, dx, r, w, m, lap);
    for (int64_t i = 0; i < N; ++i) mu[i] = (c2 * (m[i] * m[i] * m[i]) - c1 * m[i]) - lap[i];
    /* dm/dt = L mu - c3 sum_a D1_a (m j_a) */
    orc_laplacian(ndim, n, dx, r, w, mu, rhs);
    for (int a = 0; a < ndim; ++a) {
        const double *ja = in + (int64_t)(1 + a) * N;
        for (int64_t i = 0; i < N; ++i) t[i] = m[i] * ja[i];
        orc_d1(a, n, dx, r, w1, t, d);
        for (int64_t i = 0; i < N; ++i) rhs[i] = rhs[i] - c3 * d[i];
    }
    /* dj_a/dt = L j_a + c3 m D1_a mu */
    for (int a = 0; a < ndim; ++a) {
        const double *ja = in + (int64_t)(1 + a) * N;
        double *ra = rhs + (int64_t)(1 + a) * N;
        orc_laplacian(ndim, n, dx, r, w, ja, ra);
        orc_d1(a, n, dx, r, w1, mu, d);
        for (int64_t i = 0; i < N; ++i) ra[i] = ra[i] + c3 * (m[i] * d[i]);
    }
    free(lap);
    free(mu);
    free(t);
    free(d);
}

/* nsteps forward-Euler steps of orc_rhs_mh, in place on 1 + ndim fields. */
void orc_run_mh(int ndim, const int64_t n[3], double dx, double dt, int r, const double *w,
                const double *w1, const double *params, double *fields, int64_t nsteps)
{
    const int64_t M = nsites(n) * (1 + ndim);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)M);
    for (int64_t s = 0; s < nsteps; ++s) {
        orc_rhs_mh(ndim, n, dx, r, w, w1, params, fields, rhs);
        for (int64_t i = 0; i < M; ++i) fields[i] = fields[i] + dt * rhs[i];
    }
    free(rhs);
}

/* nsteps forward-Euler steps of orc_rhs_chd, in place. */
void orc_run_chd(int ndim, const int64_t n[3], double dx, double dt, int r, const double *w,
                 int r4, const double *w4, const double *params, double *field, int64_t nsteps)
{
    const int64_t N = nsites(n);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)N);
    for (int64_t s = 0; s < nsteps; ++s) {
        orc_rhs_chd(ndim, n, dx, r, w, r4, w4, params, field, rhs);
        for (int64_t i = 0; i < N; ++i) field[i] = field[i] + dt * rhs[i];
    }
    free(rhs);
}

/*
 * nsteps forward-Euler steps x <- x + dt * rhs(x), in place on `fields`
 * (nfields * nsites doubles).  Returns 0 on success, -1 on a bad kind.
 */
int orc_run(int kind, int ndim, const int64_t n[3], double dx, double dt,
            int r, const double *w, const double *params,
            double *fields, int64_t nsteps)
{
    if (kind != ORC_AC && kind != ORC_CH && kind != ORC_GS && kind != ORC_MC) return -1;
    const int64_t M = nsites(n) * nfields_of(kind);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)M);
    for (int64_t s = 0; s < nsteps; ++s) {
        orc_rhs(kind, ndim, n, dx, r, w, params, fields, rhs);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < M; ++i) fields[i] = fields[i] + dt * rhs[i];
    }
    free(rhs);
    return 0;
}

/*
 * Exact summation.  The running sum is kept as a list of non-overlapping
 * doubles whose exact sum equals the exact sum of the inputs so far
 * (Shewchuk's grow-expansion, "Adaptive Precision Floating-Point Arithmetic
 * and Fast Robust Geometric Predicates", 1997, Sec. 2); at the end the list
 * is rounded once to the nearest double (ties to even).  The inputs must be
 * finite.  Returns the correctly rounded exact sum.
 */
#define ORC_MAXPART 2100
double orc_exact_sum(const double *x, int64_t count, int64_t stride)
{
    double part[ORC_MAXPART];
    int np = 0;
    for (int64_t t = 0; t < count; ++t) {
        double v = x[t * stride];
        int k = 0;
        for (int q = 0; q < np; ++q) {
            double y = part[q];
            if (fabs(v) < fabs(y)) { double tmp = v; v = y; y = tmp; }
            const double hi = v + y;
            const double lo = y - (hi - v);
            if (lo != 0.0) part[k++] = lo;
            v = hi;
        }
        part[k++] = v;
        np = k;
    }
    /* Round the expansion (increasing magnitude, non-overlapping) once. */
    if (np == 0) return 0.0;
    int q = np - 1;
    double hi = part[q];
    double lo = 0.0;
    while (q > 0) {
        const double y = part[--q];
        const double s = hi + y;
        const double yr = s - hi;
        lo = y - yr;
        hi = s;
        if (lo != 0.0) break;
    }
    /* Half-way case: the remaining partials decide the direction. */
    if (q > 0 && ((lo < 0.0 && part[q - 1] < 0.0) || (lo > 0.0 && part[q - 1] > 0.0))) {
        const double y = lo * 2.0;
        const double s = hi + y;
        if (y == s - hi) hi = s;
    }
    return hi;
}

/*
 * Per-site free-energy density of the Landau functional behind Eqs. model-a
 * and model-b:  f = -(c1/2) x^2 + (c2/4) x^4 + (1/2)|grad x|^2.  The gradient
 * term is the quadratic form of the same discrete operator, -(1/2) x (L x),
 * so that the derivative of sum_i e_i with respect to x_i is
 * -(L x)_i - c1 x_i + c2 x_i^3 (the variational derivative of the paper's
 * functional-derivative identity, reduced form).
 *   e_i = -(1/2) x_i (L x)_i + (c2/4) x_i^4 - (c1/2) x_i^2
 */
void orc_energy_density(int ndim, const int64_t n[3], double dx, int r,
                        const double *w, const double *params,
                        const double *x, double *e)
{
    const int64_t N = nsites(n);
    const double c1 = params[0], c2 = params[1];
    double *lap = (double *)malloc(sizeof(double) * (size_t)N);
    orc_laplacian(ndim, n, dx, r, w, x, lap);
    for (int64_t i = 0; i < N; ++i) {
        const double v = x[i];
        e[i] = ((-0.5 * v) * lap[i] + (0.25 * c2) * (v * v * v * v)) - (0.5 * c1) * (v * v);
    }
    free(lap);
}

/*
 * Reductions of a state: mass[f] = dx^d * sum_i x_f,i for every field and,
 * for AC/CH, energy = dx^d * sum_i e_i.  Each sum is exact, then rounded
 * once, then scaled.  Returns the number of non-finite values in the state.
 */
int64_t orc_reduce(int kind, int ndim, const int64_t n[3], double dx, int r,
                   const double *w, const double *params,
                   const double *fields, double *mass, double *energy)
{
    const int64_t N = nsites(n);
    const int nf = nfields_of(kind);
    double vol = 1.0;
    for (int a = 0; a < ndim; ++a) vol *= dx;
    int64_t bad = 0;
    for (int64_t i = 0; i < N * nf; ++i)
        if (!isfinite(fields[i])) ++bad;
    if (bad) return bad;
    for (int f = 0; f < nf; ++f) mass[f] = vol * orc_exact_sum(fields + f * N, N, 1);
    if ((kind == ORC_AC || kind == ORC_CH) && energy) {
        double *e = (double *)malloc(sizeof(double) * (size_t)N);
        orc_energy_density(ndim, n, dx, r, w, params, fields, e);
        *energy = vol * orc_exact_sum(e, N, 1);
        free(e);
    }
    return 0;
}
