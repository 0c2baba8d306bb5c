/* Exercise every entry point of the FP64 oracle on small grids, for a build
 * under AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
 * The checks here are coarse (round trips, norms); the oracle's accuracy is
 * pinned by the Python tests.  What this adds is that every array access of
 * the oracle stays in bounds and no arithmetic is undefined, including for
 * rejected arguments.  Exit status 0 and "oracle selftest ok" on success. */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

int orc_fft(cplx *a, int ndim, const int64_t *n, int sign, int ncomp);
int orc_norm(int ndim, const int64_t *n, const double *xmin, const double *xmax, int ncomp, const cplx *psi,
             double *out);
int orc_overlap(int ndim, const int64_t *n, const double *xmin, const double *xmax, int ncomp, const cplx *a,
                const cplx *b, double *out2);
int orc_schrodinger(int ndim, const int64_t *n, const double *xmin, const double *xmax, double dt, double mass,
                    double hbar, const double *V0, const double *ebar, cplx *psi, int64_t step0, int64_t nsteps,
                    int dir, double *norms);
int orc_schrodinger_velocity(int ndim, const int64_t *n, const double *xmin, const double *xmax, double dt,
                             double mass, double hbar, double charge, const double *V0, const double *abar,
                             const double *a2bar, cplx *psi, int64_t step0, int64_t nsteps);
int orc_schrodinger_adjoint(int ndim, const int64_t *n, const double *xmin, const double *xmax, double dt,
                            double mass, double hbar, const double *V0, const double *ebar, const cplx *psi0,
                            cplx *g, int64_t step0, int64_t nsteps, double *dL_debar, double *dL_dV0);
int orc_dirac2d(const int64_t *n, const double *xmin, const double *xmax, double dt, double mass, double charge,
                double c, double hbar, const double *V0, const double *abar_y, cplx *psi, int64_t step0,
                int64_t nsteps, int dir);
int orc_dirac1d(int64_t n, double xmin, double xmax, double dt, double mass, double charge, double c, double hbar,
                const double *V0, const double *abar, cplx *psi, int64_t step0, int64_t nsteps);

static int failures = 0;

static void check(int cond, const char *what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s\n", what);
        failures++;
    }
}

/* exactly sized heap buffers, so that ASan sees any access past their ends */
static cplx *cbuf(int64_t n)
{
    cplx *p = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!p) abort();
    return p;
}
static double *dbuf(int64_t n)
{
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    if (!p) abort();
    return p;
}

static void fill(cplx *p, int64_t n, unsigned seed)
{
    srand(seed);
    for (int64_t i = 0; i < n; i++)
        p[i] = (rand() / (double)RAND_MAX - 0.5) + I * (rand() / (double)RAND_MAX - 0.5);
}

static double max_diff(const cplx *a, const cplx *b, int64_t n, double scale)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; i++) {
        const double d = cabs(a[i] * scale - b[i]);
        if (d > m) m = d;
    }
    return m;
}

static void test_fft(void)
{
    const int64_t shapes[3][3] = {{16, 1, 1}, {8, 4, 1}, {4, 8, 2}};
    for (int nd = 1; nd <= 3; nd++) {
        const int64_t *n = shapes[nd - 1];
        const int64_t N = n[0] * n[1] * n[2];
        for (int ncomp = 1; ncomp <= 2; ncomp++) {
            cplx *a = cbuf(N * ncomp), *b = cbuf(N * ncomp);
            fill(a, N * ncomp, 1u + (unsigned)nd);
            memcpy(b, a, sizeof(cplx) * (size_t)(N * ncomp));
            check(orc_fft(a, nd, n, -1, ncomp) == 0, "fft forward");
            check(orc_fft(a, nd, n, +1, ncomp) == 0, "fft inverse");
            check(max_diff(a, b, N * ncomp, 1.0 / (double)N) < 1e-13, "fft round trip");
            free(a);
            free(b);
        }
    }
    const int64_t bad[1] = {12};
    cplx *a = cbuf(12);
    fill(a, 12, 3);
    check(orc_fft(a, 1, bad, -1, 1) != 0, "fft rejects a length that is not a power of two");
    check(orc_fft(a, 4, bad, -1, 1) != 0, "fft rejects ndim 4");
    check(orc_fft(a, 1, bad, 2, 1) != 0, "fft rejects sign 2");
    free(a);
}

static void test_schrodinger(void)
{
    const int64_t shapes[3][3] = {{32, 1, 1}, {16, 8, 1}, {8, 8, 4}};
    const double lo[3] = {-4.0, -3.0, -2.0}, hi[3] = {4.0, 3.0, 2.0};
    for (int nd = 1; nd <= 3; nd++) {
        const int64_t *n = shapes[nd - 1];
        const int64_t N = n[0] * n[1] * n[2];
        const int64_t S = 5;
        cplx *psi = cbuf(N), *p0 = cbuf(N), *g = cbuf(N);
        double *V0 = dbuf(N), *ebar = dbuf(S * nd), *norms = dbuf(S + 1);
        for (int64_t i = 0; i < N; i++) V0[i] = 0.1 * (double)(i % 7);
        for (int64_t i = 0; i < S * nd; i++) ebar[i] = 0.01 * (double)(i % 3);
        fill(psi, N, 10u + (unsigned)nd);
        memcpy(p0, psi, sizeof(cplx) * (size_t)N);
        check(orc_schrodinger(nd, n, lo, hi, 0.05, 1.0, 1.0, V0, ebar, psi, 0, S, 1, norms) == 0, "schrodinger");
        check(fabs(norms[S] / norms[0] - 1.0) < 1e-12, "schrodinger norm");
        check(orc_schrodinger(nd, n, lo, hi, 0.05, 1.0, 1.0, V0, ebar, psi, 0, S, -1, NULL) == 0,
              "schrodinger inverse");
        check(max_diff(psi, p0, N, 1.0) < 1e-12, "schrodinger round trip");
        /* adjoint from the stored trajectory */
        double *dE = dbuf(S * nd), *dV = dbuf(N);
        fill(g, N, 20u + (unsigned)nd);
        check(orc_schrodinger_adjoint(nd, n, lo, hi, 0.05, 1.0, 1.0, V0, ebar, p0, g, 0, S, dE, dV) == 0, "adjoint");
        /* velocity gauge */
        double *abar = dbuf(S * nd), *a2bar = dbuf(S);
        for (int64_t i = 0; i < S * nd; i++) abar[i] = 0.02 * (double)(i % 5);
        for (int64_t s = 0; s < S; s++) a2bar[s] = 0.001 * (double)s;
        check(orc_schrodinger_velocity(nd, n, lo, hi, 0.05, 1.0, 1.0, -1.0, V0, abar, a2bar, psi, 0, S) == 0,
              "velocity gauge");
        double nrm = 0.0, ov[2] = {0.0, 0.0};
        check(orc_norm(nd, n, lo, hi, 1, psi, &nrm) == 0 && fabs(nrm / norms[0] - 1.0) < 1e-12,
              "velocity gauge norm");
        check(orc_overlap(nd, n, lo, hi, 1, p0, psi, ov) == 0, "overlap");
        check(orc_schrodinger(nd, n, lo, hi, -0.05, 1.0, 1.0, V0, ebar, psi, -1, S, 1, NULL) != 0,
              "schrodinger rejects a negative first step");
        free(psi), free(p0), free(g), free(V0), free(ebar), free(norms), free(dE), free(dV), free(abar), free(a2bar);
    }
}

static void test_dirac(void)
{
    const int64_t n[2] = {16, 8};
    const double lo[2] = {-2.0, -1.0}, hi[2] = {2.0, 1.0};
    const int64_t N = n[0] * n[1], S = 3;
    cplx *psi = cbuf(4 * N), *p0 = cbuf(4 * N);
    double *V0 = dbuf(N), *abar = dbuf(S * n[0]);
    for (int64_t i = 0; i < N; i++) V0[i] = -1.0 / sqrt(1.0 + (double)(i % 11));
    for (int64_t i = 0; i < S * n[0]; i++) abar[i] = 1e-4 * (double)(i % 13);
    fill(psi, 4 * N, 31);
    memcpy(p0, psi, sizeof(cplx) * (size_t)(4 * N));
    check(orc_dirac2d(n, lo, hi, 1e-3, 1.0, -1.0, 137.036, 1.0, V0, abar, psi, 0, S, 1) == 0, "dirac2d");
    check(orc_dirac2d(n, lo, hi, 1e-3, 1.0, -1.0, 137.036, 1.0, V0, abar, psi, 0, S, -1) == 0, "dirac2d inverse");
    check(max_diff(psi, p0, 4 * N, 1.0) < 1e-12, "dirac2d round trip");
    free(psi), free(p0), free(V0), free(abar);

    const int64_t m = 32;
    cplx *q = cbuf(2 * m);
    double *W0 = dbuf(m), *ab = dbuf(S * m);
    for (int64_t i = 0; i < m; i++) W0[i] = 0.5 * (double)(i % 4);
    for (int64_t i = 0; i < S * m; i++) ab[i] = 1e-3 * (double)(i % 9);
    fill(q, 2 * m, 41);
    double n0 = 0.0, n1 = 0.0;
    const int64_t mm[1] = {m};
    const double l1[1] = {-3.0}, h1[1] = {3.0};
    orc_norm(1, mm, l1, h1, 2, q, &n0);
    check(orc_dirac1d(m, -3.0, 3.0, 1e-3, 1.0, -1.0, 137.036, 1.0, W0, ab, q, 0, S) == 0, "dirac1d");
    orc_norm(1, mm, l1, h1, 2, q, &n1);
    check(fabs(n1 / n0 - 1.0) < 1e-12, "dirac1d norm");
    check(orc_dirac1d(12, -3.0, 3.0, 1e-3, 1.0, -1.0, 137.036, 1.0, W0, ab, q, 0, S) != 0,
          "dirac1d rejects a length that is not a power of two");
    free(q), free(W0), free(ab);
}

int main(void)
{
    test_fft();
    test_schrodinger();
    test_dirac();
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle selftest ok\n");
    return 0;
}
