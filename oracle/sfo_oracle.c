/*
 * Plain FP64 CPU oracle for the Fourier split-operator step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library: it has its own FFT, its own phase evaluation and its
 * own reductions, all in double precision, written for readability rather
 * than speed (the only concession to speed is an OpenMP loop over the
 * independent lines of a multi-dimensional transform).
 *
 * What it follows (Bauke & Keitel, "Accelerating the Fourier split operator
 * method via graphics processing units"):
 *   - Sec. 2.1, eqs. (U_split), (step_t_to_t+dt), (step_t_to_t+dt_F): one
 *     step is  U_A1(1/2) F^-1 { U~_A2(1) F { U_A1(1/2) w } }, second order.
 *     Both half steps use the same step-integrated potential (reading:
 *     midpoint/step integral, the same for both halves).
 *   - Sec. 2.1: the continuous transform is replaced by the DFT on a regular
 *     lattice.  Reading: unnormalised forward DFT exp(-2 pi i j m / N), the
 *     inverse carries 1/N_tot; momenta k_m = 2 pi m / L with m in
 *     [-N/2, N/2) in FFT order, so the Nyquist mode is negative.
 *   - Sec. 2.2: Schroedinger split.  Real-space factor
 *     exp(-(i/hbar) delta Int V dt'), momentum-space factor
 *     exp(-(i/hbar) tau |hbar k|^2 / (2m)) (dipole approximation, length
 *     gauge: the field enters the potential as x.E(t)).
 *   - Sec. 2.3: Dirac split for d = 2 (4-spinor, Dirac representation).
 *     Real-space factor = scalar phase of the potential times
 *     exp(i delta q c Abar . alpha / hbar) evaluated with the closed form of
 *     eq. (exp_alpha); momentum-space factor eq. (U_A_2_DE) evaluated as
 *     cos(E tau/hbar) I - i sin(E tau/hbar) H(p)/E, which equals the
 *     diagonalised form u^dagger diag(e^{-iE tau}, e^{+iE tau}) u of the paper
 *     because H(p)^2 = E(p)^2 I by the Dirac algebra.
 *   - Adjoint (gradient of a real loss through the unitary steps): derived
 *     from the step above; computed here from a STORED forward trajectory,
 *     a different algorithm from the GPU's reverse recomputation.
 *
 * Layout shared with the callers (an interface, not code): a state is
 * [comp][z][y][x] with x fastest; axis a = 0 is x.  x_j = xmin + j*dx with
 * dx = (xmax - xmin)/n, right end excluded.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------ FFT --
 * Iterative radix-2 Cooley-Tukey transform, unnormalised:
 *   out[m] = sum_j in[j] exp(sign * 2 pi i j m / n),  sign = -1 forward.
 * Twiddles come from cos/sin of each index directly (no recurrence). */

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

typedef struct {
    int64_t n;
    int sign;
    cplx *w; /* w[k] = exp(sign 2 pi i k / n), k < n/2 */
} fft_plan;

static int plan_make(fft_plan *p, int64_t n, int sign)
{
    p->n = n;
    p->sign = sign;
    p->w = (cplx *)malloc(sizeof(cplx) * (size_t)(n / 2 + 1));
    if (!p->w) return -1;
    for (int64_t k = 0; k < n / 2 + 1; k++) {
        double ang = (double)sign * TWO_PI * (double)k / (double)n;
        p->w[k] = cos(ang) + I * sin(ang);
    }
    return 0;
}

static void plan_free(fft_plan *p) { free(p->w); p->w = NULL; }

static void fft_line(const fft_plan *p, cplx *a)
{
    const int64_t n = p->n;
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < n; i++) {
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    /* butterflies: sub-transforms of length len combine two halves */
    for (int64_t len = 2; len <= n; len <<= 1) {
        const int64_t half = len / 2, step = n / len;
        for (int64_t i = 0; i < n; i += len) {
            for (int64_t k = 0; k < half; k++) {
                cplx w = p->w[k * step];
                cplx u = a[i + k];
                cplx v = a[i + k + half] * w;
                a[i + k] = u + v;
                a[i + k + half] = u - v;
            }
        }
    }
}

/* n-dimensional transform of one component: 1-D transforms along every axis. */
static int fft_nd(cplx *a, int ndim, const int64_t *n, int sign)
{
    int64_t ntot = 1;
    for (int d = 0; d < ndim; d++) ntot *= n[d];
    for (int ax = 0; ax < ndim; ax++) {
        const int64_t len = n[ax];
        if (len == 1) continue;
        int64_t stride = 1;
        for (int d = 0; d < ax; d++) stride *= n[d];
        const int64_t nlines = ntot / len;
        fft_plan p;
        if (plan_make(&p, len, sign)) return -1;
        int fail = 0;
#pragma omp parallel
        {
            cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)len);
            if (!buf) {
#pragma omp atomic write
                fail = 1;
            } else {
#pragma omp for schedule(static)
                for (int64_t L = 0; L < nlines; L++) {
                    const int64_t inner = L % stride, outer = L / stride;
                    const int64_t base = inner + outer * stride * len;
                    for (int64_t j = 0; j < len; j++) buf[j] = a[base + j * stride];
                    fft_line(&p, buf);
                    for (int64_t j = 0; j < len; j++) a[base + j * stride] = buf[j];
                }
                free(buf);
            }
        }
        plan_free(&p);
        if (fail) return -1;
    }
    return 0;
}

int orc_fft(cplx *a, int ndim, const int64_t *n, int sign, int ncomp)
{
    if (ndim < 1 || ndim > 3 || (sign != 1 && sign != -1) || ncomp < 1) return -1;
    int64_t ntot = 1;
    for (int d = 0; d < ndim; d++) {
        if (!is_pow2(n[d])) return -1;
        ntot *= n[d];
    }
    for (int c = 0; c < ncomp; c++)
        if (fft_nd(a + (size_t)c * ntot, ndim, n, sign)) return -1;
    return 0;
}

/* --------------------------------------------------------------- grids -- */

typedef struct {
    int ndim;
    int64_t n[3];
    int64_t ntot;
    double xmin[3], dx[3];
    double kmul[3]; /* k_m = kmul * m, kmul = 2 pi / L */
} grid;

static int grid_make(grid *g, int ndim, const int64_t *n, const double *xmin, const double *xmax)
{
    if (ndim < 1 || ndim > 3) return -1;
    g->ndim = ndim;
    g->ntot = 1;
    for (int d = 0; d < 3; d++) {
        if (d < ndim) {
            if (!is_pow2(n[d]) || !(xmax[d] > xmin[d])) return -1;
            g->n[d] = n[d];
            g->xmin[d] = xmin[d];
            g->dx[d] = (xmax[d] - xmin[d]) / (double)n[d];
            g->kmul[d] = TWO_PI / (xmax[d] - xmin[d]);
        } else {
            g->n[d] = 1;
            g->xmin[d] = 0.0;
            g->dx[d] = 0.0;
            g->kmul[d] = 0.0;
        }
        g->ntot *= g->n[d];
    }
    return 0;
}

/* coordinates of flat index i */
static void grid_x(const grid *g, int64_t i, double *x)
{
    int64_t r = i;
    for (int d = 0; d < 3; d++) {
        int64_t j = r % g->n[d];
        r /= g->n[d];
        x[d] = g->xmin[d] + (double)j * g->dx[d];
    }
}

/* wave numbers of flat index i in FFT order, Nyquist negative */
static void grid_k(const grid *g, int64_t i, double *k)
{
    int64_t r = i;
    for (int d = 0; d < 3; d++) {
        int64_t j = r % g->n[d];
        r /= g->n[d];
        int64_t m = (j < g->n[d] / 2) ? j : j - g->n[d];
        k[d] = g->kmul[d] * (double)m;
    }
}

static double grid_dv(const grid *g)
{
    double v = 1.0;
    for (int d = 0; d < g->ndim; d++) v *= g->dx[d];
    return v;
}

/* -------------------------------------------------------- reductions --
 * ||psi||^2 = dV sum |psi|^2 ;  <a|b> = dV sum conj(a) b  (all components) */

int orc_norm(int ndim, const int64_t *n, const double *xmin, const double *xmax, int ncomp,
             const cplx *psi, double *out)
{
    grid g;
    if (grid_make(&g, ndim, n, xmin, xmax)) return -1;
    double s = 0.0;
    for (int64_t i = 0; i < g.ntot * ncomp; i++) s += creal(psi[i] * conj(psi[i]));
    *out = s * grid_dv(&g);
    return 0;
}

int orc_overlap(int ndim, const int64_t *n, const double *xmin, const double *xmax, int ncomp,
                const cplx *a, const cplx *b, double *out2)
{
    grid g;
    if (grid_make(&g, ndim, n, xmin, xmax)) return -1;
    cplx s = 0.0;
    for (int64_t i = 0; i < g.ntot * ncomp; i++) s += conj(a[i]) * b[i];
    s *= grid_dv(&g);
    out2[0] = creal(s);
    out2[1] = cimag(s);
    return 0;
}

/* ------------------------------------------------------- Schroedinger --
 * Potential energy over step n:  Int_{t_n}^{t_n+tau} V dt' = tau V0(x) + x . Ebar_n
 * (length gauge, electron charge q = -1 folded in: V = V0 + x.E(t)).
 * Half step: psi <- exp(-i/(2 hbar) [tau V0 + x.Ebar_n]) psi.
 * Kinetic:   psit <- exp(-i hbar tau |k|^2 / (2 m)) psit / N_tot.
 * dir = +1 applies S_n; dir = -1 applies S_n^{-1} = S_n^dagger (all phases
 * conjugated; the step is palindromic, so the order is unchanged). */

typedef struct {
    grid g;
    double dt, mass, hbar;
    const double *V0;
    const double *ebar; /* nsteps_total x ndim, or NULL */
    /* velocity gauge (abar != NULL; ebar is then NULL): per step n the
     * integrals abar[n ndim + a] = int A_a dt' and a2bar[n] = int |A|^2 dt'
     * over the step, and the charge q */
    const double *abar, *a2bar;
    double charge;
} schro;

static double schro_theta(const schro *s, int64_t i, int64_t step)
{
    double x[3];
    grid_x(&s->g, i, x);
    double v = s->dt * s->V0[i];
    if (s->ebar)
        for (int d = 0; d < s->g.ndim; d++) v += x[d] * s->ebar[step * s->g.ndim + d];
    return v / (2.0 * s->hbar);
}

static void schro_half(const schro *s, cplx *psi, int64_t step, int dir)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->g.ntot; i++) {
        double th = schro_theta(s, i, step);
        psi[i] *= cexp(-I * (double)dir * th);
    }
}

/* Kinetic factor of step `step` (the momentum-space operator of the
 * dipole-approximation split, eq. SE_K): with p = hbar k,
 *   exp(-(i/hbar) int_t^{t+tau} (p - q A(t'))^2 / (2m) dt')
 *   = exp(-i/(2 m hbar) [tau p^2 - 2 q p.Abar_n + q^2 A2bar_n]),
 * which is exp(-i hbar tau |k|^2 / (2m)) in the length gauge (A = 0). */
static void schro_kinetic(const schro *s, cplx *psi, int64_t step, int dir)
{
    const double inv = 1.0 / (double)s->g.ntot;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->g.ntot; i++) {
        double k[3];
        grid_k(&s->g, i, k);
        double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        double ph = s->hbar * s->dt * k2 / (2.0 * s->mass);
        if (s->abar) {
            double pa = 0.0;
            for (int d = 0; d < s->g.ndim; d++) pa += s->hbar * k[d] * s->abar[step * s->g.ndim + d];
            ph += (-2.0 * s->charge * pa + s->charge * s->charge * s->a2bar[step]) / (2.0 * s->mass * s->hbar);
        }
        psi[i] *= cexp(-I * (double)dir * ph) * inv;
    }
}

static int schro_step(const schro *s, cplx *psi, int64_t step, int dir)
{
    schro_half(s, psi, step, dir);
    if (fft_nd(psi, s->g.ndim, s->g.n, -1)) return -1;
    schro_kinetic(s, psi, step, dir);
    if (fft_nd(psi, s->g.ndim, s->g.n, +1)) return -1;
    schro_half(s, psi, step, dir);
    return 0;
}

/* Forward: steps step0 .. step0+nsteps-1.  Inverse (dir=-1): undoes those
 * steps, last first.  norms (optional, nsteps+1 doubles) gets ||psi||^2 at
 * every step boundary visited. */
int orc_schrodinger(int ndim, const int64_t *n, const double *xmin, const double *xmax, double dt,
                    double mass, double hbar, const double *V0, const double *ebar, cplx *psi,
                    int64_t step0, int64_t nsteps, int dir, double *norms)
{
    schro s;
    if (grid_make(&s.g, ndim, n, xmin, xmax) || !V0 || !psi || nsteps < 0 || step0 < 0 ||
        (dir != 1 && dir != -1) || !(mass > 0) || !(hbar > 0))
        return -1;
    s.dt = dt;
    s.mass = mass;
    s.hbar = hbar;
    s.V0 = V0;
    s.ebar = ebar;
    s.abar = s.a2bar = NULL;
    s.charge = -1.0;
    if (norms) orc_norm(ndim, n, xmin, xmax, 1, psi, &norms[0]);
    for (int64_t j = 0; j < nsteps; j++) {
        int64_t step = (dir > 0) ? step0 + j : step0 + nsteps - 1 - j;
        if (schro_step(&s, psi, step, dir)) return -1;
        if (norms) orc_norm(ndim, n, xmin, xmax, 1, psi, &norms[j + 1]);
    }
    return 0;
}

/* Velocity-gauge steps (no scalar field term): the potential half steps use
 * tau V0 only, the kinetic factor carries the vector potential of the
 * field through its per-step integrals abar (nsteps_total x ndim) and a2bar
 * (nsteps_total).  Forward only. */
int orc_schrodinger_velocity(int ndim, const int64_t *n, const double *xmin, const double *xmax, double dt,
                             double mass, double hbar, double charge, const double *V0, const double *abar,
                             const double *a2bar, cplx *psi, int64_t step0, int64_t nsteps)
{
    schro s;
    if (grid_make(&s.g, ndim, n, xmin, xmax) || !V0 || !psi || !abar || !a2bar || nsteps < 0 || step0 < 0 ||
        !(mass > 0) || !(hbar > 0))
        return -1;
    s.dt = dt;
    s.mass = mass;
    s.hbar = hbar;
    s.V0 = V0;
    s.ebar = NULL;
    s.abar = abar;
    s.a2bar = a2bar;
    s.charge = charge;
    for (int64_t j = 0; j < nsteps; j++)
        if (schro_step(&s, psi, step0 + j, 1)) return -1;
    return 0;
}

/* Gradient of a real loss L(psi_T) through nsteps Schroedinger steps.
 * Input gT = 2 dL/d conj(psi_T) (the convention of complex autograd).
 * With S_n = P_n A P_n, P_n = diag(exp(-i theta_n(x))), A unitary:
 *   g_n = S_n^dagger g_{n+1},
 *   dL/dtheta_n(x) = Im( conj(g_{n+1}) psi_{n+1} + conj(g_n) psi_n )(x),
 *   dL/dEbar_{n,a} = sum_x x_a/(2 hbar) dL/dtheta_n(x),
 *   dL/dV0(x)      = sum_n tau/(2 hbar) dL/dtheta_n(x).
 * The forward trajectory psi_0..psi_S is STORED here (memory (S+1) N_tot);
 * on exit psi0_g holds g_0 = dL/d conj(psi_0) * 2. */
int orc_schrodinger_adjoint(int ndim, const int64_t *n, const double *xmin, const double *xmax,
                            double dt, double mass, double hbar, const double *V0, const double *ebar,
                            const cplx *psi0, cplx *g, int64_t step0, int64_t nsteps,
                            double *dL_debar, double *dL_dV0)
{
    schro s;
    if (grid_make(&s.g, ndim, n, xmin, xmax) || !V0 || !psi0 || !g || nsteps < 0 || step0 < 0)
        return -1;
    s.dt = dt;
    s.mass = mass;
    s.hbar = hbar;
    s.V0 = V0;
    s.ebar = ebar;
    s.abar = s.a2bar = NULL;
    s.charge = -1.0;
    const int64_t N = s.g.ntot;
    cplx *traj = (cplx *)malloc(sizeof(cplx) * (size_t)N * (size_t)(nsteps + 1));
    if (!traj) return -2;
    memcpy(traj, psi0, sizeof(cplx) * (size_t)N);
    for (int64_t j = 0; j < nsteps; j++) {
        memcpy(traj + (size_t)N * (j + 1), traj + (size_t)N * j, sizeof(cplx) * (size_t)N);
        if (schro_step(&s, traj + (size_t)N * (j + 1), step0 + j, +1)) { free(traj); return -1; }
    }
    if (dL_dV0) memset(dL_dV0, 0, sizeof(double) * (size_t)N);
    if (dL_debar) memset(dL_debar, 0, sizeof(double) * (size_t)nsteps * ndim);
    double *im_next = (double *)malloc(sizeof(double) * (size_t)N);
    if (!im_next) { free(traj); return -2; }
    {
        const cplx *pT = traj + (size_t)N * nsteps;
        for (int64_t i = 0; i < N; i++) im_next[i] = cimag(conj(g[i]) * pT[i]);
    }
    for (int64_t j = nsteps - 1; j >= 0; j--) {
        /* g_j = S_j^dagger g_{j+1} (adjoint of a unitary step = its inverse) */
        if (schro_step(&s, g, step0 + j, -1)) { free(im_next); free(traj); return -1; }
        const cplx *pj = traj + (size_t)N * j;
        for (int64_t i = 0; i < N; i++) {
            double im_here = cimag(conj(g[i]) * pj[i]);
            double dth = im_next[i] + im_here;
            if (dL_dV0) dL_dV0[i] += dt / (2.0 * hbar) * dth;
            if (dL_debar) {
                double x[3];
                grid_x(&s.g, i, x);
                for (int d = 0; d < ndim; d++) dL_debar[j * ndim + d] += x[d] / (2.0 * hbar) * dth;
            }
            im_next[i] = im_here;
        }
    }
    free(im_next);
    free(traj);
    return 0;
}

/* Gradient of a real loss L(psi_T) through nsteps velocity-gauge steps
 * (orc_schrodinger_velocity), from a STORED FP64 trajectory.  Input gT =
 * 2 dL/d conj(psi_T); on exit g holds the same at psi_0.  With
 * S_n = P F^-1 K_n F P and K_n = exp(-i/(2 m hbar) [tau p^2 - 2 q p.Abar_n +
 * q^2 A2bar_n]) (p = hbar k), the derivatives of K_n are
 *   dK_n/dAbar_{n,a} = (i q k_a / m) K_n,   dK_n/dA2bar_n = (-i q^2 / (2 m hbar)) K_n,
 * so, written out step by step,
 *   dL/dAbar_{n,a} = Re sum_x conj(g_{n+1}) [P F^-1 (i q k_a / m) K_n F P psi_n](x),
 *   dL/dA2bar_n   = Re sum_x conj(g_{n+1}) [P F^-1 (-i q^2/(2 m hbar)) K_n F P psi_n](x),
 * and dL/dV0 as in the length gauge (the half factors are the same). */
int orc_schrodinger_velocity_adjoint(int ndim, const int64_t *n, const double *xmin, const double *xmax, double dt,
                                     double mass, double hbar, double charge, const double *V0, const double *abar,
                                     const double *a2bar, const cplx *psi0, cplx *g, int64_t step0, int64_t nsteps,
                                     double *dL_dabar, double *dL_da2bar, double *dL_dV0)
{
    schro s;
    if (grid_make(&s.g, ndim, n, xmin, xmax) || !V0 || !psi0 || !g || !abar || !a2bar || nsteps < 0 ||
        step0 < 0 || !(mass > 0) || !(hbar > 0))
        return -1;
    s.dt = dt;
    s.mass = mass;
    s.hbar = hbar;
    s.V0 = V0;
    s.ebar = NULL;
    s.abar = abar;
    s.a2bar = a2bar;
    s.charge = charge;
    const int64_t N = s.g.ntot;
    cplx *traj = (cplx *)malloc(sizeof(cplx) * (size_t)N * (size_t)(nsteps + 1));
    cplx *u = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    cplx *du = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    double *im_next = (double *)malloc(sizeof(double) * (size_t)N);
    if (!traj || !u || !du || !im_next) {
        free(traj), free(u), free(du), free(im_next);
        return -2;
    }
    int rc = 0;
    memcpy(traj, psi0, sizeof(cplx) * (size_t)N);
    for (int64_t j = 0; j < nsteps && !rc; j++) {
        memcpy(traj + (size_t)N * (j + 1), traj + (size_t)N * j, sizeof(cplx) * (size_t)N);
        rc = schro_step(&s, traj + (size_t)N * (j + 1), step0 + j, +1);
    }
    if (dL_dV0) memset(dL_dV0, 0, sizeof(double) * (size_t)N);
    {
        const cplx *pT = traj + (size_t)N * nsteps;
        for (int64_t i = 0; i < N; i++) im_next[i] = cimag(conj(g[i]) * pT[i]);
    }
    for (int64_t j = nsteps - 1; j >= 0 && !rc; j--) {
        const int64_t step = step0 + j;
        const cplx *pj = traj + (size_t)N * j;
        /* K_n F P psi_n (with the 1/N of the inverse transform) */
        memcpy(u, pj, sizeof(cplx) * (size_t)N);
        schro_half(&s, u, step, +1);
        if ((rc = fft_nd(u, ndim, s.g.n, -1))) break;
        schro_kinetic(&s, u, step, +1);
        for (int d = 0; d <= ndim; d++) {
            /* d < ndim: the factor i q k_d / m;  d = ndim: -i q^2 / (2 m hbar) */
            for (int64_t i = 0; i < N; i++) {
                double k[3];
                grid_k(&s.g, i, k);
                const cplx f = d < ndim ? I * charge * k[d] / mass : -I * charge * charge / (2.0 * mass * hbar);
                du[i] = f * u[i];
            }
            if ((rc = fft_nd(du, ndim, s.g.n, +1))) break;
            schro_half(&s, du, step, +1);
            double acc = 0.0;
            for (int64_t i = 0; i < N; i++) acc += creal(conj(g[i]) * du[i]);
            if (d < ndim) {
                if (dL_dabar) dL_dabar[j * ndim + d] = acc;
            } else if (dL_da2bar) {
                dL_da2bar[j] = acc;
            }
        }
        if (rc) break;
        /* g_j = S_j^dagger g_{j+1} */
        if ((rc = schro_step(&s, g, step, -1))) break;
        for (int64_t i = 0; i < N; i++) {
            const double im_here = cimag(conj(g[i]) * pj[i]);
            if (dL_dV0) dL_dV0[i] += dt / (2.0 * hbar) * (im_next[i] + im_here);
            im_next[i] = im_here;
        }
    }
    free(traj), free(u), free(du), free(im_next);
    return rc ? -1 : 0;
}

/* ------------------------------------------------------------ Dirac 2D --
 * Dirac representation (eq. Dirac_repr); 4-spinor stored as 4 planes. */

static void dirac_matrices(cplx a1[4][4], cplx a2[4][4], cplx b[4][4])
{
    memset(a1, 0, sizeof(cplx) * 16);
    memset(a2, 0, sizeof(cplx) * 16);
    memset(b, 0, sizeof(cplx) * 16);
    a1[0][3] = 1; a1[1][2] = 1; a1[2][1] = 1; a1[3][0] = 1;
    a2[0][3] = -I; a2[1][2] = I; a2[2][1] = -I; a2[3][0] = I;
    b[0][0] = 1; b[1][1] = 1; b[2][2] = -1; b[3][3] = -1;
}

static void mat4_apply(cplx m[4][4], cplx v[4])
{
    cplx r[4];
    for (int i = 0; i < 4; i++) {
        r[i] = 0;
        for (int j = 0; j < 4; j++) r[i] += m[i][j] * v[j];
    }
    for (int i = 0; i < 4; i++) v[i] = r[i];
}

typedef struct {
    grid g;
    double dt, mass, charge, c, hbar;
    const double *V0;
    const double *abar_y; /* nsteps_total x n[0]: Int A_y dt' over step n, as a function of x */
    cplx al1[4][4], al2[4][4], be[4][4];
} dirac;

/* Real-space half step: exp(-i tau V0/(2 hbar)) * exp(i a alpha_2),
 * a = (1/2) q c Abar_y / hbar, exp(i a alpha_2) = cos a I + i sin a alpha_2
 * (eq. exp_alpha with a single component). dir = -1: the inverse. */
static void dirac_half(const dirac *s, cplx *psi, int64_t step, int dir)
{
    const int64_t N = s->g.ntot, nx = s->g.n[0];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        double a = 0.0;
        if (s->abar_y) a = 0.5 * s->charge * s->c * s->abar_y[step * nx + (i % nx)] / s->hbar;
        a *= (double)dir;
        cplx m[4][4];
        for (int r = 0; r < 4; r++)
            for (int q = 0; q < 4; q++) m[r][q] = (r == q ? cos(a) : 0.0) + I * sin(a) * s->al2[r][q];
        cplx ph = cexp(-I * (double)dir * s->dt * s->V0[i] / (2.0 * s->hbar));
        cplx v[4];
        for (int c = 0; c < 4; c++) v[c] = psi[c * N + i];
        mat4_apply(m, v);
        for (int c = 0; c < 4; c++) psi[c * N + i] = ph * v[c];
    }
}

/* Momentum-space step: exp(-i tau H(p)/hbar) / N_tot with
 * H(p) = c alpha.p + m c^2 beta, p = hbar k, E = sqrt(m^2 c^4 + c^2 p^2). */
static void dirac_kinetic(const dirac *s, cplx *psi, int dir)
{
    const int64_t N = s->g.ntot;
    const double inv = 1.0 / (double)N;
    const double mc2 = s->mass * s->c * s->c;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        double k[3];
        grid_k(&s->g, i, k);
        double px = s->hbar * k[0], py = s->hbar * k[1];
        double E = sqrt(mc2 * mc2 + s->c * s->c * (px * px + py * py));
        double ct = cos(E * s->dt / s->hbar), st = (double)dir * sin(E * s->dt / s->hbar);
        cplx u[4][4];
        for (int r = 0; r < 4; r++)
            for (int q = 0; q < 4; q++) {
                cplx H = s->c * (s->al1[r][q] * px + s->al2[r][q] * py) + mc2 * s->be[r][q];
                u[r][q] = (r == q ? ct : 0.0) - I * st / E * H;
            }
        cplx v[4];
        for (int c = 0; c < 4; c++) v[c] = psi[c * N + i];
        mat4_apply(u, v);
        for (int c = 0; c < 4; c++) psi[c * N + i] = v[c] * inv;
    }
}

int orc_dirac2d(const int64_t *n, const double *xmin, const double *xmax, double dt, double mass,
                double charge, double c, double hbar, const double *V0, const double *abar_y,
                cplx *psi, int64_t step0, int64_t nsteps, int dir)
{
    dirac s;
    if (grid_make(&s.g, 2, n, xmin, xmax) || !V0 || !psi || nsteps < 0 || step0 < 0 ||
        (dir != 1 && dir != -1) || !(c > 0) || !(hbar > 0))
        return -1;
    s.dt = dt;
    s.mass = mass;
    s.charge = charge;
    s.c = c;
    s.hbar = hbar;
    s.V0 = V0;
    s.abar_y = abar_y;
    dirac_matrices(s.al1, s.al2, s.be);
    const int64_t N = s.g.ntot;
    for (int64_t j = 0; j < nsteps; j++) {
        int64_t step = (dir > 0) ? step0 + j : step0 + nsteps - 1 - j;
        dirac_half(&s, psi, step, dir);
        for (int comp = 0; comp < 4; comp++)
            if (fft_nd(psi + comp * N, 2, s.g.n, -1)) return -1;
        dirac_kinetic(&s, psi, dir);
        for (int comp = 0; comp < 4; comp++)
            if (fft_nd(psi + comp * N, 2, s.g.n, +1)) return -1;
        dirac_half(&s, psi, step, dir);
    }
    return 0;
}

/* ------------------------------------------------------------ Dirac 1D --
 * Two-component Dirac equation on a line (the paper's one-dimensional Dirac
 * representation: alpha_1 = sigma_x, beta = sigma_z), 2-spinor stored as two
 * planes [2][N].  Real-space half step: exp(-i tau V0 / (2 hbar)) (cos a +
 * i sin a alpha_1), a = (1/2) q c Abar_1(x) / hbar (the one-dimensional form
 * of the interaction operator, delta = 1/2); momentum-space step: exp(-i tau
 * H(p) / hbar) / N with H(p) = c p alpha_1 + m c^2 beta, written as
 * cos(E tau/hbar) - i sin(E tau/hbar) H(p) / E since H(p)^2 = E^2. */
int orc_dirac1d(int64_t n, double xmin, double xmax, double dt, double mass, double charge, double c,
                double hbar, const double *V0, const double *abar, cplx *psi, int64_t step0, int64_t nsteps)
{
    grid g;
    int64_t nn[1] = {n};
    double lo[1] = {xmin}, hi[1] = {xmax};
    if (grid_make(&g, 1, nn, lo, hi) || !V0 || !psi || nsteps < 0 || step0 < 0 || !(c > 0) || !(hbar > 0))
        return -1;
    const double mc2 = mass * c * c, inv = 1.0 / (double)n;
    cplx *p0 = psi, *p1 = psi + n;
    for (int64_t j = 0; j < nsteps; j++) {
        const int64_t step = step0 + j;
        for (int half = 0; half < 2; half++) {
            for (int64_t i = 0; i < n; i++) {
                const double a = abar ? 0.5 * charge * c * abar[step * n + i] / hbar : 0.0;
                const cplx ph = cexp(-I * dt * V0[i] / (2.0 * hbar));
                const cplx u = p0[i], v = p1[i];
                p0[i] = ph * (cos(a) * u + I * sin(a) * v);
                p1[i] = ph * (I * sin(a) * u + cos(a) * v);
            }
            if (half == 1) break;
            if (fft_nd(p0, 1, g.n, -1) || fft_nd(p1, 1, g.n, -1)) return -1;
            for (int64_t i = 0; i < n; i++) {
                double k[3];
                grid_k(&g, i, k);
                const double p = hbar * k[0];
                const double E = sqrt(mc2 * mc2 + c * c * p * p);
                const double ct = cos(E * dt / hbar), st = sin(E * dt / hbar);
                /* cos - i sin/E [[mc2, c p], [c p, -mc2]] */
                const cplx u00 = ct - I * st * mc2 / E, u01 = -I * st * c * p / E, u11 = ct + I * st * mc2 / E;
                const cplx u = p0[i], v = p1[i];
                p0[i] = (u00 * u + u01 * v) * inv;
                p1[i] = (u01 * u + u11 * v) * inv;
            }
            if (fft_nd(p0, 1, g.n, +1) || fft_nd(p1, 1, g.n, +1)) return -1;
        }
    }
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
