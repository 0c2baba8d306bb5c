// C ABI layer: validation, library-owned device tables, and the pass
// sequences of a split-operator run.  See include/sfo.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "sfo.h"
#include "sfo_batch.h"
#include "sfo_impl.h"

using namespace sfo;

// Scratch memory of the allocation-free reverse sweep (sfo_adjoint_noalloc):
// the moment partials of every step boundary, 16 MiB.  Each device the
// library runs on holds its own copy until the process ends.  In host code
// this name only stands for the symbol: its device address on each device
// is looked up once (scratch_setup) and only that address is passed to
// kernels.
constexpr int64_t kNoAllocScratchDoubles = int64_t(1) << 21;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

thread_local std::string g_err;

sfo_status fail(sfo_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
sfo_status fail(sfo_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? SFO_E_NOMEM : SFO_E_HIP, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                   \
    } while (0)

// Debug injection of device allocation failures.  With the environment
// variable SFO_FAIL_ALLOC=<n> set, the n-th device allocation made within one
// ABI call on this thread (counted from 1; entry points that allocate start
// the count with an AllocCount) fails with hipErrorOutOfMemory without
// calling the runtime, so the error paths that release what a call had
// allocated can be exercised.
thread_local int t_alloc_seq = 0;
struct AllocCount {
    AllocCount() { t_alloc_seq = 0; }
};
template <typename T> hipError_t dev_malloc(T **p, size_t bytes)
{
    const int k = ++t_alloc_seq;
    if (const char *e = std::getenv("SFO_FAIL_ALLOC")) {
        if (k == std::atoi(e)) {
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
    }
    return hipMalloc((void **)p, bytes);
}

using check::is_pow2;

// Status and reason of a host-side argument check (sfo_validate.h) as the ABI reports it.
sfo_status checked(sfo_status s, const std::string &why)
{
    if (s != SFO_OK) g_err = why;
    return s;
}

// No C++ exception crosses the C ABI: a host allocation sized by the caller
// that fails reports SFO_E_NOMEM.
template <typename F> sfo_status no_throw(F &&f)
{
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return fail(SFO_E_NOMEM, "host allocation failed");
    } catch (const std::exception &ex) {
        return fail(SFO_E_INVALID, "%s", ex.what());
    }
}

// Device copy of a host table; on failure nothing stays allocated.
sfo_status upload_table(const double *host, size_t count, double **out)
{
    *out = nullptr;
    if (count == 0) return SFO_OK;
    double *d = nullptr;
    HIP_TRY(dev_malloc(&d, sizeof(double) * count));
    const hipError_t e = hipMemcpy(d, host, sizeof(double) * count, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(SFO_E_HIP, "table upload: %s", hipGetErrorString(e));
    }
    *out = d;
    return SFO_OK;
}

// Device address of `scratch` per device (null until looked up), and the
// error of a failed lookup.
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxScratchDevices] = {};
hipError_t g_scratch_err[kMaxScratchDevices] = {};

// Once per device, with that device current: look up the device address of
// the scratch array.  A failure is remembered and reported by the entry point
// that needs the array, not by the caller of this set-up.
void scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxScratchDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[dev] || g_scratch_err[dev] != hipSuccess) return;
    double *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        g_scratch_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        return;
    }
    g_scratch_dev[dev] = ptr;
}

}  // namespace

struct sfo_grid_s {
    sfo_grid_desc d{};
    hipStream_t st = nullptr;
    int dev = 0;  // the HIP device current at creation
    int ndim = 1;
    int ncomp = 1;
    int64_t n[3] = {1, 1, 1};
    int64_t ntot = 1;
    double dx[3] = {0, 0, 0};
    double dv = 1;
    bool c128 = false;
    void *V0 = nullptr;
    double v0max = 0.0;   // max |V0|, for the bound of the potential phase
    int row_var = 0;      // tile variants chosen for the x pass and the y/z passes
    int col_var[3] = {0, 0, 0};
    int row_var2 = -1;    // the same for the two-state passes of the reverse sweep (-1: as above)
    int col_var2[3] = {-1, -1, -1};
    std::vector<double> ebar;  // host copy, nsteps x ndim
    double *ebar_d = nullptr;  // device copy, nsteps x ndim (the 1-D and batched kernels read it)
    int64_t ebar_steps = 0;
    std::vector<double> abar;  // Dirac: nsteps x n[0]
    double *abar_d = nullptr;
    int64_t abar_steps = 0;
    void *tw[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};  // per-axis stage twiddles, radix 8 / 16
    double2 *kin[3] = {nullptr, nullptr, nullptr}; // per-axis kinetic factors (1/Ntot in axis 0)
    double *kvec[3] = {nullptr, nullptr, nullptr}; // per-axis wave numbers (Dirac)
    double2 *one = nullptr;                        // {1, 0}
    double *red = nullptr;                         // reduction partials + result
    // adjoint scratch: moment partials per step boundary and row work-group
    // (the autocorrelation run keeps its overlap partials here too)
    double *part = nullptr;
    int64_t part_cap = 0;
    void *chi_ref = nullptr;  // autocorrelation: reference state in k-space
    size_t chi_ref_bytes = 0;
    double2 *du = nullptr;  // 1-D Dirac: U00, U01, U11 of the momentum-space step per k
    double2 *eig_acc = nullptr;  // windowed eigenfunction: FP64 accumulator (ntot)
    // velocity gauge: per-step, per-axis kinetic factors (vsteps x n[a] each)
    double2 *vtab[3] = {nullptr, nullptr, nullptr};
    int64_t vsteps = 0;
    // norm watch (sfo_set_norm_watch): sfo_norm reports a relative drift from
    // watch_ref beyond watch_tol; watch_ref = 0 is off
    double watch_ref = 0.0, watch_tol = 0.0;
    // kernel timing: event pairs per kernel kind while profiling is on
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[SFO_KERNEL_KINDS];
    std::vector<hipEvent_t> ev_pool;
};

namespace {

// Tile shape of the row pass / axis-ax pass for ns states (ns = 2: reverse sweep).
int row_shape(const sfo_grid g, int ns) { return ns == 2 && g->row_var2 >= 0 ? g->row_var2 : g->row_var; }
int col_shape(const sfo_grid g, int ax, int ns) { return ns == 2 && g->col_var2[ax] >= 0 ? g->col_var2[ax] : g->col_var[ax]; }

void prof_clear(sfo_grid g)
{
    for (auto &v : g->ev) {
        for (auto &p : v) {
            g->ev_pool.push_back(p.first);
            g->ev_pool.push_back(p.second);
        }
        v.clear();
    }
}

void free_grid(sfo_grid g)
{
    if (!g) return;
    prof_clear(g);
    for (hipEvent_t e : g->ev_pool) (void)hipEventDestroy(e);
    (void)hipFree(g->V0);
    (void)hipFree(g->ebar_d);
    (void)hipFree(g->abar_d);
    for (int a = 0; a < 3; ++a) {
        (void)hipFree(g->tw[a][0]);
        (void)hipFree(g->tw[a][1]);
        (void)hipFree(g->kin[a]);
        (void)hipFree(g->kvec[a]);
    }
    (void)hipFree(g->one);
    (void)hipFree(g->red);
    (void)hipFree(g->part);
    (void)hipFree(g->chi_ref);
    for (int a = 0; a < 3; ++a) (void)hipFree(g->vtab[a]);
    (void)hipFree(g->du);
    (void)hipFree(g->eig_acc);
    delete g;
}

// Wave number of FFT index j on an axis of n points and length L (Nyquist negative).
double wavenumber(int64_t j, int64_t n, double L)
{
    const int64_t m = j < n / 2 ? j : j - n;
    return 2.0 * M_PI * (double)m / L;
}

// exp(-2 pi i j / n) for j < n, from an angle reduced to the first octant so
// that symmetric entries are exact mirrors of each other.
void unit_root(int64_t j, int64_t n, double &c, double &s)
{
    // angle = 2 pi j / n; work with j/n in eighths
    const int64_t n8 = n >= 8 ? n / 8 : 0;
    if (n8 == 0) {
        const double a = 2.0 * M_PI * (double)j / (double)n;
        c = std::cos(a);
        s = -std::sin(a);
        if (std::fabs(c) < 1e-17) c = 0.0;
        if (std::fabs(s) < 1e-17) s = 0.0;
        return;
    }
    const int64_t oct = j / n8, r = j % n8;
    // base angle within the octant, mirrored for odd octants
    const bool mirror = (oct & 1) != 0;
    const int64_t rr = mirror ? n8 - r : r;
    const double a = 2.0 * M_PI * (double)rr / (double)n;  // in [0, pi/4]
    double cb = std::cos(a), sb = std::sin(a);
    if (rr == n8) cb = sb = std::sqrt(0.5);
    // point on the unit circle at angle oct*pi/4 +- a (cos, sin)
    double cc, ss;
    switch (oct & 7) {
    case 0: cc = cb; ss = sb; break;
    case 1: cc = sb; ss = cb; break;
    case 2: cc = -sb; ss = cb; break;
    case 3: cc = -cb; ss = sb; break;
    case 4: cc = -cb; ss = -sb; break;
    case 5: cc = -sb; ss = -cb; break;
    case 6: cc = sb; ss = -cb; break;
    default: cc = cb; ss = -sb; break;
    }
    c = cc;
    s = -ss;  // forward root: exp(-i angle)
}

// Stage twiddle tables of axis a for radix 8 and 16 (the layout of
// LineShape::tw_offset): stage (radix r, span L > 1) holds W_{L r}^{j k} at
// offset + (j - 1) L + k.
sfo_status make_twiddles(sfo_grid g, int a)
{
    const int n = (int)g->n[a];
    for (int ri = 0; ri < 2; ++ri) {
        const int rad = ri == 0 ? 8 : 16;
        int radix[16], span[16], nst = 0;
        line_stages(n, rad, radix, span, &nst);
        std::vector<double> cr, ci;
        for (int s = 0; s < nst; ++s) {
            const int r = radix[s], L = span[s];
            if (L == 1) continue;
            for (int j = 1; j < r; ++j)
                for (int k = 0; k < L; ++k) {
                    double c, sn;
                    unit_root((int64_t)j * k * (n / (L * r)), n, c, sn);
                    cr.push_back(c);
                    ci.push_back(sn);
                }
        }
        const size_t cnt = cr.size() ? cr.size() : 1;
        if (cr.empty()) { cr.push_back(1.0); ci.push_back(0.0); }
        if (g->c128) {
            std::vector<TwEntry<double>> h(cnt);
            for (size_t i = 0; i < cnt; ++i) { h[i].r = cr[i]; h[i].i = ci[i]; }
            HIP_TRY(dev_malloc(&g->tw[a][ri], sizeof(TwEntry<double>) * cnt));
            HIP_TRY(hipMemcpy(g->tw[a][ri], h.data(), sizeof(TwEntry<double>) * cnt, hipMemcpyHostToDevice));
        } else {
            std::vector<TwEntry<float>> h(cnt);
            for (size_t i = 0; i < cnt; ++i) {
                h[i].hr = (float)cr[i];
                h[i].hi = (float)ci[i];
                h[i].lr = (float)(cr[i] - (double)h[i].hr);
                h[i].li = (float)(ci[i] - (double)h[i].hi);
            }
            HIP_TRY(dev_malloc(&g->tw[a][ri], sizeof(TwEntry<float>) * cnt));
            HIP_TRY(hipMemcpy(g->tw[a][ri], h.data(), sizeof(TwEntry<float>) * cnt, hipMemcpyHostToDevice));
        }
    }
    return SFO_OK;
}

// exp(-i hbar tau k^2 / (2 m)) per axis; axis 0 also carries 1/Ntot (a power of two: exact).
sfo_status make_kinetic(sfo_grid g, int a)
{
    const int64_t n = g->n[a];
    const double L = g->d.xmax[a] - g->d.xmin[a];
    std::vector<double2> h(n);
    std::vector<double> kv(n);
    const double scale = a == 0 ? 1.0 / (double)g->ntot : 1.0;
    for (int64_t j = 0; j < n; ++j) {
        const double k = wavenumber(j, n, L);
        kv[j] = k;
        const double ph = g->d.hbar * g->d.dt * k * k / (2.0 * g->d.mass);
        h[j].x = std::cos(ph) * scale;
        h[j].y = -std::sin(ph) * scale;
    }
    HIP_TRY(dev_malloc(&g->kin[a], sizeof(double2) * n));
    HIP_TRY(hipMemcpy(g->kin[a], h.data(), sizeof(double2) * n, hipMemcpyHostToDevice));
    HIP_TRY(dev_malloc(&g->kvec[a], sizeof(double) * n));
    HIP_TRY(hipMemcpy(g->kvec[a], kv.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    return SFO_OK;
}

// 1-D Dirac (alpha_1 = sigma_x, beta = sigma_z): the momentum-space step
// exp(-i tau H(p) / hbar) / N, H(p) = c p sigma_x + m c^2 sigma_z, p = hbar
// k, is cos(E tau / hbar) - i sin(E tau / hbar) H(p) / E since H^2 = E^2
// (E = sqrt(m^2 c^4 + c^2 p^2)); stored as U00, U01 (= U10), U11 per k.
sfo_status make_dirac1d_kinetic(sfo_grid g)
{
    const int64_t n = g->n[0];
    const double L = g->d.xmax[0] - g->d.xmin[0];
    const double c = g->d.c, mc2 = g->d.mass * c * c, hb = g->d.hbar, tau = g->d.dt, inv = 1.0 / (double)n;
    std::vector<double2> h((size_t)(3 * n));
    for (int64_t j = 0; j < n; ++j) {
        const double p = hb * wavenumber(j, n, L);
        const double E = std::sqrt(mc2 * mc2 + c * c * p * p);
        const double ct = std::cos(E * tau / hb), st = std::sin(E * tau / hb);
        h[(size_t)(3 * j)] = {ct * inv, -st * mc2 / E * inv};
        h[(size_t)(3 * j + 1)] = {0.0, -st * c * p / E * inv};
        h[(size_t)(3 * j + 2)] = {ct * inv, st * mc2 / E * inv};
    }
    HIP_TRY(dev_malloc(&g->du, sizeof(double2) * h.size()));
    HIP_TRY(hipMemcpy(g->du, h.data(), sizeof(double2) * h.size(), hipMemcpyHostToDevice));
    return SFO_OK;
}

// Velocity gauge (the dipole split's momentum-space operator with A(t)):
// the kinetic factor of step n, exp(-i/(2 m hbar) int (p - q A)^2 dt') with
// p = hbar k, factorises per axis as exp(-i [hbar tau k_a^2 / (2m) - q k_a
// Abar_{n,a} / m]), times the global exp(-i q^2 A2bar_n / (2 m hbar)) and
// 1/Ntot on axis 0.  Tables of every step, built in FP64 on the host.
void release_vector_tables(sfo_grid g)
{
    for (int a = 0; a < 3; ++a) {
        (void)hipFree(g->vtab[a]);
        g->vtab[a] = nullptr;
    }
    g->vsteps = 0;
}

sfo_status make_vector_tables(sfo_grid g, const double *abar, const double *a2bar, int64_t nsteps)
{
    const double q = g->d.charge, m = g->d.mass, hb = g->d.hbar, tau = g->d.dt;
    for (int a = 0; a < g->ndim; ++a) {
        const int64_t n = g->n[a];
        const double L = g->d.xmax[a] - g->d.xmin[a];
        const double scale = a == 0 ? 1.0 / (double)g->ntot : 1.0;
        std::vector<double2> h((size_t)(n * nsteps));
        for (int64_t st = 0; st < nsteps; ++st)
            for (int64_t j = 0; j < n; ++j) {
                const double k = wavenumber(j, n, L);
                double ph = hb * tau * k * k / (2.0 * m) - q * k * abar[st * g->ndim + a] / m;
                if (a == 0) ph += q * q * a2bar[st] / (2.0 * m * hb);
                h[(size_t)(st * n + j)].x = std::cos(ph) * scale;
                h[(size_t)(st * n + j)].y = -std::sin(ph) * scale;
            }
        HIP_TRY(dev_malloc(&g->vtab[a], sizeof(double2) * h.size()));
        HIP_TRY(hipMemcpy(g->vtab[a], h.data(), sizeof(double2) * h.size(), hipMemcpyHostToDevice));
    }
    g->vsteps = nsteps;
    return SFO_OK;
}

hipEvent_t prof_event(sfo_grid g)
{
    if (!g->ev_pool.empty()) {
        hipEvent_t e = g->ev_pool.back();
        g->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch `fn` bracketed by events of kind `kind` when profiling is on.
template <typename F> hipError_t timed(sfo_grid g, int kind, F &&fn)
{
    if (!g->prof) return fn();
    hipEvent_t a = prof_event(g), b = prof_event(g);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, g->st);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(b, g->st);
    if (e == hipSuccess) g->ev[kind].push_back({a, b});
    return e;
}

// Field integral of step s along axis a (zero without a table).
double ebar_at(const sfo_grid g, int64_t s, int a)
{
    if (s < 0 || s >= g->ebar_steps) return 0.0;  // callers check step ranges; timing runs may not
    return g->ebar[(size_t)(s * g->ndim + a)];
}

// Real-space factor covering the second half of step `sa` and the first half
// of step `sb` (either may be -1 for "none"); sgn = -1 conjugates.
PhaseArgs phase_args(const sfo_grid g, int64_t sa, int64_t sb, int sgn)
{
    PhaseArgs p{};
    const double inv2h = 1.0 / (2.0 * g->d.hbar);
    const int halves = (sa >= 0) + (sb >= 0);
    p.aV = g->d.dt * inv2h * halves;
    for (int a = 0; a < 3; ++a) {
        double e = 0.0;
        if (a < g->ndim) {
            if (sa >= 0) e += ebar_at(g, sa, a);
            if (sb >= 0) e += ebar_at(g, sb, a);
        }
        p.e[a] = e * inv2h;
        p.xmin[a] = a < g->ndim ? g->d.xmin[a] : 0.0;
        p.dx[a] = a < g->ndim ? g->dx[a] : 0.0;
    }
    p.sgn = sgn;
    p.small = (std::fabs(p.aV) * g->v0max <= 0.125) ? 1 : 0;
    double bound = std::fabs(p.aV) * g->v0max;
    for (int a = 0; a < g->ndim; ++a)
        bound += std::fabs(p.e[a]) * std::max(std::fabs(g->d.xmin[a]), std::fabs(g->d.xmax[a]));
    p.small32 = bound <= 0.125 ? 1 : 0;
    return p;
}

// Row pass over one state (adj == null) or a state and its adjoint.
template <typename R>
sfo_status schro_xpass(sfo_grid g, void *psi, void *adj, int64_t sa, int64_t sb, int sgn, int mode,
                       const GradArgs &ga = GradArgs{})
{
    const PhaseArgs ph = phase_args(g, sa, sb, sgn);
    const StatePtrs<R> S{{(cx<R> *)psi, (cx<R> *)adj}};
    HIP_TRY(timed(g, SFO_KERNEL_ROW, [&] {
        return launch_xpass<R>(row_shape(g, adj ? 2 : 1), (int)g->n[0], adj ? 2 : 1, S, g->n[1] * g->n[2], (int)g->n[1], g->V0,
                               (const void *const *)g->tw[0], ph, ga, mode, g->st);
    }));
    return SFO_OK;
}

// Forward/inverse transforms and the kinetic factor along the non-x axes.
// mode: M_FWD, M_INV, M_KIN combinations (in the order FWD, KIN, INV).
// chi_part: the k-space pass (the one with the kinetic factor) also forms
// the overlap partials with g->chi_ref (M_CHI) into chi_part.
// kstep: the step whose kinetic factor applies (velocity gauge: per-step tables).
template <typename R>
sfo_status schro_colpasses(sfo_grid g, void *psi, void *adj, int mode, int sgn, double *chi_part = nullptr,
                           int64_t kstep = 0, double *vpart = nullptr)
{
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const StatePtrs<R> S{{(cx<R> *)psi, (cx<R> *)adj}};
    const int ns = adj ? 2 : 1;
    const void *const *tw1 = (const void *const *)g->tw[1];
    const void *const *tw2 = (const void *const *)g->tw[2];
    const int cmode = (chi_part ? (mode | M_CHI) : mode) | (vpart ? M_VGRAD : 0);
    const bool vg = g->vsteps > 0;
    const double2 *kx = vg ? g->vtab[0] + kstep * nx : g->kin[0];
    const double2 *ky = vg ? g->vtab[1] + kstep * ny : g->kin[1];
    const double2 *kz = vg && g->ndim == 3 ? g->vtab[2] + kstep * nz : g->kin[2];
    if (g->ndim == 2) {
        KinArgs k{kx, g->one, ky, (int)nx, sgn, g->chi_ref, chi_part};
        if (vpart) {
            k.kvA = g->kvec[0];
            k.kvL = g->kvec[1];
            k.vpart = vpart;
        }
        HIP_TRY(timed(g, SFO_KERNEL_COLUMN, [&] {
            return launch_colpass<R>(col_shape(g, 1, ns), (int)ny, ns, S, nx, nx, 1, 0, tw1, k, cmode, g->st);
        }));
    } else {
        // 3-D: y-forward, z (forward, kinetic, inverse), y-inverse
        KinArgs none{g->one, g->one, g->one, 1, 1};
        KinArgs k{kx, ky, kz, (int)nx, sgn, g->chi_ref, chi_part};
        if (vpart) {
            k.kvA = g->kvec[0];
            k.kvB = g->kvec[1];
            k.kvL = g->kvec[2];
            k.vpart = vpart;
        }
        if (mode & M_FWD)
            HIP_TRY(timed(g, SFO_KERNEL_COLUMN, [&] {
                return launch_colpass<R>(col_shape(g, 1, ns), (int)ny, ns, S, nx, nx, (int)nz, nx * ny, tw1, none, M_FWD,
                                         g->st);
            }));
        HIP_TRY(timed(g, SFO_KERNEL_ZCOLUMN, [&] {
            return launch_colpass<R>(col_shape(g, 2, ns), (int)nz, ns, S, nx * ny, nx * ny, 1, 0, tw2, k, cmode, g->st);
        }));
        // (the y passes around the z pass never carry the gradient partials: their
        // mode has no M_KIN, and M_VGRAD goes only to the pass above)
        if (mode & M_INV)
            HIP_TRY(timed(g, SFO_KERNEL_COLUMN, [&] {
                return launch_colpass<R>(col_shape(g, 1, ns), (int)ny, ns, S, nx, nx, (int)nz, nx * ny, tw1, none, M_INV,
                                         g->st);
            }));
    }
    return SFO_OK;
}

sfo_status check_steps(const sfo_grid g, int64_t step0, int64_t nsteps)
{
    std::string why;
    sfo_status s = check::step_range(step0, nsteps, g->ebar_steps, "field", &why);
    if (s == SFO_OK) s = check::step_range(step0, nsteps, g->vsteps, "vector-field", &why);
    if (s == SFO_OK && g->d.equation == SFO_DIRAC)
        s = check::step_range(step0, nsteps, g->abar_steps, "vector-potential", &why);
    return checked(s, why);
}

// Schroedinger run of nsteps, forward (dir = +1) or inverse (dir = -1, last step first).
template <typename R> sfo_status schro_run(sfo_grid g, void *psi, int64_t step0, int64_t nsteps, int dir)
{
    if (nsteps == 0) return SFO_OK;
    auto step_of = [&](int64_t s) { return dir > 0 ? step0 + s : step0 + nsteps - 1 - s; };
    if (g->ndim == 1) {
        Run1DArgs a{};
        // velocity gauge: step st's kinetic factors are row st of the per-step table
        a.kin = g->vsteps > 0 ? g->vtab[0] : g->kin[0];
        a.kin_stride = g->vsteps > 0 ? g->n[0] : 0;
        a.ebar = g->ebar_steps ? g->ebar_d : nullptr;
        a.step0 = step0;
        a.nsteps = nsteps;
        a.aV_half = g->d.dt / (2.0 * g->d.hbar);
        a.inv_2hbar = 1.0 / (2.0 * g->d.hbar);
        a.xmin = g->d.xmin[0];
        a.dx = g->dx[0];
        a.dir = dir;
        HIP_TRY(timed(g, SFO_KERNEL_LINE1D, [&] {
            return launch_1d<R>((int)g->n[0], (cx<R> *)psi, 1, g->ntot, g->V0, g->tw[0][1], a, g->st);
        }));
        return SFO_OK;
    }
    sfo_status s;
    if (g->d.flags & SFO_UNFUSED) {
        // the paper's sequence: phase kernel, FFT, kinetic kernel, inverse FFT, phase kernel
        for (int64_t j = 0; j < nsteps; ++j) {
            const int64_t st = step_of(j);
            if ((s = schro_xpass<R>(g, psi, nullptr, -1, st, dir, M_PHASE))) return s;
            if ((s = schro_xpass<R>(g, psi, nullptr, -1, -1, dir, M_FWD))) return s;
            if ((s = schro_colpasses<R>(g, psi, nullptr, M_FWD, dir))) return s;
            if ((s = schro_colpasses<R>(g, psi, nullptr, M_KIN, dir, nullptr, st))) return s;
            if ((s = schro_colpasses<R>(g, psi, nullptr, M_INV, dir))) return s;
            if ((s = schro_xpass<R>(g, psi, nullptr, -1, -1, dir, M_INV))) return s;
            if ((s = schro_xpass<R>(g, psi, nullptr, st, -1, dir, M_PHASE))) return s;
        }
        return SFO_OK;
    }
    if ((s = schro_xpass<R>(g, psi, nullptr, -1, step_of(0), dir, M_PHASE | M_FWD))) return s;
    for (int64_t j = 0; j < nsteps; ++j) {
        if ((s = schro_colpasses<R>(g, psi, nullptr, M_FWD | M_KIN | M_INV, dir, nullptr, step_of(j)))) return s;
        const bool more = j + 1 < nsteps;
        if ((s = schro_xpass<R>(g, psi, nullptr, step_of(j), more ? step_of(j + 1) : -1, dir,
                                M_INV | M_PHASE | (more ? M_FWD : 0))))
            return s;
    }
    return SFO_OK;
}

// Autocorrelation run (the eigenstate method): chi_j = dV sum_x conj(psi_0)
// psi_j, j < nsteps, while psi advances nsteps steps.  With a
// time-independent potential every step's first half factor P = exp(-i tau
// V0 / 2 hbar) is the same unitary diagonal, so chi_j = dV sum conj(P psi_0)
// (P psi_j) = (dV / Ntot) sum_k conj(F P psi_0)(F P psi_j) (Parseval,
// unnormalised transform).  The k-space pass of step j holds F P psi_j right
// after its forward transform and forms the overlap with the stored F P psi_0
// there: FP64 partials per work-group, summed in slot order afterwards.
// Arguments of a 1-D eigenstate run (time-independent potential, forward).
Run1DArgs eigen1d_args(const sfo_grid g, int64_t nsteps)
{
    Run1DArgs a{};
    a.kin = g->kin[0];
    a.step0 = 0;
    a.nsteps = nsteps;
    a.aV_half = g->d.dt / (2.0 * g->d.hbar);
    a.inv_2hbar = 1.0 / (2.0 * g->d.hbar);
    a.xmin = g->d.xmin[0];
    a.dx = g->dx[0];
    a.dir = 1;
    a.tau = g->d.dt;
    a.hbar = g->d.hbar;
    a.dv = g->dv;
    return a;
}

// A state-sized buffer of the handle for the eigenstate runs' reference state.
sfo_status ensure_chi_ref(sfo_grid g, size_t sbytes)
{
    if (g->chi_ref_bytes >= sbytes) return SFO_OK;
    HIP_TRY(hipStreamSynchronize(g->st));
    (void)hipFree(g->chi_ref);
    g->chi_ref = nullptr;
    g->chi_ref_bytes = 0;
    HIP_TRY(dev_malloc(&g->chi_ref, sbytes));
    g->chi_ref_bytes = sbytes;
    return SFO_OK;
}

template <typename R> sfo_status schro_autocorr(sfo_grid g, void *psi, int64_t nsteps, double *chi)
{
    if (nsteps == 0) return SFO_OK;
    if (g->ndim == 1) {
        // the whole run in one work-group; chi_j written by the kernel itself
        sfo_status s = ensure_chi_ref(g, sizeof(cx<R>) * (size_t)g->ntot);
        if (s) return s;
        Run1DArgs a = eigen1d_args(g, nsteps);
        a.chi = chi;
        a.ref = g->chi_ref;
        HIP_TRY(timed(g, SFO_KERNEL_LINE1D, [&] {
            return launch_1d_eigen<R>((int)g->n[0], (cx<R> *)psi, g->V0, g->tw[0][1], a, g->st);
        }));
        return SFO_OK;
    }
    const int kax = g->ndim - 1;
    const int64_t ncols = kax == 1 ? g->n[0] : g->n[0] * g->n[1];
    const int nslots = (int)(ncols / kColVariants[col_shape(g, kax, 1)].cols);
    const size_t sbytes = sizeof(cx<R>) * (size_t)g->ntot;
    if (sfo_status s0 = ensure_chi_ref(g, sbytes)) return s0;
    const int64_t need = 2 * (int64_t)nslots * nsteps;
    if (g->part_cap < need) {
        HIP_TRY(hipStreamSynchronize(g->st));
        (void)hipFree(g->part);
        g->part = nullptr;
        g->part_cap = 0;
        HIP_TRY(dev_malloc(&g->part, sizeof(double) * need));
        g->part_cap = need;
    }
    // reference F P psi_0: the run's first row pass and the forward transforms of the other axes
    HIP_TRY(hipMemcpyAsync(g->chi_ref, psi, sbytes, hipMemcpyDeviceToDevice, g->st));
    sfo_status s;
    if ((s = schro_xpass<R>(g, g->chi_ref, nullptr, -1, 0, +1, M_PHASE | M_FWD))) return s;
    if ((s = schro_colpasses<R>(g, g->chi_ref, nullptr, M_FWD, +1))) return s;
    // the fused run, the k-space pass of step j writing the partials of step j
    if ((s = schro_xpass<R>(g, psi, nullptr, -1, 0, +1, M_PHASE | M_FWD))) return s;
    for (int64_t j = 0; j < nsteps; ++j) {
        if ((s = schro_colpasses<R>(g, psi, nullptr, M_FWD | M_KIN | M_INV, +1, g->part + 2 * (int64_t)nslots * j)))
            return s;
        const bool more = j + 1 < nsteps;
        if ((s = schro_xpass<R>(g, psi, nullptr, 0, more ? 0 : -1, +1, M_INV | M_PHASE | (more ? M_FWD : 0))))
            return s;
    }
    HIP_TRY(launch_chi_sum(g->part, nslots, nsteps, g->dv / (double)g->ntot, chi, g->st));
    return SFO_OK;
}

// Windowed eigenfunction (the eigenstate method): Psi_E = sum_j tau w_j
// exp(i E j tau / hbar) psi_j, j < nsteps, w_j = 1 - cos(2 pi j / nsteps),
// while psi advances nsteps steps.  Between the column pass of step j - 1
// and the row pass of step j the buffer holds F_x P^-1 psi_j (P the half
// factor, the same for every step with a time-independent potential), and
// F_x P^-1 is linear and fixed, so the weighted sum of those buffers is
// F_x P^-1 Psi_E: it is accumulated in FP64 there (w_0 = 0, so step 0 adds
// nothing), and one inverse x-transform with the half factor at the end
// gives Psi_E.
template <typename R> sfo_status schro_eigen(sfo_grid g, void *psi, int64_t nsteps, double E, void *out)
{
    const int64_t n = g->ntot;
    if (!g->eig_acc) HIP_TRY(dev_malloc(&g->eig_acc, sizeof(double2) * (size_t)n));
    if (g->ndim == 1) {
        // the whole run in one work-group: the sum accumulated per point in
        // FP64 by the thread that owns it, P^-1 applied at the end
        Run1DArgs a = eigen1d_args(g, nsteps);
        a.eig_acc = g->eig_acc;
        a.eig_out = out;
        a.eig_E = E;
        HIP_TRY(timed(g, SFO_KERNEL_LINE1D, [&] {
            return launch_1d_eigen<R>((int)g->n[0], (cx<R> *)psi, g->V0, g->tw[0][1], a, g->st);
        }));
        return SFO_OK;
    }
    HIP_TRY(hipMemsetAsync(g->eig_acc, 0, sizeof(double2) * (size_t)n, g->st));
    const double tau = g->d.dt, hb = g->d.hbar;
    sfo_status s;
    if (nsteps > 0) {
        if ((s = schro_xpass<R>(g, psi, nullptr, -1, 0, +1, M_PHASE | M_FWD))) return s;
        for (int64_t j = 0; j < nsteps; ++j) {
            if ((s = schro_colpasses<R>(g, psi, nullptr, M_FWD | M_KIN | M_INV, +1))) return s;
            const int64_t b = j + 1;  // the step boundary now in the buffer
            if (b < nsteps) {
                const double w = tau * (1.0 - std::cos(2.0 * M_PI * (double)b / (double)nsteps));
                const double ph = E * tau * (double)b / hb;
                HIP_TRY(launch_eig_axpy<R>((const cx<R> *)psi, g->eig_acc, n, w * std::cos(ph), w * std::sin(ph),
                                           g->st));
            }
            const bool more = j + 1 < nsteps;
            if ((s = schro_xpass<R>(g, psi, nullptr, 0, more ? 0 : -1, +1, M_INV | M_PHASE | (more ? M_FWD : 0))))
                return s;
        }
    }
    // Psi_E = P F_x^-1 acc, in the state's precision
    HIP_TRY(launch_acc_to_state<R>(g->eig_acc, (cx<R> *)out, n, g->st));
    return schro_xpass<R>(g, out, nullptr, -1, 0, +1, M_INV | M_PHASE);
}

// ------------------------------------------------------------- planning --
// Tile shapes chosen by timing, remembered per grid shape for the process
// and optionally in a text file named by SFO_TUNE_CACHE (one line per shape:
// "<key> <row> <y-pass> <z-pass>").
std::mutex g_plan_mu;
std::map<std::string, std::vector<int>> g_plans;
bool g_plans_loaded = false;

std::string plan_key(const sfo_grid g)
{
    std::ostringstream k;
    k << (g->c128 ? "c128" : "c64") << ":" << (g->d.equation == SFO_DIRAC ? "dirac" : "schro") << ":" << g->n[0]
      << "x" << g->n[1] << "x" << g->n[2];
    return k.str();
}

void load_plan_file()
{
    if (g_plans_loaded) return;
    g_plans_loaded = true;
    const char *path = std::getenv("SFO_TUNE_CACHE");
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string key;
    int a, b, c;
    while (f >> key >> a >> b >> c) g_plans[key] = {a, b, c};
}

void store_plan(const std::string &key, const std::vector<int> &p)
{
    g_plans[key] = p;
    const char *path = std::getenv("SFO_TUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << p[0] << " " << p[1] << " " << p[2] << "\n";
}

template <typename R> bool plan_valid(const sfo_grid g, const int *p)
{
    if (g->d.equation == SFO_DIRAC && g->ndim == 2)
        return dirac_row_variant_ok<R>(p[0], (int)g->n[0], g->n[1]) &&
               dirac_col_variant_ok<R>(p[1], (int)g->n[1], g->n[0]);
    if (!xpass_variant_ok<R>(p[0], (int)g->n[0])) return false;
    if (g->ndim >= 2 && !colpass_variant_ok<R>(p[1], (int)g->n[1], g->n[0])) return false;
    if (g->ndim == 3 && !colpass_variant_ok<R>(p[2], (int)g->n[2], g->n[0] * g->n[1])) return false;
    return true;
}

// Milliseconds of `reps` launches of fn (after two warm-up launches); -1 if a launch fails.
template <typename F> double time_launches_on(hipStream_t st, hipEvent_t a, hipEvent_t b, int reps, F &&fn)
{
    for (int i = 0; i < 2; ++i)
        if (fn() != hipSuccess) return -1.0;
    if (hipEventRecord(a, st) != hipSuccess) return -1.0;
    for (int i = 0; i < reps; ++i)
        if (fn() != hipSuccess) return -1.0;
    if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return -1.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.0;
    return ms;
}
template <typename F> double time_launches(sfo_grid g, hipEvent_t a, hipEvent_t b, int reps, F &&fn)
{
    return time_launches_on(g->st, a, b, reps, fn);
}

// Back-to-back launches of one pass shape on a scratch state (row pass:
// inverse transform, potential factor, forward transform; axis-ax pass:
// transform, kinetic factor on the last axis, inverse transform).
template <typename R> double time_row(sfo_grid g, int v, cx<R> *psi, hipEvent_t ea, hipEvent_t eb, int reps)
{
    const PhaseArgs ph = phase_args(g, -1, 0, +1);
    return time_launches(g, ea, eb, reps, [&] {
        return launch_xpass<R>(v, (int)g->n[0], 1, StatePtrs<R>{{psi, nullptr}}, g->n[1] * g->n[2], (int)g->n[1],
                               g->V0, (const void *const *)g->tw[0], ph, GradArgs{}, M_INV | M_PHASE | M_FWD, g->st);
    });
}

template <typename R>
double time_col(sfo_grid g, int ax, int v, cx<R> *psi, hipEvent_t ea, hipEvent_t eb, int reps)
{
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const int64_t ncols = ax == 1 ? nx : nx * ny;
    const int nslab = (ax == 1 && g->ndim == 3) ? (int)nz : 1;
    const bool kinetic = ax == g->ndim - 1;
    const KinArgs k{g->kin[0], ax == 2 ? g->kin[1] : g->one, g->kin[ax], (int)nx, 1};
    const KinArgs none{g->one, g->one, g->one, 1, 1};
    return time_launches(g, ea, eb, reps, [&] {
        return launch_colpass<R>(v, (int)g->n[ax], 1, StatePtrs<R>{{psi, nullptr}}, ncols, ncols, nslab, nx * ny,
                                 (const void *const *)g->tw[ax], kinetic ? k : none,
                                 kinetic ? (M_FWD | M_KIN | M_INV) : M_FWD, g->st);
    });
}

// The reverse sweep's row pass (two states, gradient partials) and axis-ax
// pass (two states) on scratch buffers.
template <typename R>
double time_row2(sfo_grid g, int v, cx<R> *psi, cx<R> *adj, double *acc, double *part, hipEvent_t ea, hipEvent_t eb,
                 int reps)
{
    const PhaseArgs ph = phase_args(g, -1, 0, -1);
    GradArgs ga{};
    ga.acc = acc;
    ga.wacc = 1.0;
    ga.part = part;
    return time_launches(g, ea, eb, reps, [&] {
        return launch_xpass<R>(v, (int)g->n[0], 2, StatePtrs<R>{{psi, adj}}, g->n[1] * g->n[2], (int)g->n[1], g->V0,
                               (const void *const *)g->tw[0], ph, ga, M_INV | M_PHASE | M_GRAD | M_FWD, g->st);
    });
}

template <typename R>
double time_col2(sfo_grid g, int ax, int v, cx<R> *psi, cx<R> *adj, hipEvent_t ea, hipEvent_t eb, int reps)
{
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const int64_t ncols = ax == 1 ? nx : nx * ny;
    const int nslab = (ax == 1 && g->ndim == 3) ? (int)nz : 1;
    const bool kinetic = ax == g->ndim - 1;
    const KinArgs k{g->kin[0], ax == 2 ? g->kin[1] : g->one, g->kin[ax], (int)nx, -1};
    const KinArgs none{g->one, g->one, g->one, 1, -1};
    return time_launches(g, ea, eb, reps, [&] {
        return launch_colpass<R>(v, (int)g->n[ax], 2, StatePtrs<R>{{psi, adj}}, ncols, ncols, nslab, nx * ny,
                                 (const void *const *)g->tw[ax], kinetic ? k : none,
                                 kinetic ? (M_FWD | M_KIN | M_INV) : M_FWD, g->st);
    });
}

// One step of the pass sequence a propagation runs, with the given shapes,
// on scratch buffers: the row pass, then (2-D) the column pass with the
// kinetic factor, or (3-D) y-forward, z with the kinetic factor, y-inverse.
// ns = 2: the reverse sweep's two-state passes (adjoint, dL/dV0 accumulator
// and partial slots).  The launch of kind `ek` (the first y-pass for
// SFO_KERNEL_COLUMN in 3-D) is timestamped by its own dispatch with ev.
template <typename R>
hipError_t step_sequence(sfo_grid g, int rv, const int *cv, int ns, cx<R> *psi, cx<R> *adj, double *acc,
                         double *part, int ek = -1, const hipEvent_t *ev = nullptr)
{
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const StatePtrs<R> S{{psi, ns == 2 ? adj : nullptr}};
    const int sgn = ns == 2 ? -1 : +1;
    const PhaseArgs ph = phase_args(g, -1, 0, sgn);
    GradArgs ga{};
    if (ns == 2) {
        ga.acc = acc;
        ga.wacc = 1.0;
        ga.part = part;
    }
    auto evk = [&](int k) { return k == ek ? ev : nullptr; };
    const int rmode = M_INV | M_PHASE | M_FWD | (ns == 2 ? M_GRAD : 0);
    hipError_t e = launch_xpass<R>(rv, (int)nx, ns, S, ny * nz, (int)ny, g->V0, (const void *const *)g->tw[0], ph, ga,
                                   rmode, g->st, GroupArgs<R>{}, 1, evk(SFO_KERNEL_ROW));
    if (e != hipSuccess) return e;
    const void *const *tw1 = (const void *const *)g->tw[1];
    const int cmode = M_FWD | M_KIN | M_INV;
    if (g->ndim == 2) {
        const KinArgs k{g->kin[0], g->one, g->kin[1], (int)nx, sgn};
        return launch_colpass<R>(cv[1], (int)ny, ns, S, nx, nx, 1, 0, tw1, k, cmode, g->st, GroupArgs<R>{}, 1,
                                 evk(SFO_KERNEL_COLUMN));
    }
    const KinArgs none{g->one, g->one, g->one, 1, 1};
    const KinArgs k{g->kin[0], g->kin[1], g->kin[2], (int)nx, sgn};
    e = launch_colpass<R>(cv[1], (int)ny, ns, S, nx, nx, (int)nz, nx * ny, tw1, none, M_FWD, g->st, GroupArgs<R>{}, 1,
                          evk(SFO_KERNEL_COLUMN));
    if (e != hipSuccess) return e;
    e = launch_colpass<R>(cv[2], (int)nz, ns, S, nx * ny, nx * ny, 1, 0, (const void *const *)g->tw[2], k, cmode,
                          g->st, GroupArgs<R>{}, 1, evk(SFO_KERNEL_ZCOLUMN));
    if (e != hipSuccess) return e;
    return launch_colpass<R>(cv[1], (int)ny, ns, S, nx, nx, (int)nz, nx * ny, tw1, none, M_INV, g->st);
}

// Scratch state and an event pair for the timing helpers.
struct TimingScratch {
    void *mem = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    ~TimingScratch()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        (void)hipFree(mem);
    }
};

template <typename R> sfo_status timing_setup(sfo_grid g, TimingScratch &ts)
{
    const size_t bytes = sizeof(cx<R>) * (size_t)g->ntot * g->ncomp;
    HIP_TRY(dev_malloc(&ts.mem, bytes));
    HIP_TRY(hipMemsetAsync(ts.mem, 0, bytes, g->st));
    HIP_TRY(hipEventCreate(&ts.a));
    HIP_TRY(hipEventCreate(&ts.b));
    return SFO_OK;
}

DiracPhaseArgs dirac_phase_args(const sfo_grid g, int64_t sa, int64_t sb, int sgn);
DiracKinArgs dirac_kin_args(const sfo_grid g, int sgn);

template <typename R> sfo_status autotune_impl(sfo_grid g, int reps)
{
    TimingScratch ts;
    sfo_status s = timing_setup<R>(g, ts);
    if (s) return s;
    cx<R> *psi = (cx<R> *)ts.mem;
    // best of three trials per shape: one trial is easily disturbed
    auto best_of = [&](auto &&timer) {
        double m = 1e30;
        for (int trial = 0; trial < 3; ++trial) {
            const double t = timer();
            if (t < 0) return -1.0;
            m = std::min(m, t);
        }
        return m;
    };
    double best = 1e30;
    if (g->d.equation == SFO_DIRAC && g->ndim == 2) {
        // whole steps (row pass, then column pass): rows given the column
        // shape, then columns given the row shape
        const DiracPhaseArgs ph = dirac_phase_args(g, 0, 0, +1);
        const DiracKinArgs k = dirac_kin_args(g, +1);
        auto steps = [&](int r, int c) {
            return time_launches(g, ts.a, ts.b, reps, [&] {
                hipError_t e = launch_dirac_xpass<R>(r, (int)g->n[0], psi, (int)g->n[1], g->ntot, g->V0,
                                                     (const void *const *)g->tw[0], ph, M_INV | M_PHASE | M_FWD, g->st);
                if (e != hipSuccess) return e;
                return launch_dirac_colpass<R>(c, (int)g->n[1], psi, (int)g->n[0], g->ntot,
                                               (const void *const *)g->tw[1], k, M_FWD | M_KIN | M_INV, g->st);
            });
        };
        for (int v = 0; v < kNumDiracRowVariants; ++v) {
            if (!dirac_row_variant_ok<R>(v, (int)g->n[0], g->n[1])) continue;
            const double ms = best_of([&] { return steps(v, g->col_var[1]); });
            if (ms >= 0 && ms < best) { best = ms; g->row_var = v; }
        }
        best = 1e30;
        for (int v = 0; v < kNumDiracColVariants; ++v) {
            if (!dirac_col_variant_ok<R>(v, (int)g->n[1], g->n[0])) continue;
            const double ms = best_of([&] { return steps(g->row_var, v); });
            if (ms >= 0 && ms < best) { best = ms; g->col_var[1] = v; }
        }
        HIP_TRY(hipStreamSynchronize(g->st));
        return SFO_OK;
    }
    const bool seq = g->d.equation == SFO_SCHRODINGER && g->ndim >= 2;
    if (seq) {
        // whole steps of the propagation's pass sequence: a pass reads what
        // the other passes wrote (a back-to-back launch of one pass would
        // find its own output in the caches); rows given the current column
        // shapes, then each column axis given the rest
        auto tune = [&](int ns, int &rv, int *cv, cx<R> *adj, double *acc, double *part) {
            auto steps = [&](int r, const int *c) {
                return time_launches(g, ts.a, ts.b, reps,
                                     [&] { return step_sequence<R>(g, r, c, ns, psi, adj, acc, part); });
            };
            // shapes whose kernel spills registers move the spilled values
            // through memory on every launch: never chosen
            auto rows = [&] {
                double b = 1e30;
                for (int v = 0; v < kNumRowVariants; ++v) {
                    if (!xpass_variant_ok<R>(v, (int)g->n[0]) || xpass_scratch<R>(v, (int)g->n[0], ns) != 0)
                        continue;
                    const double ms = best_of([&] { return steps(v, cv); });
                    if (ms >= 0 && ms < b) { b = ms; rv = v; }
                }
            };
            rows();
            double b;
            for (int ax = 1; ax < g->ndim; ++ax) {
                const int64_t ncols = ax == 1 ? g->n[0] : g->n[0] * g->n[1];
                b = 1e30;
                int keep = cv[ax];
                for (int v = 0; v < kNumColVariants; ++v) {
                    if (!colpass_variant_ok<R>(v, (int)g->n[ax], ncols, ns) ||
                        colpass_scratch<R>(v, (int)g->n[ax], ns) != 0)
                        continue;
                    cv[ax] = v;
                    const double ms = best_of([&] { return steps(rv, cv); });
                    if (ms >= 0 && ms < b) { b = ms; keep = v; }
                }
                cv[ax] = keep;
            }
            // the row shape again, given the column shapes chosen (the passes
            // share the memory system; the best row shape depends on them)
            rows();
        };
        int cv[3] = {0, g->col_var[1], g->col_var[2]};
        tune(1, g->row_var, cv, nullptr, nullptr, nullptr);
        g->col_var[1] = cv[1];
        g->col_var[2] = cv[2];
        // the reverse sweep's two-state passes, on a second state, an accumulator and partial slots
        const int64_t nrows = g->n[1] * g->n[2];
        const size_t sbytes = sizeof(cx<R>) * (size_t)g->ntot;
        const size_t ebytes = sbytes + sizeof(double) * (size_t)(g->ntot + 3 * nrows);
        void *extra = nullptr;
        HIP_TRY(dev_malloc(&extra, ebytes));
        hipError_t he = hipMemsetAsync(extra, 0, ebytes, g->st);
        if (he == hipSuccess) {
            double *acc = (double *)((char *)extra + sbytes);
            int rv2 = g->row_var, cv2[3] = {0, col_shape(g, 1, 2), g->ndim == 3 ? col_shape(g, 2, 2) : 0};
            tune(2, rv2, cv2, (cx<R> *)extra, acc, acc + g->ntot);
            g->row_var2 = rv2;
            g->col_var2[1] = cv2[1];
            g->col_var2[2] = cv2[2];
            he = hipStreamSynchronize(g->st);
        }
        (void)hipFree(extra);
        if (he != hipSuccess) return fail(SFO_E_HIP, "autotune (reverse sweep): %s", hipGetErrorString(he));
        return SFO_OK;
    }
    for (int v = 0; v < kNumRowVariants; ++v) {
        if (!xpass_variant_ok<R>(v, (int)g->n[0]) || xpass_scratch<R>(v, (int)g->n[0], 1) != 0) continue;
        const double ms = best_of([&] { return time_row<R>(g, v, psi, ts.a, ts.b, reps); });
        if (ms >= 0 && ms < best) { best = ms; g->row_var = v; }
    }
    for (int ax = 1; ax < g->ndim; ++ax) {
        const int64_t ncols = ax == 1 ? g->n[0] : g->n[0] * g->n[1];
        best = 1e30;
        for (int v = 0; v < kNumColVariants; ++v) {
            if (!colpass_variant_ok<R>(v, (int)g->n[ax], ncols) || colpass_scratch<R>(v, (int)g->n[ax], 1) != 0)
                continue;
            const double ms = best_of([&] { return time_col<R>(g, ax, v, psi, ts.a, ts.b, reps); });
            if (ms >= 0 && ms < best) { best = ms; g->col_var[ax] = v; }
        }
    }
    if (g->d.equation != SFO_SCHRODINGER) return SFO_OK;
    // the reverse sweep's two-state passes, on a second state, an accumulator and partial slots
    const int64_t nrows = g->n[1] * g->n[2];
    const size_t sbytes = sizeof(cx<R>) * (size_t)g->ntot;
    void *extra = nullptr;
    HIP_TRY(dev_malloc(&extra, sbytes + sizeof(double) * (size_t)(g->ntot + 3 * nrows)));
    hipError_t he = hipMemsetAsync(extra, 0, sbytes + sizeof(double) * (size_t)(g->ntot + 3 * nrows), g->st);
    cx<R> *adj = (cx<R> *)extra;
    double *acc = (double *)((char *)extra + sbytes);
    double *part = acc + g->ntot;
    if (he == hipSuccess) {
        best = 1e30;
        for (int v = 0; v < kNumRowVariants; ++v) {
            if (!xpass_variant_ok<R>(v, (int)g->n[0]) || xpass_scratch<R>(v, (int)g->n[0], 2) != 0) continue;
            const double ms = best_of([&] { return time_row2<R>(g, v, psi, adj, acc, part, ts.a, ts.b, reps); });
            if (ms >= 0 && ms < best) { best = ms; g->row_var2 = v; }
        }
        for (int ax = 1; ax < g->ndim; ++ax) {
            const int64_t ncols = ax == 1 ? g->n[0] : g->n[0] * g->n[1];
            best = 1e30;
            for (int v = 0; v < kNumColVariants; ++v) {
                if (!colpass_variant_ok<R>(v, (int)g->n[ax], ncols, 2) || colpass_scratch<R>(v, (int)g->n[ax], 2) != 0)
                    continue;
                const double ms = best_of([&] { return time_col2<R>(g, ax, v, psi, adj, ts.a, ts.b, reps); });
                if (ms >= 0 && ms < best) { best = ms; g->col_var2[ax] = v; }
            }
        }
        he = hipStreamSynchronize(g->st);
    }
    (void)hipFree(extra);
    if (he != hipSuccess) return fail(SFO_E_HIP, "autotune (reverse sweep): %s", hipGetErrorString(he));
    return SFO_OK;
}

template <typename R> sfo_status time_pass_impl(sfo_grid g, int kind, int reps, double *avg_ms)
{
    TimingScratch ts;
    sfo_status s = timing_setup<R>(g, ts);
    if (s) return s;
    cx<R> *psi = (cx<R> *)ts.mem;
    if (kind & SFO_TIME_IN_STEP) {
        // steps of the propagation's pass sequence; each launch of the pass is
        // timestamped by its own dispatch (one event pair per step)
        kind &= ~SFO_TIME_IN_STEP;
        const int cv[3] = {0, g->col_var[1], g->col_var[2]};
        std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
        hipError_t e = hipSuccess;
        for (size_t i = 0; i < ev.size() && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
        for (int i = 0; i < 2 && e == hipSuccess; ++i)
            e = step_sequence<R>(g, g->row_var, cv, 1, psi, nullptr, nullptr, nullptr);
        for (int i = 0; i < reps && e == hipSuccess; ++i)
            e = step_sequence<R>(g, g->row_var, cv, 1, psi, nullptr, nullptr, nullptr, kind, &ev[2 * (size_t)i]);
        if (e == hipSuccess) e = hipStreamSynchronize(g->st);
        double total = 0.0;
        for (int i = 0; i < reps && e == hipSuccess; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[2 * (size_t)i], ev[2 * (size_t)i + 1]);
            total += ms;
        }
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
        if (e != hipSuccess) return fail(SFO_E_HIP, "in-step timing failed: %s", hipGetErrorString(e));
        *avg_ms = total / reps;
        return SFO_OK;
    }
    double ms = -1.0;
    if (kind == SFO_KERNEL_ROW) ms = time_row<R>(g, g->row_var, psi, ts.a, ts.b, reps);
    else if (kind == SFO_KERNEL_COLUMN) ms = time_col<R>(g, 1, g->col_var[1], psi, ts.a, ts.b, reps);
    else ms = time_col<R>(g, 2, g->col_var[2], psi, ts.a, ts.b, reps);
    if (ms < 0) return fail(SFO_E_HIP, "timing launches failed: %s", hipGetErrorString(hipGetLastError()));
    *avg_ms = ms / reps;
    return SFO_OK;
}

// Default tile shapes before any tuning: the first shape in table order that
// exists for each pass of this grid.
template <typename R> void default_plan(sfo_grid g)
{
    if (g->d.equation == SFO_DIRAC && g->ndim == 2) {
        for (int v = 0; v < kNumDiracRowVariants; ++v)
            if (dirac_row_variant_ok<R>(v, (int)g->n[0], g->n[1])) { g->row_var = v; break; }
        for (int v = 0; v < kNumDiracColVariants; ++v)
            if (dirac_col_variant_ok<R>(v, (int)g->n[1], g->n[0])) { g->col_var[1] = v; break; }
        return;
    }
    for (int v = 0; v < kNumRowVariants; ++v)
        if (xpass_variant_ok<R>(v, (int)g->n[0])) { g->row_var = v; break; }
    for (int ax = 1; ax < g->ndim; ++ax) {
        const int64_t ncols = ax == 1 ? g->n[0] : g->n[0] * g->n[1];
        for (int v = 0; v < kNumColVariants; ++v)
            if (colpass_variant_ok<R>(v, (int)g->n[ax], ncols)) { g->col_var[ax] = v; break; }
    }
}

// Reverse sweep (see include/sfo.h, sfo_adjoint).  Boundary n of the run
// (n = 0..nsteps, state psi_{step0+n}) contributes b_n = Im(conj(g_n) psi_n):
//   dL/dV0 += (tau/2hbar) w_n b_n,  w_n = 1 at the two ends and 2 inside,
//   mom[n] = sum_x (x, y, z) b_n,  dL/dEbar[s] = (mom[s+1] + mom[s]) / (2 hbar).
// Moment partial slots per step boundary of the reverse sweep (the row
// work-groups of its two-state row pass; 1 for 1-D), 0 if there is no shape.
template <typename R> int adjoint_slots(const sfo_grid g)
{
    const int64_t nrows = g->n[1] * g->n[2];
    return g->ndim == 1 ? 1 : xpass_groups<R>(row_shape(g, 2), (int)g->n[0], nrows);
}

// The reverse sweep with its moment partials in `part` (at least
// 3 adjoint_slots (nsteps + 1) doubles of device memory; every slot that
// launch_ebar_grad reads is written first, so it needs no clearing).
// Velocity gauge (vpart != null): each step's k-space pass uses that step's
// kinetic tables and writes the gradient partials of the step (vslots x 4
// doubles per step, see KinArgs) to vpart.
template <typename R>
sfo_status schro_adjoint_in(sfo_grid g, void *psi, void *gv, int64_t step0, int64_t nsteps, double *dE, double *dV,
                            double *part, double *vpart = nullptr, int vslots = 0)
{
    const int nslots = adjoint_slots<R>(g);
    if (nslots < 1) return fail(SFO_E_STATE, "no row pass shape for this grid");
    const double wbase = g->d.dt / (2.0 * g->d.hbar);
    const bool vg = g->vsteps > 0;
    if (g->ndim == 1) {
        Run1DArgs a{};
        a.kin = vg ? g->vtab[0] : g->kin[0];
        a.kin_stride = vg ? g->n[0] : 0;
        a.kv = g->kvec[0];
        a.vmom = vpart;
        a.ebar = g->ebar_steps ? g->ebar_d : nullptr;
        a.step0 = step0;
        a.nsteps = nsteps;
        a.aV_half = g->d.dt / (2.0 * g->d.hbar);
        a.inv_2hbar = 1.0 / (2.0 * g->d.hbar);
        a.xmin = g->d.xmin[0];
        a.dx = g->dx[0];
        a.dir = -1;
        HIP_TRY(timed(g, SFO_KERNEL_LINE1D, [&] {
            return launch_1d_adjoint<R>((int)g->n[0], (cx<R> *)psi, (cx<R> *)gv, g->V0, g->tw[0][1], a, wbase, dV,
                                        part, g->st);
        }));
    } else {
        GradArgs ga{};
        ga.acc = dV;
        sfo_status s;
        auto st_of = [&](int64_t j) { return step0 + j; };
        ga.wacc = wbase;
        ga.acc_init = 1;
        ga.part = part + 3 * (int64_t)nslots * nsteps;
        const int first = nsteps > 0 ? (M_PHASE | M_FWD | M_GRAD) : M_GRAD;
        if ((s = schro_xpass<R>(g, psi, gv, -1, nsteps > 0 ? st_of(nsteps - 1) : -1, -1, first, ga))) return s;
        for (int64_t j = nsteps - 1; j >= 0; --j) {
            if ((s = schro_colpasses<R>(g, psi, gv, M_FWD | M_KIN | M_INV, -1, nullptr, st_of(j),
                                        vpart ? vpart + 4 * (int64_t)vslots * j : nullptr)))
                return s;
            ga.acc_init = 0;
            ga.wacc = (j > 0 ? 2.0 : 1.0) * wbase;
            ga.part = part + 3 * (int64_t)nslots * j;
            if ((s = schro_xpass<R>(g, psi, gv, st_of(j), j > 0 ? st_of(j - 1) : -1, -1,
                                    M_INV | M_PHASE | M_GRAD | (j > 0 ? M_FWD : 0), ga)))
                return s;
        }
    }
    if (dE) HIP_TRY(launch_ebar_grad(part, nslots, nsteps, g->ndim, 1.0 / (2.0 * g->d.hbar), dE, g->st));
    return SFO_OK;
}

// The reverse sweep with the moment partials in the handle's own buffer,
// grown (after the stream has drained) when the run needs more.
template <typename R>
sfo_status schro_adjoint(sfo_grid g, void *psi, void *gv, int64_t step0, int64_t nsteps, double *dE, double *dV)
{
    const int nslots = adjoint_slots<R>(g);
    if (nslots < 1) return fail(SFO_E_STATE, "no row pass shape for this grid");
    const int64_t need = 3 * (int64_t)nslots * (nsteps + 1);
    if (g->part_cap < need) {
        HIP_TRY(hipStreamSynchronize(g->st));
        (void)hipFree(g->part);
        g->part = nullptr;
        g->part_cap = 0;
        HIP_TRY(dev_malloc(&g->part, sizeof(double) * need));
        g->part_cap = need;
    }
    return schro_adjoint_in<R>(g, psi, gv, step0, nsteps, dE, dV, g->part);
}

// Work-groups of the reverse sweep's k-space pass (its velocity-gauge
// partial slots; 1 for 1-D).
template <typename R> int vgrad_slots(const sfo_grid g)
{
    if (g->ndim == 1) return 1;
    const int ax = g->ndim - 1;
    const int64_t ncols = ax == 1 ? g->n[0] : g->n[0] * g->n[1];
    return (int)(ncols / kColVariants[col_shape(g, ax, 2)].cols);
}

// Reverse sweep of a velocity-gauge run (sfo_adjoint_velocity): the row
// moment partials (unused here: no field table) and the k-space partials in
// the handle's buffer, then dL/dAbar = -q/(m N) sum_k k_a Im(conj(g~) psi~)
// and dL/dA2bar = q^2/(2 m hbar N) sum_k Im(conj(g~) psi~) per step.
template <typename R>
sfo_status schro_adjoint_velocity(sfo_grid g, void *psi, void *gv, int64_t step0, int64_t nsteps, double *dA,
                                  double *dA2, double *dV)
{
    const int nslots = adjoint_slots<R>(g), vslots = vgrad_slots<R>(g);
    if (nslots < 1 || vslots < 1) return fail(SFO_E_STATE, "no pass shape for this grid");
    const int64_t nrow = 3 * (int64_t)nslots * (nsteps + 1), need = nrow + 4 * (int64_t)vslots * nsteps;
    if (g->part_cap < need) {
        HIP_TRY(hipStreamSynchronize(g->st));
        (void)hipFree(g->part);
        g->part = nullptr;
        g->part_cap = 0;
        HIP_TRY(dev_malloc(&g->part, sizeof(double) * need));
        g->part_cap = need;
    }
    double *vpart = g->part + nrow;
    sfo_status s = schro_adjoint_in<R>(g, psi, gv, step0, nsteps, nullptr, dV, g->part, vpart, vslots);
    if (s) return s;
    const double q = g->d.charge, m = g->d.mass, hb = g->d.hbar, N = (double)g->ntot;
    HIP_TRY(launch_vgrad_sum(vpart, vslots, nsteps, g->ndim, -q / (m * N), q * q / (2.0 * m * hb * N), dA, dA2, g->st));
    return SFO_OK;
}

// The same with the partials in the device's static scratch array (see
// sfo_adjoint_noalloc): no allocation of any kind.  Kernel timing
// (sfo_profile_enable) is not recorded for this call, since recording it can
// create events.
template <typename R>
sfo_status schro_adjoint_noalloc(sfo_grid g, void *psi, void *gv, int64_t step0, int64_t nsteps, double *dE,
                                 double *dV, double *scratch_dev)
{
    const int nslots = adjoint_slots<R>(g);
    if (nslots < 1) return fail(SFO_E_STATE, "no row pass shape for this grid");
    const int64_t need = 3 * (int64_t)nslots * (nsteps + 1);
    if (need > kNoAllocScratchDoubles)
        return fail(SFO_E_UNSUPPORTED,
                    "the reverse sweep needs %lld doubles of partials (%d slots x %lld boundaries x 3), more than the "
                    "%lld of the static scratch array; use sfo_adjoint or split the run",
                    (long long)need, nslots, (long long)(nsteps + 1), (long long)kNoAllocScratchDoubles);
    const bool prof = g->prof;
    g->prof = false;
    const sfo_status s = schro_adjoint_in<R>(g, psi, gv, step0, nsteps, dE, dV, scratch_dev);
    g->prof = prof;
    return s;
}

// ----------------------------------------------------------------- Dirac --
DiracPhaseArgs dirac_phase_args(const sfo_grid g, int64_t sa, int64_t sb, int sgn)
{
    DiracPhaseArgs p{};
    const double inv2h = 1.0 / (2.0 * g->d.hbar);
    const int halves = (sa >= 0) + (sb >= 0);
    p.aV = g->d.dt * inv2h * halves;
    p.aA = g->d.charge * g->d.c * inv2h;
    if (g->abar_steps > 0) {
        if (sa >= 0) p.abar_a = g->abar_d + sa * g->n[0];
        if (sb >= 0) p.abar_b = g->abar_d + sb * g->n[0];
    }
    p.ca = 1.0;
    p.cb = 1.0;
    p.sgn = sgn;
    return p;
}

template <typename R> sfo_status dirac_xpass(sfo_grid g, void *psi, int64_t sa, int64_t sb, int sgn, int mode)
{
    const DiracPhaseArgs ph = dirac_phase_args(g, sa, sb, sgn);
    HIP_TRY(timed(g, SFO_KERNEL_ROW, [&] {
        return launch_dirac_xpass<R>(g->row_var, (int)g->n[0], (cx<R> *)psi, (int)g->n[1], g->ntot, g->V0,
                                     (const void *const *)g->tw[0], ph, mode, g->st);
    }));
    return SFO_OK;
}

DiracKinArgs dirac_kin_args(const sfo_grid g, int sgn)
{
    DiracKinArgs k{};
    k.kx = g->kvec[0];
    k.ky = g->kvec[1];
    k.c = g->d.c;
    k.mc2 = g->d.mass * g->d.c * g->d.c;
    k.hbar = g->d.hbar;
    k.tau_over_hbar = g->d.dt / g->d.hbar;
    k.inv_ntot = 1.0 / (double)g->ntot;
    k.sgn = sgn;
    return k;
}

template <typename R> sfo_status dirac_colpass(sfo_grid g, void *psi, int mode, int sgn)
{
    const DiracKinArgs k = dirac_kin_args(g, sgn);
    HIP_TRY(timed(g, SFO_KERNEL_COLUMN, [&] {
        return launch_dirac_colpass<R>(g->col_var[1], (int)g->n[1], (cx<R> *)psi, (int)g->n[0], g->ntot,
                                       (const void *const *)g->tw[1], k, mode, g->st);
    }));
    return SFO_OK;
}

template <typename R> sfo_status dirac_run(sfo_grid g, void *psi, int64_t step0, int64_t nsteps, int dir)
{
    if (nsteps == 0) return SFO_OK;
    if (g->ndim == 1) {
        // the whole run of the line in one work-group (forward steps only)
        if (dir != 1) return fail(SFO_E_UNSUPPORTED, "1-D Dirac runs forward");
        Dirac1DArgs a{};
        a.u = g->du;
        a.abar = g->abar_steps ? g->abar_d : nullptr;
        a.step0 = step0;
        a.nsteps = nsteps;
        a.aV_half = g->d.dt / (2.0 * g->d.hbar);
        a.aA = 0.5 * g->d.charge * g->d.c / g->d.hbar;
        HIP_TRY(timed(g, SFO_KERNEL_LINE1D, [&] {
            return launch_dirac1d<R>((int)g->n[0], (cx<R> *)psi, g->V0, (const void *const *)g->tw[0], a, g->st);
        }));
        return SFO_OK;
    }
    auto step_of = [&](int64_t s) { return dir > 0 ? step0 + s : step0 + nsteps - 1 - s; };
    sfo_status s;
    if (g->d.flags & SFO_UNFUSED) {
        for (int64_t j = 0; j < nsteps; ++j) {
            const int64_t st = step_of(j);
            if ((s = dirac_xpass<R>(g, psi, -1, st, dir, M_PHASE))) return s;
            if ((s = dirac_xpass<R>(g, psi, -1, -1, dir, M_FWD))) return s;
            if ((s = dirac_colpass<R>(g, psi, M_FWD, dir))) return s;
            if ((s = dirac_colpass<R>(g, psi, M_KIN, dir))) return s;
            if ((s = dirac_colpass<R>(g, psi, M_INV, dir))) return s;
            if ((s = dirac_xpass<R>(g, psi, -1, -1, dir, M_INV))) return s;
            if ((s = dirac_xpass<R>(g, psi, st, -1, dir, M_PHASE))) return s;
        }
        return SFO_OK;
    }
    if ((s = dirac_xpass<R>(g, psi, -1, step_of(0), dir, M_PHASE | M_FWD))) return s;
    for (int64_t j = 0; j < nsteps; ++j) {
        if ((s = dirac_colpass<R>(g, psi, M_FWD | M_KIN | M_INV, dir))) return s;
        const bool more = j + 1 < nsteps;
        if ((s = dirac_xpass<R>(g, psi, step_of(j), more ? step_of(j + 1) : -1, dir,
                                M_INV | M_PHASE | (more ? M_FWD : 0))))
            return s;
    }
    return SFO_OK;
}

template <typename R> sfo_status do_fft(sfo_grid g, void *psi, int sign)
{
    const int mode = sign < 0 ? M_FWD : M_INV;
    for (int c = 0; c < g->ncomp; ++c) {
        cx<R> *p = (cx<R> *)psi + c * g->ntot;
        PhaseArgs ph{};
        ph.sgn = 1;
        const StatePtrs<R> S{{p, nullptr}};
        HIP_TRY(launch_xpass<R>(g->row_var, (int)g->n[0], 1, S, g->n[1] * g->n[2], (int)g->n[1], g->V0,
                                (const void *const *)g->tw[0], ph, GradArgs{}, mode, g->st));
        if (g->ndim >= 2) {
            const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
            KinArgs none{g->one, g->one, g->one, 1, 1};
            HIP_TRY(launch_colpass<R>(g->col_var[1], (int)ny, 1, S, nx, nx, (int)nz, nx * ny,
                                      (const void *const *)g->tw[1], none, mode, g->st));
            if (g->ndim == 3)
                HIP_TRY(launch_colpass<R>(g->col_var[2], (int)nz, 1, S, nx * ny, nx * ny, 1, 0,
                                          (const void *const *)g->tw[2], none, mode, g->st));
        }
    }
    return SFO_OK;
}

}  // namespace

// ------------------------------------------------------------------ batch --
// Problems are grouped by shape; a grouped launch covers one group (see
// GroupArgs).  The launch sequence of a run is the single-grid one with every
// pass launched once per group, captured once per (direction, step0, nsteps)
// in a HIP graph and replayed on the caller's stream.
struct sfo_batch_s {
    std::vector<sfo_grid> grids;
    bool c128 = false;
    hipStream_t st = nullptr;    // the caller's stream: every launch or replay goes here
    hipStream_t cap = nullptr;   // private streams the graphs are captured on
    hipStream_t side = nullptr;  //   (1-D whole runs go on the side branch)
    hipEvent_t fork = nullptr, join = nullptr;
    // captured graphs: each 2-D group's sequence on a branch of its own (the
    // groups' problems are independent, so their launches may overlap)
    std::vector<hipStream_t> br;
    std::vector<hipEvent_t> br_join;
    struct Group {
        int ndim, nx, ny;
        int off, count;  // ids[off .. off+count)
        sfo_grid rep;    // a grid of the group: its tables and tile shapes serve all
        // the shapes chosen for the grouped launches of the forward runs and
        // of the reverse sweep (sfo_batch_autotune); -1: those of rep
        int row_f = -1, col_f = -1, row2_f = -1, col2_f = -1;
    };
    std::vector<Group> groups;
    std::vector<int> ids;
    int *ids_d = nullptr;
    void *probs_d = nullptr;      // BatchProb<R>[count]
    std::vector<char> probs_h;    // what probs_d holds
    double *work = nullptr;       // reverse sweep: moments and partials
    int64_t work_cap = 0;
    bool use_graph = true;
    struct Graph {
        int dir;
        int64_t step0, nsteps;
        std::vector<int> shapes;  // tile shapes the captured launches were made with
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
};

namespace {

void free_batch(sfo_batch b)
{
    if (!b) return;
    for (auto &gr : b->graphs) (void)hipGraphExecDestroy(gr.exec);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    for (hipEvent_t e : b->br_join)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t q : b->br)
        if (q) (void)hipStreamDestroy(q);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->side) (void)hipStreamDestroy(b->side);
    (void)hipFree(b->ids_d);
    (void)hipFree(b->probs_d);
    (void)hipFree(b->work);
    delete b;
}

// The grids of a batch grouped by shape, in order of first appearance.
void group_batch(sfo_batch b, const sfo_grid *grids, int count)
{
    b->grids.assign(grids, grids + count);
    for (int i = 0; i < count; ++i) {
        const sfo_grid g = grids[i];
        bool found = false;
        for (const auto &G : b->groups)
            found |= G.ndim == g->ndim && G.nx == (int)g->n[0] && G.ny == (int)g->n[1];
        if (found) continue;
        sfo_batch_s::Group G{g->ndim, (int)g->n[0], (int)g->n[1], (int)b->ids.size(), 0, g};
        for (int k = i; k < count; ++k)
            if (grids[k]->ndim == G.ndim && (int)grids[k]->n[0] == G.nx && (int)grids[k]->n[1] == G.ny) {
                b->ids.push_back(k);
                ++G.count;
            }
        b->groups.push_back(G);
    }
}

// Descriptors of every problem for one call; *work_need: the moment and
// partial workspace of a reverse sweep (doubles).
// Shapes of a 2-D group's grouped launches with ns states.
int group_row(const sfo_batch_s::Group &G, int ns)
{
    const int f = ns == 1 ? G.row_f : G.row2_f;
    return f >= 0 ? f : row_shape(G.rep, ns);
}
int group_col(const sfo_batch_s::Group &G, int ns)
{
    const int f = ns == 1 ? G.col_f : G.col2_f;
    return f >= 0 ? f : col_shape(G.rep, 1, ns);
}

template <typename R>
std::vector<BatchProb<R>> batch_probs(const sfo_batch b, void *const *psi, void *const *gadj, double *const *dE,
                                      double *const *dV, int64_t nsteps, int64_t *work_need)
{
    const int n = (int)b->grids.size();
    std::vector<BatchProb<R>> P(n);
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        const sfo_grid g = b->grids[i];
        BatchProb<R> &q = P[i];
        std::memset(&q, 0, sizeof q);
        q.ndim = g->ndim;
        q.nx = (int)g->n[0];
        q.ny = (int)g->n[1];
        q.psi = (cx<R> *)psi[i];
        q.ebar = g->ebar_steps ? g->ebar_d : nullptr;
        q.kin_x = g->kin[0];
        q.kin_y = g->ndim > 1 ? g->kin[1] : nullptr;
        q.one = g->one;
        for (int a = 0; a < 3; ++a) {
            q.xmin[a] = a < g->ndim ? g->d.xmin[a] : 0.0;
            q.dx[a] = g->dx[a];
            q.xabs[a] = a < g->ndim ? std::max(std::fabs(g->d.xmin[a]), std::fabs(g->d.xmax[a])) : 0.0;
        }
        q.aV_half = g->d.dt / (2.0 * g->d.hbar);
        q.inv_2hbar = 1.0 / (2.0 * g->d.hbar);
        q.v0max = g->v0max;
        q.V0 = (decltype(q.V0))g->V0;
        q.gslots = 1;
        if (g->ndim == 2) {
            for (const auto &G : b->groups)
                if (G.ndim == 2 && G.nx == q.nx && G.ny == q.ny)
                    q.gslots = std::max(1, xpass_groups<R>(group_row(G, 2), q.nx, q.ny));
        }
        if (gadj) {
            q.gadj = (cx<R> *)gadj[i];
            q.dE = dE ? dE[i] : nullptr;
            q.dV = dV ? dV[i] : nullptr;
            q.part = b->work ? b->work + off : nullptr;
            off += 3 * (int64_t)q.gslots * (nsteps + 1);
        }
    }
    *work_need = off;
    return P;
}

// The tile shapes of every 2-D group's passes: a captured graph holds launches
// of these shapes (grid sizes, and in the reverse sweep the partial-slot
// stride of the row pass), so it is valid only while they are unchanged.
std::vector<int> batch_shapes(const sfo_batch b)
{
    std::vector<int> v;
    for (const auto &G : b->groups)
        if (G.ndim == 2)
            for (int ns = 1; ns <= 2; ++ns) {
                v.push_back(group_row(G, ns));
                v.push_back(group_col(G, ns));
            }
    return v;
}

// The launches of one batched run on stream s (1-D whole runs on `side`
// when it is given, joined back before the end).
template <typename R>
hipError_t batch_enqueue(sfo_batch b, int dir, int64_t step0, int64_t nsteps, hipStream_t s, hipStream_t side,
                         int only = -1)
{
    const BatchProb<R> *pd = (const BatchProb<R> *)b->probs_d;
    const int ns = dir < 0 ? 2 : 1;
    if (dir < 0) {
        // the reverse sweep's row work-groups write their moment partials at
        // slot blockIdx.x of a block of gslots slots per boundary: the
        // uploaded descriptors must have been made for these launch shapes
        const BatchProb<R> *ph = (const BatchProb<R> *)b->probs_h.data();
        for (const auto &G : b->groups) {
            if (G.ndim != 2) continue;
            const int launched = std::max(1, xpass_groups<R>(group_row(G, 2), G.nx, G.ny));
            for (int k = 0; k < G.count; ++k)
                if (b->probs_h.size() < sizeof(BatchProb<R>) * b->grids.size() || ph[b->ids[G.off + k]].gslots != launched)
                    return hipErrorInvalidValue;
        }
    }
    const StatePtrs<R> none{{nullptr, nullptr}};
    auto grp_of = [&](const sfo_batch_s::Group &G, int64_t sa, int64_t sb, int64_t jmom, double wmul, int init) {
        GroupArgs<R> a{};
        a.probs = pd;
        a.ids = b->ids_d + G.off;
        a.sa = sa;
        a.sb = sb;
        a.jmom = jmom;
        a.wmul = wmul;
        a.acc_init = init;
        return a;
    };
    hipError_t e = hipSuccess;
    // 1-D problems: one whole-run launch per length
    hipStream_t s1 = side ? side : s;
    if (e == hipSuccess && side) {
        e = hipEventRecord(b->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, b->fork, 0);
    }
    for (const auto &G : b->groups) {
        if (e != hipSuccess || G.ndim != 1 || only >= 0) continue;
        Run1DArgs a{};
        a.step0 = step0;
        a.nsteps = nsteps;
        a.dir = dir;
        const GroupArgs<R> grp = grp_of(G, -1, -1, 0, 1.0, 0);
        e = dir > 0 ? launch_1d<R>(G.nx, nullptr, G.count, 0, nullptr, G.rep->tw[0][1], a, s1, grp)
                    : launch_1d_adjoint<R>(G.nx, nullptr, nullptr, nullptr, G.rep->tw[0][1], a, 0.0, nullptr,
                                           nullptr, s1, grp, G.count);
    }
    // 2-D problems: the fused single-grid sequence of each group (a launch
    // covers the group's problems), on the group's own branch when side
    // branches are given (capture), otherwise one group after the other on s
    auto group_seq = [&](const sfo_batch_s::Group &G, hipStream_t gs) {
        auto xpass = [&](int64_t sa, int64_t sb, int mode, int64_t jmom, double wmul, int init) {
            if (e != hipSuccess) return;
            PhaseArgs ph{};
            ph.sgn = dir;
            e = launch_xpass<R>(group_row(G, ns), G.nx, ns, none, G.ny, G.ny, nullptr,
                                (const void *const *)G.rep->tw[0], ph, GradArgs{}, mode, gs,
                                grp_of(G, sa, sb, jmom, wmul, init), G.count);
        };
        auto colpass = [&]() {
            if (e != hipSuccess) return;
            KinArgs k{nullptr, nullptr, nullptr, 1, dir};
            e = launch_colpass<R>(group_col(G, ns), G.ny, ns, none, G.nx, G.nx, 1, 0,
                                  (const void *const *)G.rep->tw[1], k, M_FWD | M_KIN | M_INV, gs,
                                  grp_of(G, -1, -1, 0, 1.0, 0), G.count);
        };
        if (dir > 0) {
            if (nsteps > 0) {
                xpass(-1, step0, M_PHASE | M_FWD, 0, 1.0, 0);
                for (int64_t j = 0; j < nsteps; ++j) {
                    colpass();
                    const bool more = j + 1 < nsteps;
                    xpass(step0 + j, more ? step0 + j + 1 : -1, M_INV | M_PHASE | (more ? M_FWD : 0), 0, 1.0, 0);
                }
            }
        } else {
            // reverse sweep (as schro_adjoint): boundary nsteps first, then each step backwards
            xpass(-1, nsteps > 0 ? step0 + nsteps - 1 : -1, nsteps > 0 ? (M_PHASE | M_FWD | M_GRAD) : M_GRAD, nsteps,
                  1.0, 1);
            for (int64_t j = nsteps - 1; j >= 0; --j) {
                colpass();
                xpass(step0 + j, j > 0 ? step0 + j - 1 : -1, M_INV | M_PHASE | M_GRAD | (j > 0 ? M_FWD : 0), j,
                      j > 0 ? 2.0 : 1.0, 0);
            }
        }
    };
    size_t k2 = 0;
    for (const auto &G : b->groups) {
        if (e != hipSuccess || G.ndim != 2) continue;
        if (only >= 0 && &G != &b->groups[(size_t)only]) {
            ++k2;
            continue;
        }
        const bool own = side && k2 < b->br.size();
        hipStream_t gs = own ? b->br[k2] : s;
        if (own) e = hipStreamWaitEvent(gs, b->fork, 0);
        group_seq(G, gs);
        if (e == hipSuccess && own) {
            e = hipEventRecord(b->br_join[k2], gs);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, b->br_join[k2], 0);
        }
        ++k2;
    }
    if (e == hipSuccess && side) {
        e = hipEventRecord(b->join, side);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join, 0);
    }
    if (e == hipSuccess && dir < 0) e = launch_batch_ebar_grad<R>(pd, (int)b->grids.size(), nsteps, s);
    return e;
}

// Tile shapes of the grouped forward launches (sfo_batch_autotune): each 2-D
// group's sequence alone, `reps` steps on scratch states, rows given the
// column shape, then columns given the row shape.
template <typename R> sfo_status batch_tune(sfo_batch b, int reps)
{
    const int n = (int)b->grids.size();
    size_t total = 0;
    for (const sfo_grid g : b->grids) total += (size_t)g->ntot;
    HIP_TRY(hipStreamSynchronize(b->st));
    TimingScratch ts;
    HIP_TRY(dev_malloc(&ts.mem, sizeof(cx<R>) * total));
    HIP_TRY(hipMemsetAsync(ts.mem, 0, sizeof(cx<R>) * total, b->st));
    HIP_TRY(hipEventCreate(&ts.a));
    HIP_TRY(hipEventCreate(&ts.b));
    std::vector<void *> ptr((size_t)n);
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        ptr[(size_t)i] = (cx<R> *)ts.mem + off;
        off += (size_t)b->grids[(size_t)i]->ntot;
    }
    int64_t need = 0;
    const std::vector<BatchProb<R>> P = batch_probs<R>(b, ptr.data(), nullptr, nullptr, nullptr, 0, &need);
    const size_t bytes = sizeof(BatchProb<R>) * P.size();
    HIP_TRY(hipMemcpy(b->probs_d, P.data(), bytes, hipMemcpyHostToDevice));
    b->probs_h.assign((const char *)P.data(), (const char *)P.data() + bytes);
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        sfo_batch_s::Group &G = b->groups[gi];
        if (G.ndim != 2) continue;
        // steps within every member's field table
        int64_t steps = reps;
        for (int k = 0; k < G.count; ++k) {
            const sfo_grid g = b->grids[(size_t)b->ids[(size_t)(G.off + k)]];
            if (g->ebar_steps > 0) steps = std::min<int64_t>(steps, g->ebar_steps);
        }
        auto time_seq = [&]() {
            double best = -1.0;
            for (int trial = 0; trial < 3; ++trial) {
                const double ms = time_launches_on(b->st, ts.a, ts.b, 1, [&] {
                    return batch_enqueue<R>(b, +1, 0, steps, b->st, nullptr, (int)gi);
                });
                if (ms >= 0 && (best < 0 || ms < best)) best = ms;
            }
            return best;
        };
        G.row_f = row_shape(G.rep, 1);
        G.col_f = col_shape(G.rep, 1, 1);
        double best = time_seq();
        int keep = G.row_f;
        for (int v = 0; v < kNumRowVariants; ++v) {
            if (!xpass_variant_ok<R>(v, G.nx) || xpass_scratch<R>(v, G.nx, 1) != 0) continue;
            G.row_f = v;
            const double ms = time_seq();
            if (ms >= 0 && ms < best) { best = ms; keep = v; }
        }
        G.row_f = keep;
        keep = G.col_f;
        for (int v = 0; v < kNumColVariants; ++v) {
            if (!colpass_variant_ok<R>(v, G.ny, G.nx) || colpass_scratch<R>(v, G.ny, 1) != 0) continue;
            G.col_f = v;
            const double ms = time_seq();
            if (ms >= 0 && ms < best) { best = ms; keep = v; }
        }
        G.col_f = keep;
    }
    // the reverse sweep's two-state launches: scratch adjoint states; the
    // partial slots follow the row shape being timed (descriptors rebuilt)
    TimingScratch ga;
    HIP_TRY(dev_malloc(&ga.mem, sizeof(cx<R>) * total));
    HIP_TRY(hipMemsetAsync(ga.mem, 0, sizeof(cx<R>) * total, b->st));
    std::vector<void *> gptr((size_t)n);
    off = 0;
    for (int i = 0; i < n; ++i) {
        gptr[(size_t)i] = (cx<R> *)ga.mem + off;
        off += (size_t)b->grids[(size_t)i]->ntot;
    }
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        sfo_batch_s::Group &G = b->groups[gi];
        if (G.ndim != 2) continue;
        int64_t steps = reps;
        for (int k = 0; k < G.count; ++k) {
            const sfo_grid g = b->grids[(size_t)b->ids[(size_t)(G.off + k)]];
            if (g->ebar_steps > 0) steps = std::min<int64_t>(steps, g->ebar_steps);
        }
        sfo_status err = SFO_OK;
        auto time_rev = [&]() {
            int64_t wneed = 0;
            (void)batch_probs<R>(b, ptr.data(), gptr.data(), nullptr, nullptr, steps, &wneed);
            if (hipStreamSynchronize(b->st) != hipSuccess) return -1.0;
            if (wneed > b->work_cap) {
                (void)hipFree(b->work);
                b->work = nullptr;
                b->work_cap = 0;
                if (dev_malloc(&b->work, sizeof(double) * wneed) != hipSuccess) {
                    err = fail(SFO_E_NOMEM, "batch autotune: device allocation failed");
                    return -1.0;
                }
                b->work_cap = wneed;
            }
            const std::vector<BatchProb<R>> Q = batch_probs<R>(b, ptr.data(), gptr.data(), nullptr, nullptr, steps, &wneed);
            const size_t qb = sizeof(BatchProb<R>) * Q.size();
            if (hipMemcpy(b->probs_d, Q.data(), qb, hipMemcpyHostToDevice) != hipSuccess) return -1.0;
            b->probs_h.assign((const char *)Q.data(), (const char *)Q.data() + qb);
            double best = -1.0;
            for (int trial = 0; trial < 3; ++trial) {
                const double ms = time_launches_on(b->st, ts.a, ts.b, 1, [&] {
                    return batch_enqueue<R>(b, -1, 0, steps, b->st, nullptr, (int)gi);
                });
                if (ms >= 0 && (best < 0 || ms < best)) best = ms;
            }
            return best;
        };
        G.row2_f = row_shape(G.rep, 2);
        G.col2_f = col_shape(G.rep, 1, 2);
        double best = time_rev();
        int keep = G.row2_f;
        for (int v = 0; v < kNumRowVariants && !err; ++v) {
            if (!xpass_variant_ok<R>(v, G.nx) || xpass_scratch<R>(v, G.nx, 2) != 0) continue;
            G.row2_f = v;
            const double ms = time_rev();
            if (ms >= 0 && ms < best) { best = ms; keep = v; }
        }
        G.row2_f = keep;
        keep = G.col2_f;
        for (int v = 0; v < kNumColVariants && !err; ++v) {
            if (!colpass_variant_ok<R>(v, G.ny, G.nx, 2) || colpass_scratch<R>(v, G.ny, 2) != 0) continue;
            G.col2_f = v;
            const double ms = time_rev();
            if (ms >= 0 && ms < best) { best = ms; keep = v; }
        }
        G.col2_f = keep;
        if (err) return err;
    }
    HIP_TRY(hipStreamSynchronize(b->st));
    return SFO_OK;
}

template <typename R>
sfo_status batch_run(sfo_batch b, void *const *psi, void *const *gadj, int64_t step0, int64_t nsteps, double *const *dE,
                     double *const *dV)
{
    const int n = (int)b->grids.size();
    const int dir = gadj ? -1 : +1;
    for (int i = 0; i < n; ++i) {
        if (!psi[i] || (gadj && !gadj[i])) return fail(SFO_E_INVALID, "problem %d: null state", i);
        sfo_status s = check_steps(b->grids[i], step0, nsteps);
        if (s) return fail(s, "problem %d: %s", i, g_err.c_str());
    }
    if (dir > 0 && nsteps == 0) return SFO_OK;
    int64_t need = 0;
    (void)batch_probs<R>(b, psi, gadj, dE, dV, nsteps, &need);
    if (need > b->work_cap) {
        HIP_TRY(hipStreamSynchronize(b->st));
        (void)hipFree(b->work);
        b->work = nullptr;
        b->work_cap = 0;
        HIP_TRY(dev_malloc(&b->work, sizeof(double) * need));
        b->work_cap = need;
    }
    const std::vector<BatchProb<R>> P = batch_probs<R>(b, psi, gadj, dE, dV, nsteps, &need);
    const size_t bytes = sizeof(BatchProb<R>) * P.size();
    if (b->probs_h.size() != bytes || std::memcmp(b->probs_h.data(), P.data(), bytes) != 0) {
        // earlier launches may still read the descriptors: let them finish first
        HIP_TRY(hipStreamSynchronize(b->st));
        HIP_TRY(hipMemcpy(b->probs_d, P.data(), bytes, hipMemcpyHostToDevice));
        b->probs_h.assign((const char *)P.data(), (const char *)P.data() + bytes);
    }
    if (!b->use_graph) {
        HIP_TRY(batch_enqueue<R>(b, dir, step0, nsteps, b->st, nullptr));
        return SFO_OK;
    }
    hipGraphExec_t exec = nullptr;
    const std::vector<int> shapes = batch_shapes(b);
    for (auto &gr : b->graphs)
        if (gr.dir == dir && gr.step0 == step0 && gr.nsteps == nsteps && gr.shapes == shapes) exec = gr.exec;
    if (!exec) {
        if (b->graphs.size() >= 16) {
            HIP_TRY(hipStreamSynchronize(b->st));
            (void)hipGraphExecDestroy(b->graphs.front().exec);
            b->graphs.erase(b->graphs.begin());
        }
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
        const hipError_t le = batch_enqueue<R>(b, dir, step0, nsteps, b->cap, b->side);
        const hipError_t ce = hipStreamEndCapture(b->cap, &graph);
        if (le != hipSuccess && graph) (void)hipGraphDestroy(graph);
        HIP_TRY(le);
        HIP_TRY(ce);
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_TRY(ie);
        b->graphs.push_back({dir, step0, nsteps, shapes, exec});
    }
    HIP_TRY(hipGraphLaunch(exec, b->st));
    return SFO_OK;
}

}  // namespace

extern "C" {

const char *sfo_last_error(void) { return g_err.c_str(); }

const char *sfo_version(void) { return "sfo 0.1 (gfx950)"; }

sfo_status sfo_create_grid(const sfo_grid_desc *desc, void *hip_stream, sfo_grid *out)
{
    AllocCount alloc_count;
    g_err.clear();
    if (!desc || !out) return fail(SFO_E_INVALID, "null descriptor or output handle");
    *out = nullptr;
    const sfo_grid_desc &d = *desc;
    int64_t ntot = 1;
    std::string why;
    if (sfo_status vs = check::grid_desc(desc, &why, &ntot)) return checked(vs, why);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    int ndev = 0;
    if (e == hipSuccess) e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) return fail(SFO_E_HIP, "no HIP device: %s", hipGetErrorString(e));

    sfo_grid g = new (std::nothrow) sfo_grid_s;
    if (!g) return fail(SFO_E_NOMEM, "host allocation failed");
    g->d = d;
    g->st = (hipStream_t)hip_stream;
    g->dev = dev;
    scratch_setup(dev);
    g->ndim = d.ndim;
    g->ncomp = d.equation == SFO_DIRAC ? (d.ndim == 1 ? 2 : 4) : 1;
    g->ntot = ntot;
    g->c128 = d.dtype == SFO_C128;
    g->dv = 1.0;
    for (int a = 0; a < 3; ++a) {
        g->n[a] = a < d.ndim ? d.n[a] : 1;
        g->dx[a] = a < d.ndim ? (d.xmax[a] - d.xmin[a]) / (double)d.n[a] : 0.0;
        if (a < d.ndim) g->dv *= g->dx[a];
    }
    if (g->c128)
        default_plan<double>(g);
    else
        default_plan<float>(g);
    sfo_status s = SFO_OK;
    auto guard = [&](sfo_status r) { if (r != SFO_OK) { free_grid(g); } return r; };
    for (int a = 0; a < d.ndim && s == SFO_OK; ++a) s = no_throw([&] { return make_twiddles(g, a); });
    for (int a = 0; a < d.ndim && s == SFO_OK; ++a) s = no_throw([&] { return make_kinetic(g, a); });
    if (s == SFO_OK && d.equation == SFO_DIRAC && d.ndim == 1) s = no_throw([&] { return make_dirac1d_kinetic(g); });
    if (s != SFO_OK) return guard(s);
    const double2 one = {1.0, 0.0};
    hipError_t he = dev_malloc(&g->one, sizeof(double2));
    if (he == hipSuccess) he = hipMemcpy(g->one, &one, sizeof(double2), hipMemcpyHostToDevice);
    if (he == hipSuccess) he = dev_malloc(&g->red, sizeof(double) * (2 * kReduceBlocks + 4));
    const size_t vbytes = (g->c128 ? sizeof(double) : sizeof(float)) * (size_t)ntot;
    if (he == hipSuccess) he = dev_malloc(&g->V0, vbytes);
    if (he == hipSuccess) he = hipMemset(g->V0, 0, vbytes);
    if (he != hipSuccess)
        return guard(fail(he == hipErrorOutOfMemory ? SFO_E_NOMEM : SFO_E_HIP, "allocation: %s", hipGetErrorString(he)));
    *out = g;
    return SFO_OK;
}

sfo_status sfo_destroy_grid(sfo_grid g)
{
    if (!g) return fail(SFO_E_INVALID, "null grid");
    (void)hipStreamSynchronize(g->st);
    free_grid(g);
    return SFO_OK;
}

sfo_status sfo_set_potential(sfo_grid g, const double *V0_dev)
{
    if (!g || !V0_dev) return fail(SFO_E_INVALID, "null grid or potential");
    // checked before it replaces the handle's potential
    double *res = g->red + 2 * kReduceBlocks;
    HIP_TRY(launch_absmax(V0_dev, g->ntot, g->red, res, g->st));
    double m = 0.0;
    HIP_TRY(hipMemcpyAsync(&m, res, sizeof(double), hipMemcpyDeviceToHost, g->st));
    HIP_TRY(hipStreamSynchronize(g->st));
    if (!std::isfinite(m)) return fail(SFO_E_INVALID, "potential holds a non-finite value");
    HIP_TRY(launch_convert_v0(V0_dev, g->V0, g->c128, g->ntot, g->st));
    g->v0max = m;
    return SFO_OK;
}

sfo_status sfo_set_field(sfo_grid g, const double *ebar_host, int64_t nsteps)
{
    AllocCount alloc_count;
    if (!g) return fail(SFO_E_INVALID, "null grid");
    if (g->d.equation != SFO_SCHRODINGER) return fail(SFO_E_INVALID, "field table is for the Schroedinger equation");
    std::string why;
    if (sfo_status vs = check::step_table(ebar_host, nsteps, g->ndim, 0.0, 0.0, "field", &why))
        return checked(vs, why);
    const size_t count = (size_t)nsteps * g->ndim;
    return no_throw([&]() -> sfo_status {
        std::vector<double> host(ebar_host, ebar_host + count);
        double *dev = nullptr;
        sfo_status s = upload_table(host.data(), count, &dev);
        if (s) return s;
        const hipError_t e = hipStreamSynchronize(g->st);
        if (e != hipSuccess) {
            (void)hipFree(dev);
            return fail(SFO_E_HIP, "stream: %s", hipGetErrorString(e));
        }
        // the new table replaces the old one (and any velocity-gauge tables)
        // only once it is complete
        release_vector_tables(g);
        (void)hipFree(g->ebar_d);
        g->ebar_d = dev;
        g->ebar.swap(host);
        g->ebar_steps = nsteps;
        return SFO_OK;
    });
}

sfo_status sfo_set_vector_field(sfo_grid g, const double *abar_host, const double *a2bar_host, int64_t nsteps)
{
    AllocCount alloc_count;
    if (!g) return fail(SFO_E_INVALID, "null grid");
    if (g->d.equation != SFO_SCHRODINGER) return fail(SFO_E_INVALID, "the vector field is for the Schroedinger equation");
    int64_t per = 0;
    for (int a = 0; a < g->ndim; ++a) per += g->n[a];
    std::string why;
    sfo_status vs = check::step_table(abar_host, nsteps, g->ndim, 0.0, 0.0, "vector-field", &why);
    if (vs == SFO_OK) vs = check::step_table(a2bar_host, nsteps, 1, 0.0, 0.0, "vector-field", &why);
    if (vs) return checked(vs, why);
    // the device tables: per-step, per-axis complex factors, nsteps x (n[0] + n[1] + n[2]) x 16 bytes
    if ((double)nsteps * (double)per * sizeof(double2) > kMaxTableBytes)
        return fail(SFO_E_UNSUPPORTED, "vector-field tables of %lld steps exceed 1 GiB", (long long)nsteps);
    HIP_TRY(hipStreamSynchronize(g->st));
    release_vector_tables(g);
    // the velocity gauge replaces the length-gauge field
    (void)hipFree(g->ebar_d);
    g->ebar_d = nullptr;
    g->ebar.clear();
    g->ebar_steps = 0;
    if (nsteps == 0) return SFO_OK;
    // on failure the grid is left with no field at all
    sfo_status s = no_throw([&] { return make_vector_tables(g, abar_host, a2bar_host, nsteps); });
    if (s) release_vector_tables(g);
    return s;
}

sfo_status sfo_set_vector_potential(sfo_grid g, const double *abar_y_host, int64_t nsteps)
{
    AllocCount alloc_count;
    if (!g) return fail(SFO_E_INVALID, "null grid");
    if (g->d.equation != SFO_DIRAC) return fail(SFO_E_INVALID, "vector potential is for the Dirac equation");
    std::string why;
    if (sfo_status vs = check::step_table(abar_y_host, nsteps, g->n[0], sizeof(double), kMaxTableBytes,
                                          "vector-potential", &why))
        return checked(vs, why);
    const size_t count = (size_t)nsteps * g->n[0];
    return no_throw([&]() -> sfo_status {
        std::vector<double> host(abar_y_host, abar_y_host + count);
        double *dev = nullptr;
        sfo_status s = upload_table(host.data(), count, &dev);
        if (s) return s;
        const hipError_t e = hipStreamSynchronize(g->st);
        if (e != hipSuccess) {
            (void)hipFree(dev);
            return fail(SFO_E_HIP, "stream: %s", hipGetErrorString(e));
        }
        // the new table replaces the old one only once it is complete
        (void)hipFree(g->abar_d);
        g->abar_d = dev;
        g->abar.swap(host);
        g->abar_steps = nsteps;
        return SFO_OK;
    });
}

sfo_status sfo_propagate(sfo_grid g, void *psi_dev, int64_t step0, int64_t nsteps)
{
    if (!g || !psi_dev) return fail(SFO_E_INVALID, "null grid or state");
    sfo_status s = check_steps(g, step0, nsteps);
    if (s) return s;
    if (g->d.equation == SFO_DIRAC)
        return g->c128 ? dirac_run<double>(g, psi_dev, step0, nsteps, +1) : dirac_run<float>(g, psi_dev, step0, nsteps, +1);
    return g->c128 ? schro_run<double>(g, psi_dev, step0, nsteps, +1) : schro_run<float>(g, psi_dev, step0, nsteps, +1);
}

sfo_status sfo_step(sfo_grid g, void *psi_dev, int64_t step_index) { return sfo_propagate(g, psi_dev, step_index, 1); }

sfo_status sfo_autocorrelation(sfo_grid g, void *psi_dev, int64_t nsteps, double *chi_dev)
{
    AllocCount alloc_count;
    if (!g || !psi_dev || (!chi_dev && nsteps > 0)) return fail(SFO_E_INVALID, "null grid, state or output");
    if (nsteps < 0) return fail(SFO_E_INVALID, "negative step count");
    if (g->d.equation != SFO_SCHRODINGER)
        return fail(SFO_E_UNSUPPORTED, "the autocorrelation run is built for Schroedinger grids");
    if (g->ebar_steps > 0 || g->vsteps > 0)
        return fail(SFO_E_UNSUPPORTED, "the autocorrelation run needs a time-independent potential: clear the field table");
    return g->c128 ? schro_autocorr<double>(g, psi_dev, nsteps, chi_dev)
                   : schro_autocorr<float>(g, psi_dev, nsteps, chi_dev);
}

sfo_status sfo_eigenfunction(sfo_grid g, void *psi_dev, int64_t nsteps, double energy, void *out_dev)
{
    AllocCount alloc_count;
    if (!g || !psi_dev || !out_dev) return fail(SFO_E_INVALID, "null grid, state or output");
    if (psi_dev == out_dev) return fail(SFO_E_INVALID, "psi and the output must be distinct buffers");
    if (nsteps < 0 || !std::isfinite(energy)) return fail(SFO_E_INVALID, "need nsteps >= 0 and a finite energy");
    if (g->d.equation != SFO_SCHRODINGER)
        return fail(SFO_E_UNSUPPORTED, "the eigenfunction run is built for Schroedinger grids");
    if (g->ebar_steps > 0 || g->vsteps > 0)
        return fail(SFO_E_UNSUPPORTED, "the eigenfunction run needs a time-independent potential: clear the field table");
    return g->c128 ? schro_eigen<double>(g, psi_dev, nsteps, energy, out_dev)
                   : schro_eigen<float>(g, psi_dev, nsteps, energy, out_dev);
}

sfo_status sfo_spectrum(sfo_grid g, const double *chi_dev, int64_t nsteps, const double *energies_dev, int32_t nE,
                        double *out_dev)
{
    if (!g || !chi_dev || !energies_dev || !out_dev) return fail(SFO_E_INVALID, "null argument");
    if (nsteps < 1 || nE < 0) return fail(SFO_E_INVALID, "need nsteps >= 1 and nE >= 0");
    if (nE > (1 << 30)) return fail(SFO_E_UNSUPPORTED, "at most 2^30 energies per call");
    HIP_TRY(launch_spectrum(chi_dev, nsteps, g->d.dt, g->d.hbar, energies_dev, nE, out_dev, g->st));
    return SFO_OK;
}

sfo_status sfo_adjoint(sfo_grid g, void *psi_dev, void *g_dev, int64_t step0, int64_t nsteps, double *dL_debar_dev,
                       double *dL_dV0_dev)
{
    AllocCount alloc_count;
    if (!g || !psi_dev || !g_dev) return fail(SFO_E_INVALID, "null grid or state");
    if (psi_dev == g_dev) return fail(SFO_E_INVALID, "psi and g must be distinct buffers");
    sfo_status s = check_steps(g, step0, nsteps);
    if (s) return s;
    if (g->d.equation != SFO_SCHRODINGER) return fail(SFO_E_UNSUPPORTED, "the adjoint is built for the Schroedinger equation");
    if (g->vsteps > 0)
        return fail(SFO_E_UNSUPPORTED, "a velocity-gauge grid: its gradient is sfo_adjoint_velocity's");
    return g->c128 ? schro_adjoint<double>(g, psi_dev, g_dev, step0, nsteps, dL_debar_dev, dL_dV0_dev)
                   : schro_adjoint<float>(g, psi_dev, g_dev, step0, nsteps, dL_debar_dev, dL_dV0_dev);
}

sfo_status sfo_adjoint_velocity(sfo_grid g, void *psi_dev, void *g_dev, int64_t step0, int64_t nsteps,
                                double *dL_dabar_dev, double *dL_da2bar_dev, double *dL_dV0_dev)
{
    AllocCount alloc_count;
    if (!g || !psi_dev || !g_dev) return fail(SFO_E_INVALID, "null grid or state");
    if (psi_dev == g_dev) return fail(SFO_E_INVALID, "psi and g must be distinct buffers");
    if (g->d.equation != SFO_SCHRODINGER) return fail(SFO_E_UNSUPPORTED, "the adjoint is built for the Schroedinger equation");
    if (g->vsteps <= 0) return fail(SFO_E_STATE, "no vector-field table: set one with sfo_set_vector_field (or use sfo_adjoint)");
    sfo_status s = check_steps(g, step0, nsteps);
    if (s) return s;
    return g->c128 ? schro_adjoint_velocity<double>(g, psi_dev, g_dev, step0, nsteps, dL_dabar_dev, dL_da2bar_dev,
                                                    dL_dV0_dev)
                   : schro_adjoint_velocity<float>(g, psi_dev, g_dev, step0, nsteps, dL_dabar_dev, dL_da2bar_dev,
                                                   dL_dV0_dev);
}

sfo_status sfo_adjoint_noalloc(sfo_grid g, void *psi_dev, void *g_dev, int64_t step0, int64_t nsteps,
                               double *dL_debar_dev, double *dL_dV0_dev)
{
    if (!g || !psi_dev || !g_dev) return fail(SFO_E_INVALID, "null grid or state");
    if (psi_dev == g_dev) return fail(SFO_E_INVALID, "psi and g must be distinct buffers");
    sfo_status s = check_steps(g, step0, nsteps);
    if (s) return s;
    if (g->d.equation != SFO_SCHRODINGER) return fail(SFO_E_UNSUPPORTED, "the adjoint is built for the Schroedinger equation");
    if (g->vsteps > 0) return fail(SFO_E_UNSUPPORTED, "the adjoint is built for the length gauge");
    double *ptr = nullptr;
    hipError_t e = hipSuccess;
    if (g->dev >= 0 && g->dev < kMaxScratchDevices) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        ptr = g_scratch_dev[g->dev];
        e = g_scratch_err[g->dev];
    }
    if (!ptr)
        return fail(SFO_E_HIP, "the scratch array of device %d has no device address: %s", g->dev,
                    e != hipSuccess ? hipGetErrorString(e) : "not looked up (device number out of range)");
    return g->c128 ? schro_adjoint_noalloc<double>(g, psi_dev, g_dev, step0, nsteps, dL_debar_dev, dL_dV0_dev, ptr)
                   : schro_adjoint_noalloc<float>(g, psi_dev, g_dev, step0, nsteps, dL_debar_dev, dL_dV0_dev, ptr);
}

sfo_status sfo_norm(sfo_grid g, const void *psi_dev, double *out_host)
{
    if (!g || !psi_dev || !out_host) return fail(SFO_E_INVALID, "null argument");
    const int64_t n = g->ntot * g->ncomp;
    double *res = g->red + 2 * kReduceBlocks;
    if (g->c128)
        HIP_TRY(launch_norm<double>((const cx<double> *)psi_dev, n, g->red, res, g->st));
    else
        HIP_TRY(launch_norm<float>((const cx<float> *)psi_dev, n, g->red, res, g->st));
    double h;
    HIP_TRY(hipMemcpyAsync(&h, res, sizeof(double), hipMemcpyDeviceToHost, g->st));
    HIP_TRY(hipStreamSynchronize(g->st));
    const double nrm = h * g->dv;
    *out_host = nrm;
    // a NaN or Inf anywhere in the state reaches the FP64 sum (sums of |psi|^2 keep it)
    if (!std::isfinite(nrm)) return fail(SFO_E_NUMERIC, "the state holds a non-finite value (norm %g)", nrm);
    if (g->watch_ref > 0.0) {
        const double drift = nrm / g->watch_ref - 1.0;
        if (!(std::fabs(drift) <= g->watch_tol))
            return fail(SFO_E_NUMERIC, "norm %.17g drifted by %.3e from the watched %.17g (tolerance %.3e)", nrm,
                        drift, g->watch_ref, g->watch_tol);
    }
    return SFO_OK;
}

sfo_status sfo_set_norm_watch(sfo_grid g, double reference, double tolerance)
{
    if (!g) return fail(SFO_E_INVALID, "null grid");
    if (!std::isfinite(reference) || reference < 0.0 || !std::isfinite(tolerance) || tolerance < 0.0)
        return fail(SFO_E_INVALID, "need a finite reference >= 0 and a finite tolerance >= 0");
    g->watch_ref = reference;
    g->watch_tol = tolerance;
    return SFO_OK;
}

sfo_status sfo_overlap(sfo_grid g, const void *a_dev, const void *b_dev, double *out_host)
{
    if (!g || !a_dev || !b_dev || !out_host) return fail(SFO_E_INVALID, "null argument");
    const int64_t n = g->ntot * g->ncomp;
    double *res = g->red + 2 * kReduceBlocks;
    if (g->c128)
        HIP_TRY(launch_overlap<double>((const cx<double> *)a_dev, (const cx<double> *)b_dev, n, g->red, res, g->st));
    else
        HIP_TRY(launch_overlap<float>((const cx<float> *)a_dev, (const cx<float> *)b_dev, n, g->red, res, g->st));
    double h[2];
    HIP_TRY(hipMemcpyAsync(h, res, 2 * sizeof(double), hipMemcpyDeviceToHost, g->st));
    HIP_TRY(hipStreamSynchronize(g->st));
    out_host[0] = h[0] * g->dv;
    out_host[1] = h[1] * g->dv;
    if (!std::isfinite(out_host[0]) || !std::isfinite(out_host[1]))
        return fail(SFO_E_NUMERIC, "a state holds a non-finite value (overlap %g%+gi)", out_host[0], out_host[1]);
    return SFO_OK;
}

sfo_status sfo_autotune(sfo_grid g, int32_t reps)
{
    AllocCount alloc_count;
    if (!g) return fail(SFO_E_INVALID, "null grid");
    if (reps < 1 || reps > 10000) return fail(SFO_E_INVALID, "reps must be in 1..10000");
    if (g->ndim == 1) return SFO_OK;  // the whole-run 1-D kernel has a single shape
    const std::string key = plan_key(g);
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        load_plan_file();
        auto it = g_plans.find(key);
        if (it != g_plans.end()) {
            const int p[3] = {it->second[0], it->second[1], it->second[2]};
            auto r = g_plans.find(key + ":reverse");
            const int q[3] = {r != g_plans.end() ? r->second[0] : p[0], r != g_plans.end() ? r->second[1] : p[1],
                              r != g_plans.end() ? r->second[2] : p[2]};
            if ((g->c128 ? plan_valid<double>(g, p) : plan_valid<float>(g, p)) &&
                (g->c128 ? plan_valid<double>(g, q) : plan_valid<float>(g, q))) {
                g->row_var = p[0];
                g->col_var[1] = p[1];
                g->col_var[2] = p[2];
                g->row_var2 = q[0];
                g->col_var2[1] = q[1];
                g->col_var2[2] = q[2];
                return SFO_OK;
            }
        }
    }
    HIP_TRY(hipStreamSynchronize(g->st));
    sfo_status s = no_throw([&] { return g->c128 ? autotune_impl<double>(g, reps) : autotune_impl<float>(g, reps); });
    if (s) return s;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    store_plan(key, {g->row_var, g->col_var[1], g->col_var[2]});
    store_plan(key + ":reverse", {row_shape(g, 2), col_shape(g, 1, 2), col_shape(g, 2, 2)});
    return SFO_OK;
}

sfo_status sfo_time_pass(sfo_grid g, int32_t kind, int32_t reps, double *avg_ms)
{
    AllocCount alloc_count;
    if (!g || !avg_ms) return fail(SFO_E_INVALID, "null grid or output");
    if (g->d.equation != SFO_SCHRODINGER || g->ndim < 2)
        return fail(SFO_E_UNSUPPORTED, "pass timing is for 2-D and 3-D Schroedinger grids");
    if (reps < 1) return fail(SFO_E_INVALID, "reps must be positive");
    const int k = kind & ~SFO_TIME_IN_STEP;
    if (k != SFO_KERNEL_ROW && k != SFO_KERNEL_COLUMN && !(k == SFO_KERNEL_ZCOLUMN && g->ndim == 3))
        return fail(SFO_E_INVALID, "no pass of kind %d on this grid", kind);
    if ((kind & SFO_TIME_IN_STEP) && reps > 4096) return fail(SFO_E_INVALID, "in-step timing takes at most 4096 reps");
    return g->c128 ? time_pass_impl<double>(g, kind, reps, avg_ms) : time_pass_impl<float>(g, kind, reps, avg_ms);
}

sfo_status sfo_get_plan(sfo_grid g, int32_t *plan)
{
    if (!g || !plan) return fail(SFO_E_INVALID, "null argument");
    plan[0] = g->row_var;
    plan[1] = g->col_var[1];
    plan[2] = g->col_var[2];
    return SFO_OK;
}

sfo_status sfo_set_plan(sfo_grid g, const int32_t *plan)
{
    if (!g || !plan) return fail(SFO_E_INVALID, "null argument");
    const int p[3] = {plan[0], g->ndim >= 2 ? plan[1] : 0, g->ndim == 3 ? plan[2] : 0};
    if (!(g->c128 ? plan_valid<double>(g, p) : plan_valid<float>(g, p)))
        return fail(SFO_E_INVALID, "tile shapes (%d, %d, %d) do not exist for this grid", p[0], p[1], p[2]);
    g->row_var = p[0];
    g->col_var[1] = p[1];
    g->col_var[2] = p[2];
    g->row_var2 = -1;  // the reverse sweep follows the forced shapes
    g->col_var2[1] = g->col_var2[2] = -1;
    return SFO_OK;
}

sfo_status sfo_profile_enable(sfo_grid g, int32_t on)
{
    if (!g) return fail(SFO_E_INVALID, "null grid");
    HIP_TRY(hipStreamSynchronize(g->st));
    prof_clear(g);
    g->prof = on != 0;
    return SFO_OK;
}

sfo_status sfo_profile_read(sfo_grid g, int32_t kind, int64_t *count, double *total_ms)
{
    if (!g || !count || !total_ms) return fail(SFO_E_INVALID, "null argument");
    if (kind < 0 || kind >= SFO_KERNEL_KINDS) return fail(SFO_E_INVALID, "unknown kernel kind %d", kind);
    HIP_TRY(hipStreamSynchronize(g->st));
    double sum = 0.0;
    for (auto &p : g->ev[kind]) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.first, p.second));
        sum += ms;
    }
    *count = (int64_t)g->ev[kind].size();
    *total_ms = sum;
    return SFO_OK;
}

sfo_status sfo_create_batch(const sfo_grid *grids, int32_t count, void *hip_stream, sfo_batch *out)
{
    AllocCount alloc_count;
    g_err.clear();
    if (!grids || !out || count < 1) return fail(SFO_E_INVALID, "need an output handle and at least one grid");
    *out = nullptr;
    const bool c128 = grids[0] && grids[0]->c128;
    for (int i = 0; i < count; ++i) {
        const sfo_grid g = grids[i];
        if (!g) return fail(SFO_E_INVALID, "grid %d is null", i);
        if (g->d.equation != SFO_SCHRODINGER) return fail(SFO_E_UNSUPPORTED, "grid %d: batches hold Schroedinger grids", i);
        if (g->c128 != c128) return fail(SFO_E_INVALID, "grid %d: every grid of a batch has the same dtype", i);
        if (g->ndim > 2) return fail(SFO_E_UNSUPPORTED, "grid %d: batches hold 1-D and 2-D grids", i);
        if (g->vsteps > 0) return fail(SFO_E_UNSUPPORTED, "grid %d: batches run in the length gauge", i);
    }
    sfo_batch b = new (std::nothrow) sfo_batch_s;
    if (!b) return fail(SFO_E_NOMEM, "host allocation failed");
    sfo_status s = no_throw([&]() -> sfo_status {
        group_batch(b, grids, count);
        return SFO_OK;
    });
    if (s) {
        free_batch(b);
        return s;
    }
    b->c128 = c128;
    b->st = (hipStream_t)hip_stream;
    auto guard = [&](hipError_t e) {
        free_batch(b);
        return fail(e == hipErrorOutOfMemory ? SFO_E_NOMEM : SFO_E_HIP, "batch set-up: %s", hipGetErrorString(e));
    };
    hipError_t e = hipStreamCreate(&b->cap);
    if (e == hipSuccess) e = hipStreamCreate(&b->side);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
    for (const auto &G : b->groups) {
        if (e != hipSuccess || G.ndim != 2) continue;
        b->br.push_back(nullptr);
        b->br_join.push_back(nullptr);
        e = hipStreamCreate(&b->br.back());
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->br_join.back(), hipEventDisableTiming);
    }
    if (e == hipSuccess) e = dev_malloc(&b->ids_d, sizeof(int) * b->ids.size());
    if (e == hipSuccess) e = hipMemcpy(b->ids_d, b->ids.data(), sizeof(int) * b->ids.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = dev_malloc(&b->probs_d, (c128 ? sizeof(BatchProb<double>) : sizeof(BatchProb<float>)) * count);
    if (e != hipSuccess) return guard(e);
    *out = b;
    return SFO_OK;
}

sfo_status sfo_destroy_batch(sfo_batch b)
{
    if (!b) return fail(SFO_E_INVALID, "null batch");
    (void)hipStreamSynchronize(b->st);
    free_batch(b);
    return SFO_OK;
}

sfo_status sfo_batch_autotune(sfo_batch b, int32_t reps)
{
    AllocCount alloc_count;
    if (!b) return fail(SFO_E_INVALID, "null batch");
    if (reps < 1 || reps > 10000) return fail(SFO_E_INVALID, "reps must be in 1..10000");
    return no_throw([&] { return b->c128 ? batch_tune<double>(b, reps) : batch_tune<float>(b, reps); });
}

sfo_status sfo_batch_set_graph(sfo_batch b, int32_t on)
{
    if (!b) return fail(SFO_E_INVALID, "null batch");
    b->use_graph = on != 0;
    return SFO_OK;
}

sfo_status sfo_propagate_batch(sfo_batch b, void *const *psi_devs, int64_t step0, int64_t nsteps)
{
    AllocCount alloc_count;
    if (!b || !psi_devs) return fail(SFO_E_INVALID, "null batch or state list");
    return no_throw([&] {
        return b->c128 ? batch_run<double>(b, psi_devs, nullptr, step0, nsteps, nullptr, nullptr)
                       : batch_run<float>(b, psi_devs, nullptr, step0, nsteps, nullptr, nullptr);
    });
}

sfo_status sfo_adjoint_batch(sfo_batch b, void *const *psi_devs, void *const *g_devs, int64_t step0, int64_t nsteps,
                             double *const *dL_debar_devs, double *const *dL_dV0_devs)
{
    AllocCount alloc_count;
    if (!b || !psi_devs || !g_devs) return fail(SFO_E_INVALID, "null batch, state list or adjoint list");
    return no_throw([&] {
        return b->c128 ? batch_run<double>(b, psi_devs, g_devs, step0, nsteps, dL_debar_devs, dL_dV0_devs)
                       : batch_run<float>(b, psi_devs, g_devs, step0, nsteps, dL_debar_devs, dL_dV0_devs);
    });
}

sfo_status sfo_batch_check(sfo_batch b)
{
    if (!b) return fail(SFO_E_INVALID, "null batch");
    HIP_TRY(hipStreamSynchronize(b->st));
    return SFO_OK;
}

sfo_status sfo_fft(sfo_grid g, void *psi_dev, int32_t sign)
{
    if (!g || !psi_dev) return fail(SFO_E_INVALID, "null grid or state");
    if (sign != 1 && sign != -1) return fail(SFO_E_INVALID, "sign must be -1 or +1");
    if (g->ndim == 1 && g->n[0] > kMaxPassN)
        return fail(SFO_E_UNSUPPORTED, "stand-alone transform supports lines up to %d points", kMaxPassN);
    return g->c128 ? do_fft<double>(g, psi_dev, sign) : do_fft<float>(g, psi_dev, sign);
}

}  // extern "C"
