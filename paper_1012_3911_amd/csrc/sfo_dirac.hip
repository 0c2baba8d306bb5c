// Split-step passes of the 2-D Dirac equation for a 4-spinor stored as four
// planes [4][ny][nx] (Sec. 2.3 of the paper, Dirac representation).
//
// Row pass: inverse x-transform of the four planes, the real-space factor
//   exp(-i sgn aV V0) [cos a + i sin a alpha_2],  a(x) = sgn q c Abar_y(x) / (2 hbar)
// (eq. exp_alpha with the single component A_y; i alpha_2 maps
// (p1, p2, p3, p4) to (p4, -p3, p2, -p1), so the factor is real apart from the
// scalar phase), forward x-transform.  Consecutive half steps merge: both the
// scalar phases and the alpha_2 rotations add.
// Column pass: forward y-transform, the momentum-space factor
//   U(k) = cos(E tau/hbar) - i sgn sin(E tau/hbar) H(hbar k) / E,
//   H = c (alpha_1 p_x + alpha_2 p_y) + m c^2 beta,  E = sqrt(m^2 c^4 + c^2 p^2)
// (eq. U_A_2_DE evaluated through H^2 = E^2), times 1/N_tot, inverse transform.
// In the Dirac representation H couples (1,4) and (2,3):
//   H = [[mc2, 0, 0, w], [0, mc2, wb, 0], [0, w, -mc2, 0], [wb, 0, 0, -mc2]],
//   w = c (p_x - i p_y), wb = c (p_x + i p_y).
// The spinor factors are evaluated in FP64 and applied in FP64.
#include <type_traits>
#include <utility>

#include "pass_kernels.h"

namespace sfo {

template <typename R> __device__ __forceinline__ void dirac_rotate(cx<R> (&p)[4], double c, double s, double fr, double fi)
{
    // p <- (fr + i fi) (c p + s (p4, -p3, p2, -p1)) in FP64
    const double r0 = c * (double)p[0].re + s * (double)p[3].re, i0 = c * (double)p[0].im + s * (double)p[3].im;
    const double r1 = c * (double)p[1].re - s * (double)p[2].re, i1 = c * (double)p[1].im - s * (double)p[2].im;
    const double r2 = c * (double)p[2].re + s * (double)p[1].re, i2 = c * (double)p[2].im + s * (double)p[1].im;
    const double r3 = c * (double)p[3].re - s * (double)p[0].re, i3 = c * (double)p[3].im - s * (double)p[0].im;
    p[0] = {(R)(fr * r0 - fi * i0), (R)(fr * i0 + fi * r0)};
    p[1] = {(R)(fr * r1 - fi * i1), (R)(fr * i1 + fi * r1)};
    p[2] = {(R)(fr * r2 - fi * i2), (R)(fr * i2 + fi * r2)};
    p[3] = {(R)(fr * r3 - fi * i3), (R)(fr * i3 + fi * r3)};
}

// Planes of a work-group: all four, or one of the two pairs that the factors
// couple ((1,4) and (2,3): the alpha_2 rotation of the row pass and the
// off-diagonal terms of H map each pair to itself), so that a work-group of
// a pair holds half the registers and can take radix-16 transforms.
template <int NPL> __device__ __forceinline__ int dirac_plane(int pair, int q)
{
    return NPL == 4 ? q : (pair ? 1 + q : 3 * q);
}

template <typename R, int N, int RAD, int NPL, int THREADS>
__global__ void __launch_bounds__((RowTile<N, RAD, THREADS>::NT)) __attribute__((amdgpu_waves_per_eu(2)))
    k_dirac_xpass(cx<R> *__restrict__ psi, int64_t plane, const VStore<R> *__restrict__ V0,
                  const TwEntry<R> *__restrict__ tw, DiracPhaseArgs ph, int mode)
{
    using Sh = LineShape<N, RAD>;
    using Map = RowMap<R, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV, ROWS = RowTile<N, RAD, THREADS>::ROWS;
    __shared__ cx<R> lds[ROWS * Map::slots(N)];
    // a pair's two work-groups of the same rows are consecutive after the
    // XCD remap (one XCD, the potential read once into its L2)
    const unsigned G = gridDim.x;
    unsigned L = blockIdx.x;
    if ((G & 7u) == 0) L = (L & 7u) * (G >> 3) + (L >> 3);
    const int pair = NPL == 4 ? 0 : (int)(L & 1u);
    const unsigned rg = NPL == 4 ? L : L >> 1;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int64_t row0 = (int64_t)rg * ROWS, row = row0 + line;
    cx<R> *sh = lds + line * Map::slots(N);
    // addresses: the work-group's uniform base of plane q, element m (scalar
    // registers) plus the thread's 32-bit byte offset (see row_load)
    uint32_t lt = (uint32_t)(line * N + t) * (uint32_t)sizeof(cx<R>);
    auto at = [&](int q, int m) {
        char *b = scalar_base((char *)(psi + dirac_plane<NPL>(pair, q) * plane + row0 * N + m * T));
        return (cx<R> *)(b + lt);
    };
    // stage factors formed from each stage's W^k, read once with the line (no
    // table reads inside the transforms)
    TwBase<N, RAD> wb;
    tw_base_load(wb, tw, t);
    cx<R> v[NPL][RV];
#pragma unroll
    for (int q = 0; q < NPL; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) v[q][m] = gload(at(q, m));
    if (mode & M_INV)
#pragma unroll
        for (int q = 0; q < NPL; ++q) fft_line_pre<R, N, RAD, +1, Map>(v[q], sh, t, tw, wb);
    if (mode & M_PHASE) {
        const double sg = (double)ph.sgn;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const int x = t + m * T;
            double s, c;
            sincos_fp64(sg * ph.aV * (double)gload1(V0 + row * N + x), s, c);
            double ab = 0.0;
            if (ph.abar_a) ab += ph.ca * ph.abar_a[x];
            if (ph.abar_b) ab += ph.cb * ph.abar_b[x];
            double sa, ca;
            sincos_fp64(sg * ph.aA * ab, sa, ca);
            if constexpr (NPL == 4) {
                cx<R> p[4] = {v[0][m], v[1][m], v[2][m], v[3][m]};
                dirac_rotate(p, ca, sa, c, -s);
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q][m] = p[q];
            } else {
                // pair (1,4): (a, b) <- (c a + s b, c b - s a); pair (2,3): (c a - s b, c b + s a)
                const double ss = pair ? -sa : sa;
                const double ar = v[0][m].re, ai = v[0][m].im, br = v[1][m].re, bi = v[1][m].im;
                const double r0 = ca * ar + ss * br, i0 = ca * ai + ss * bi;
                const double r1 = ca * br - ss * ar, i1 = ca * bi - ss * ai;
                const double fr = c, fi = -s;
                v[0][m] = {(R)(fr * r0 - fi * i0), (R)(fr * i0 + fi * r0)};
                v[1][m] = {(R)(fr * r1 - fi * i1), (R)(fr * i1 + fi * r1)};
            }
        }
    }
    if (mode & M_FWD)
#pragma unroll
        for (int q = 0; q < NPL; ++q) fft_line_pre<R, N, RAD, -1, Map>(v[q], sh, t, tw, wb);
    // the offset is recomputed rather than held through the transforms
    __asm__ __volatile__("" : "+v"(lt));
#pragma unroll
    for (int q = 0; q < NPL; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) gstore(at(q, m), v[q][m]);
}

// Dirac momentum-space factor at element m of the thread's points (k-space
// values of all four planes, or of one coupled pair), in FP64:
// (1/Ntot) [cos(E tau/hbar) - i sgn sin(E tau/hbar) H/E] at p = hbar (kx, ky).
template <typename R, int NPL, int NV>
__device__ __forceinline__ void dirac_kin_point(cx<R> (&v)[NPL][NV], int m, double px, double py,
                                                const DiracKinArgs &kin, int pair)
{
    const double sg = (double)kin.sgn;
    const double E = sqrt(kin.mc2 * kin.mc2 + kin.c * kin.c * (px * px + py * py));
    double sE, cE;
    sincos_fp64(E * kin.tau_over_hbar, sE, cE);
    const double sig = sg * sE / E;
    // U = C - i sig H, scaled by 1/Ntot
    const double Cn = cE * kin.inv_ntot, sgn_ = sig * kin.inv_ntot;
    const double am = sgn_ * kin.mc2;              // diag: Cn -+ i am
    const double wr = kin.c * px, wi = -kin.c * py; // w = c (px - i py)
    // off-diagonal coefficient -i sig w = (sig wi) - i (sig wr)  [times 1/Ntot]
    const double owr = sgn_ * wi, owi = -sgn_ * wr;     // -i sig w
    const double obr = -sgn_ * wi, obi = -sgn_ * wr;    // -i sig wb, wb = conj(w)
    auto mul = [](double xr, double xi, double yr, double yi, double &zr, double &zi) {
        zr = xr * yr - xi * yi;
        zi = xr * yi + xi * yr;
    };
    double t0r, t0i, t1r, t1i;
    if constexpr (NPL == 4) {
        double a[4][2];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q][0] = (double)v[q][m].re;
            a[q][1] = (double)v[q][m].im;
        }
        // psi1' = (Cn - i am) psi1 + (-i sig w) psi4
        mul(Cn, -am, a[0][0], a[0][1], t0r, t0i);
        mul(owr, owi, a[3][0], a[3][1], t1r, t1i);
        const double n0r = t0r + t1r, n0i = t0i + t1i;
        // psi4' = (-i sig wb) psi1 + (Cn + i am) psi4
        mul(obr, obi, a[0][0], a[0][1], t0r, t0i);
        mul(Cn, am, a[3][0], a[3][1], t1r, t1i);
        const double n3r = t0r + t1r, n3i = t0i + t1i;
        // psi2' = (Cn - i am) psi2 + (-i sig wb) psi3
        mul(Cn, -am, a[1][0], a[1][1], t0r, t0i);
        mul(obr, obi, a[2][0], a[2][1], t1r, t1i);
        const double n1r = t0r + t1r, n1i = t0i + t1i;
        // psi3' = (-i sig w) psi2 + (Cn + i am) psi3
        mul(owr, owi, a[1][0], a[1][1], t0r, t0i);
        mul(Cn, am, a[2][0], a[2][1], t1r, t1i);
        const double n2r = t0r + t1r, n2i = t0i + t1i;
        v[0][m] = {(R)n0r, (R)n0i};
        v[1][m] = {(R)n1r, (R)n1i};
        v[2][m] = {(R)n2r, (R)n2i};
        v[3][m] = {(R)n3r, (R)n3i};
    } else {
        // pair (1,4): a' = (Cn - i am) a + (-i sig w) b, b' = (-i sig wb) a + (Cn + i am) b;
        // pair (2,3): the same with w and wb exchanged
        const double xr = pair ? obr : owr, xi = pair ? obi : owi;
        const double yr = pair ? owr : obr, yi = pair ? owi : obi;
        const double ar = v[0][m].re, ai = v[0][m].im, br = v[1][m].re, bi = v[1][m].im;
        mul(Cn, -am, ar, ai, t0r, t0i);
        mul(xr, xi, br, bi, t1r, t1i);
        const double nar = t0r + t1r, nai = t0i + t1i;
        mul(yr, yi, ar, ai, t0r, t0i);
        mul(Cn, am, br, bi, t1r, t1i);
        const double nbr = t0r + t1r, nbi = t0i + t1i;
        v[0][m] = {(R)nar, (R)nai};
        v[1][m] = {(R)nbr, (R)nbi};
    }
}

template <typename R, int N, int RAD, int C, int NPL>
__global__ void __launch_bounds__((C * LineShape<N, RAD>::T)) __attribute__((amdgpu_waves_per_eu(2)))
    k_dirac_colpass(cx<R> *__restrict__ psi, int64_t plane, int nx, const TwEntry<R> *__restrict__ tw,
                    DiracKinArgs kin, int mode)
{
    using Sh = LineShape<N, RAD>;
    using Map = ColMap<C>;
    constexpr int T = Sh::T, RV = Sh::RV;
    __shared__ cx<R> lds[Map::slots(N)];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const unsigned G = gridDim.x;
    unsigned L = blockIdx.x;
    if ((G & 7u) == 0) L = (L & 7u) * (G >> 3) + (L >> 3);
    const int pair = NPL == 4 ? 0 : (int)(L & 1u);
    const unsigned cg = NPL == 4 ? L : L >> 1;
    const int64_t col = (int64_t)cg * C + c;
    cx<R> *sh = lds + c;
    // addresses: uniform base of plane q, element m (scalar registers) plus the
    // thread's 32-bit byte offset (t nx + c) (see col_load; the launcher checks the range)
    uint32_t tb = ((uint32_t)t * (uint32_t)nx + (uint32_t)c) * (uint32_t)sizeof(cx<R>);
    auto at = [&](int q, int m) {
        char *b = (char *)(psi + dirac_plane<NPL>(pair, q) * plane + (int64_t)m * T * nx + (int64_t)cg * C);
        __asm__ __volatile__("" : "+s"(b));
        return (cx<R> *)(b + tb);
    };
    TwBase<N, RAD> wb;  // stage factors formed from W^k (see k_dirac_xpass)
    tw_base_load(wb, tw, t);
    cx<R> v[NPL][RV];
#pragma unroll
    for (int q = 0; q < NPL; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) v[q][m] = gload(at(q, m));
    if (mode & M_FWD)
#pragma unroll
        for (int q = 0; q < NPL; ++q) fft_line_pre<R, N, RAD, -1, Map>(v[q], sh, t, tw, wb);
    if (mode & M_KIN) {
        const double px = kin.hbar * kin.kx[col];
#pragma unroll
        for (int m = 0; m < RV; ++m) dirac_kin_point<R, NPL>(v, m, px, kin.hbar * kin.ky[t + m * T], kin, pair);
    }
    if (mode & M_INV)
#pragma unroll
        for (int q = 0; q < NPL; ++q) fft_line_pre<R, N, RAD, +1, Map>(v[q], sh, t, tw, wb);
    __asm__ __volatile__("" : "+v"(tb));
#pragma unroll
    for (int q = 0; q < NPL; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) gstore(at(q, m), v[q][m]);
}

// Tile shapes (kDiracRowVariants, kDiracColVariants): radix, planes per
// work-group (four, or one coupled pair) and, for columns, adjacent lines
// per work-group (64-byte row segments of complex128 at four); rows fill
// 256, 128 or 64 threads (whole rows; more of the smaller work-groups fit a CU).
// Shape 0 of each is the four-plane radix-8 pass.
template <typename R, int N, int V> constexpr bool dirac_row_ok()
{
    constexpr DiracVariant dv = kDiracRowVariants[V];
    using Tl = RowTile<N, dv.rad, dv.threads>;
    return Tl::ROWS * RowMap<R, dv.rad>::slots(N) * (int)sizeof(cx<R>) <= 159 * 1024;
}
template <typename R, int N, int V> constexpr bool dirac_col_ok()
{
    constexpr DiracVariant dv = kDiracColVariants[V];
    return dv.cols * LineShape<N, dv.rad>::T <= 1024 &&
           ColMap<dv.cols>::slots(N) * (int)sizeof(cx<R>) <= 159 * 1024 &&
           (sizeof(R) == 4 || dv.planes == 2 || dv.cols * LineShape<N, dv.rad>::T <= 512);
}

template <typename R, int N, int V>
static hipError_t dirac_x_v(cx<R> *psi, int ny, int64_t plane, const void *V0, const void *const *tw,
                            const DiracPhaseArgs &ph, int mode, hipStream_t st)
{
    if constexpr (!dirac_row_ok<R, N, V>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr DiracVariant dv = kDiracRowVariants[V];
        using Tl = RowTile<N, dv.rad, dv.threads>;
        if (ny % Tl::ROWS) return hipErrorInvalidValue;
        const unsigned groups = (unsigned)(ny / Tl::ROWS) * (dv.planes == 4 ? 1u : 2u);
        hipLaunchKernelGGL((k_dirac_xpass<R, N, dv.rad, dv.planes, dv.threads>), dim3(groups), dim3(Tl::NT), 0, st, psi,
                           plane, (const VStore<R> *)V0, (const TwEntry<R> *)tw[dv.rad == 8 ? 0 : 1], ph, mode);
        return hipGetLastError();
    }
}

template <typename R, int N, int V>
static hipError_t dirac_c_v(cx<R> *psi, int nx, int64_t plane, const void *const *tw, const DiracKinArgs &kin,
                            int mode, hipStream_t st)
{
    if constexpr (!dirac_col_ok<R, N, V>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr DiracVariant dv = kDiracColVariants[V];
        constexpr int C = dv.cols, T = LineShape<N, dv.rad>::T;
        if (nx % C) return hipErrorInvalidValue;
        // per-thread byte offsets within a work-group's columns are 32-bit
        if (((int64_t)(T - 1) * nx + C) * (int64_t)sizeof(cx<R>) > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
        const unsigned groups = (unsigned)(nx / C) * (dv.planes == 4 ? 1u : 2u);
        hipLaunchKernelGGL((k_dirac_colpass<R, N, dv.rad, C, dv.planes>), dim3(groups), dim3(C * T), 0, st, psi,
                           plane, nx, (const TwEntry<R> *)tw[dv.rad == 8 ? 0 : 1], kin, mode);
        return hipGetLastError();
    }
}

template <typename R, int N, size_t... I>
static hipError_t dirac_x_n(int var, cx<R> *psi, int ny, int64_t plane, const void *V0, const void *const *tw,
                            const DiracPhaseArgs &ph, int mode, hipStream_t st, std::index_sequence<I...>)
{
    hipError_t r = hipErrorInvalidValue;
    ((var == (int)I ? (r = dirac_x_v<R, N, (int)I>(psi, ny, plane, V0, tw, ph, mode, st), 0) : 0), ...);
    return r;
}

template <typename R, int N, size_t... I>
static hipError_t dirac_c_n(int var, cx<R> *psi, int nx, int64_t plane, const void *const *tw,
                            const DiracKinArgs &kin, int mode, hipStream_t st, std::index_sequence<I...>)
{
    hipError_t r = hipErrorInvalidValue;
    ((var == (int)I ? (r = dirac_c_v<R, N, (int)I>(psi, nx, plane, tw, kin, mode, st), 0) : 0), ...);
    return r;
}

template <typename R>
hipError_t launch_dirac_xpass(int variant, int N, cx<R> *psi, int ny, int64_t plane, const void *V0,
                              const void *const *tw, const DiracPhaseArgs &ph, int mode, hipStream_t st)
{
#define CALL(n) \
    dirac_x_n<R, n>(variant, psi, ny, plane, V0, tw, ph, mode, st, std::make_index_sequence<kNumDiracRowVariants>{})
    SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
}

template <typename R>
hipError_t launch_dirac_colpass(int variant, int N, cx<R> *psi, int nx, int64_t plane, const void *const *tw,
                                const DiracKinArgs &kin, int mode, hipStream_t st)
{
#define CALL(n) \
    dirac_c_n<R, n>(variant, psi, nx, plane, tw, kin, mode, st, std::make_index_sequence<kNumDiracColVariants>{})
    SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
}

template <typename R, int N, size_t... I> static bool dirac_row_ok_n(int v, std::index_sequence<I...>)
{
    bool ok = false;
    ((v == (int)I ? (ok = dirac_row_ok<R, N, (int)I>(), 0) : 0), ...);
    return ok;
}
template <typename R, int N, size_t... I> static bool dirac_col_ok_n(int v, std::index_sequence<I...>)
{
    bool ok = false;
    ((v == (int)I ? (ok = dirac_col_ok<R, N, (int)I>(), 0) : 0), ...);
    return ok;
}

template <typename R> bool dirac_row_variant_ok(int variant, int N, int64_t ny)
{
    if (variant < 0 || variant >= kNumDiracRowVariants) return false;
    bool ok = false;
    switch (N) {
#define CASE(n) case n: ok = dirac_row_ok_n<R, n>(variant, std::make_index_sequence<kNumDiracRowVariants>{}); break;
    CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096)
#undef CASE
    default: return false;
    }
    if (!ok) return false;
    const int rad = kDiracRowVariants[variant].rad, thr = kDiracRowVariants[variant].threads;
    const int T = N / (N < rad ? N : rad), rows = thr / T > 0 ? thr / T : 1;
    return ny % rows == 0;
}

template <typename R> bool dirac_col_variant_ok(int variant, int N, int64_t nx)
{
    if (variant < 0 || variant >= kNumDiracColVariants) return false;
    if (nx % kDiracColVariants[variant].cols) return false;
    switch (N) {
#define CASE(n) case n: return dirac_col_ok_n<R, n>(variant, std::make_index_sequence<kNumDiracColVariants>{});
    CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096)
#undef CASE
    default: return false;
    }
}

template bool dirac_row_variant_ok<float>(int, int, int64_t);
template bool dirac_row_variant_ok<double>(int, int, int64_t);
template bool dirac_col_variant_ok<float>(int, int, int64_t);
template bool dirac_col_variant_ok<double>(int, int, int64_t);

// ------------------------------------------------------------- 1-D Dirac --
// The whole run of one line in one work-group: both components in registers
// (cyclic layout), transformed one after the other through the same LDS
// region; the real-space factor exp(-i th) (cos a + i sin a sigma_x) and the
// momentum-space 2x2 factor are applied in FP64 with one rounding.
template <typename R, typename VT, int N, int RAD>
__global__ void __launch_bounds__((LineShape<N, RAD>::T))
    k_dirac1d_run(cx<R> *__restrict__ psi, const VT *__restrict__ V0, const TwEntry<R> *__restrict__ tw,
                  Dirac1DArgs a)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    __shared__ cx<R> sh[RowMap<R, RAD>::slots(N)];
    const int t = threadIdx.x;
    cx<R> v[2][RV];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) v[q][m] = gload(psi + (int64_t)q * N + t + m * T);
    auto abar = [&](int64_t st, int x) { return a.abar ? a.abar[st * N + x] : 0.0; };
    // halves of steps sa and sb (sb < 0: one half)
    auto potential = [&](int64_t sa, int64_t sb) {
        const double w = sb >= 0 ? 2.0 : 1.0;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            // an opaque index pins this point's table reads here (they do not
            // depend on the state; the compiler would issue them all at once)
            int x = t + m * T;
            __asm__ __volatile__("" : "+v"(x));
            const double th = w * a.aV_half * ldv(V0 + x);
            const double aa = a.aA * (abar(sa, x) + (sb >= 0 ? abar(sb, x) : 0.0));
            double s, c, sa_, ca;
            sincos_fp64(th, s, c);
            sincos_fp64(aa, sa_, ca);
            const double ur = v[0][m].re, ui = v[0][m].im, vr = v[1][m].re, vi = v[1][m].im;
            // (cos a u + i sin a v, i sin a u + cos a v), then times exp(-i th) = (c - i s)
            const double pr = ca * ur - sa_ * vi, pi = ca * ui + sa_ * vr;
            const double qr = ca * vr - sa_ * ui, qi = ca * vi + sa_ * ur;
            v[0][m] = {(R)(c * pr + s * pi), (R)(c * pi - s * pr)};
            v[1][m] = {(R)(c * qr + s * qi), (R)(c * qi - s * qr)};
            if ((m & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
    };
    if (a.nsteps > 0) potential(a.step0, -1);
#pragma unroll 1
    for (int64_t s = 0; s < a.nsteps; ++s) {
        __asm__ __volatile__("" ::: "memory");
#pragma unroll
        for (int q = 0; q < 2; ++q) fft_line<R, N, RAD, -1, RowMap<R, RAD>>(v[q], sh, t, tw);
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            int k = t + m * T;
            __asm__ __volatile__("" : "+v"(k));
            const double2 u00 = a.u[3 * k], u01 = a.u[3 * k + 1], u11 = a.u[3 * k + 2];
            const double ur = v[0][m].re, ui = v[0][m].im, vr = v[1][m].re, vi = v[1][m].im;
            v[0][m] = {(R)(u00.x * ur - u00.y * ui + u01.x * vr - u01.y * vi),
                       (R)(u00.x * ui + u00.y * ur + u01.x * vi + u01.y * vr)};
            v[1][m] = {(R)(u01.x * ur - u01.y * ui + u11.x * vr - u11.y * vi),
                       (R)(u01.x * ui + u01.y * ur + u11.x * vi + u11.y * vr)};
            if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) fft_line<R, N, RAD, +1, RowMap<R, RAD>>(v[q], sh, t, tw);
        const bool more = s + 1 < a.nsteps;
        potential(a.step0 + s, more ? a.step0 + s + 1 : -1);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) gstore(psi + (int64_t)q * N + t + m * T, v[q][m]);
}

// tws[0], tws[1]: the line's stage twiddles for radix 8 and 16.  Long lines
// use radix 8 (more threads, half the registers per thread for the two
// components).
template <typename R, int N>
static hipError_t dirac1d_n(cx<R> *psi, const void *V0, const void *const *tws, const Dirac1DArgs &a,
                            hipStream_t st)
{
    using VT = typename std::conditional<sizeof(R) == 4, float, double>::type;
    constexpr int RAD = N >= 4096 ? 8 : 16;
    hipLaunchKernelGGL((k_dirac1d_run<R, VT, N, RAD>), dim3(1), dim3(LineShape<N, RAD>::T), 0, st, psi,
                       (const VT *)V0, (const TwEntry<R> *)tws[RAD == 8 ? 0 : 1], a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_dirac1d(int N, cx<R> *psi, const void *V0, const void *const *tw, const Dirac1DArgs &a,
                          hipStream_t st)
{
    switch (N) {
    case 64: return dirac1d_n<R, 64>(psi, V0, tw, a, st);
    case 128: return dirac1d_n<R, 128>(psi, V0, tw, a, st);
    case 256: return dirac1d_n<R, 256>(psi, V0, tw, a, st);
    case 512: return dirac1d_n<R, 512>(psi, V0, tw, a, st);
    case 1024: return dirac1d_n<R, 1024>(psi, V0, tw, a, st);
    case 2048: return dirac1d_n<R, 2048>(psi, V0, tw, a, st);
    case 4096: return dirac1d_n<R, 4096>(psi, V0, tw, a, st);
    case 8192: return dirac1d_n<R, 8192>(psi, V0, tw, a, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_dirac1d<float>(int, cx<float> *, const void *, const void *const *,
                                          const Dirac1DArgs &, hipStream_t);
template hipError_t launch_dirac1d<double>(int, cx<double> *, const void *, const void *const *,
                                           const Dirac1DArgs &, hipStream_t);

template hipError_t launch_dirac_xpass<float>(int, int, cx<float> *, int, int64_t, const void *, const void *const *,
                                              const DiracPhaseArgs &, int, hipStream_t);
template hipError_t launch_dirac_xpass<double>(int, int, cx<double> *, int, int64_t, const void *, const void *const *,
                                               const DiracPhaseArgs &, int, hipStream_t);
template hipError_t launch_dirac_colpass<float>(int, int, cx<float> *, int, int64_t, const void *const *,
                                                const DiracKinArgs &, int, hipStream_t);
template hipError_t launch_dirac_colpass<double>(int, int, cx<double> *, int, int64_t, const void *const *,
                                                 const DiracKinArgs &, int, hipStream_t);

}  // namespace sfo
