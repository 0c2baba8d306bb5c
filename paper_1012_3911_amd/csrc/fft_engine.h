// In-workgroup Stockham FFT engine for gfx950 (wave64, LDS exchange).
//
// A line of N complex values is spread over T = N/RV threads, each holding
// RV values in registers in CYCLIC order: thread t owns x[t + m*T],
// m = 0..RV-1.  The transform is a sequence of Stockham autosort stages
// (radix r, span L = product of the earlier radices):
//     butterfly b in [0, N/r):  k = b mod L,  j0 = b / L
//     inputs  x[b + j N/r], j < r, the j-th scaled by W_{L r}^{j k}
//     r-point DFT, output m to position j0 L r + k + m L.
// With the cyclic layout every stage reads its butterfly inputs from the
// thread's own registers, and the LAST stage (L r = N, so j0 = 0) writes its
// outputs back into the same cyclic layout.  Only intermediate stages go
// through LDS, so a forward transform, a point-wise factor and an inverse
// transform chain with no exchange between them.
//
// Precision.  Twiddles come from FP64 tables.  For complex64 a stage reads
// only W^k of each butterfly (stored as an FP32 hi/lo pair, exact to about
// 2^-48) and forms the other factors W^{jk} from it in FP64 by a few
// products; each factor is applied in FP64 and rounded to FP32 once.  The
// internal constants of the radix-8/16 codelets are FP32 hi/lo pairs applied
// with FMAs.  Either way the rounded twiddle's modulus error (about 3e-8 for
// angles near 45 degrees in plain FP32, the same for every step) does not
// turn into a systematic norm drift; what remains is the rounding of each
// arithmetic result, which is not systematic.  Complex128 reads every factor
// from its FP64 table.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace sfo {

template <typename R>
struct __align__(2 * sizeof(R)) cx {
    R re, im;
};

// Global-memory access.  The state, potential and accumulator pointers of the
// passes always address device memory, but pointers taken from argument
// structures or batch descriptors reach the compiler as generic pointers,
// which it accesses with flat instructions.  A flat access also counts
// against the LDS wait counter, so each wait for an LDS exchange would wait
// for outstanding loads as well, and it cannot take a scalar base address.
// These accessors state the address space.
template <typename R> struct Vec2T;
template <> struct Vec2T<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <> struct Vec2T<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <typename R> __device__ __forceinline__ cx<R> gload(const cx<R> *p)
{
    typedef typename Vec2T<R>::type V;
    const V v = *(const __attribute__((address_space(1))) V *)p;
    return {v.x, v.y};
}
template <typename R> __device__ __forceinline__ void gstore(cx<R> *p, cx<R> a)
{
    typedef typename Vec2T<R>::type V;
    V v;
    v.x = a.re;
    v.y = a.im;
    *(__attribute__((address_space(1))) V *)p = v;
}
template <typename T> __device__ __forceinline__ T gload1(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}
template <typename T> __device__ __forceinline__ void gstore1(T *p, T a)
{
    *(__attribute__((address_space(1))) T *)p = a;
}

// Twiddle table entry: FP32 hi/lo pair for complex64, plain FP64 for complex128.
template <typename R> struct TwEntry;
template <> struct __align__(16) TwEntry<float> { float hr, hi, lr, li; };
template <> struct __align__(16) TwEntry<double> { double r, i; };

template <typename R> __device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }

// a * exp(DIR * i pi/2): DIR = -1 gives -i a, DIR = +1 gives i a (exact).
template <int DIR, typename R> __device__ __forceinline__ cx<R> mul_quarter(cx<R> a)
{
    if (DIR < 0) return {a.im, -a.re};
    return {-a.im, a.re};
}

// a * (wr + i wi) with the twiddle given as an FP32 hi/lo pair.  The small
// products with the lo parts are summed FIRST and each later FMA rounds the
// complete partial value, so the lo parts are not absorbed: adding them to an
// already rounded product would drop them below half an ulp and leave the
// rounded twiddle's modulus error in place, a norm loss of a few 1e-8 per
// multiply that repeats identically every step.
__device__ __forceinline__ cx<float> cmul_hl(cx<float> a, float hr, float hi, float lr, float li)
{
    float re = __builtin_fmaf(a.re, lr, -(a.im * li));
    re = __builtin_fmaf(-a.im, hi, re);
    re = __builtin_fmaf(a.re, hr, re);
    float im = __builtin_fmaf(a.re, li, a.im * lr);
    im = __builtin_fmaf(a.im, hr, im);
    im = __builtin_fmaf(a.re, hi, im);
    return {re, im};
}

__device__ __forceinline__ cx<double> cmul_d(cx<double> a, double wr, double wi)
{
    return {__builtin_fma(a.re, wr, -(a.im * wi)), __builtin_fma(a.re, wi, a.im * wr)};
}

// Table twiddle W_N^(c + k) (forward table), conjugated for the inverse
// transform.  c is a compile-time entry index and kb = k * sizeof(TwEntry)
// the thread's unsigned byte offset, so that the address is a uniform base
// plus a 32-bit vector offset (no 64-bit vector arithmetic per load).
template <int DIR>
__device__ __forceinline__ cx<float> twiddle(cx<float> a, const TwEntry<float> *tw, int c, uint32_t kb)
{
    TwEntry<float> w = *(const TwEntry<float> *)((const char *)(tw + c) + kb);
    if (DIR > 0) { w.hi = -w.hi; w.li = -w.li; }
    return cmul_hl(a, w.hr, w.hi, w.lr, w.li);
}
template <int DIR>
__device__ __forceinline__ cx<double> twiddle(cx<double> a, const TwEntry<double> *tw, int c, uint32_t kb)
{
    TwEntry<double> w = *(const TwEntry<double> *)((const char *)(tw + c) + kb);
    return cmul_d(a, w.r, DIR > 0 ? -w.i : w.i);
}

// W_N^(c + k) of the forward table in FP64 (complex64 entries: hi + lo).
__device__ __forceinline__ void twiddle_base(const TwEntry<float> *tw, int c, uint32_t kb, double &wr, double &wi)
{
    const TwEntry<float> e = *(const TwEntry<float> *)((const char *)(tw + c) + kb);
    wr = (double)e.hr + (double)e.lr;
    wi = (double)e.hi + (double)e.li;
}

// (a + i b) (c + i d) in FP64.
__device__ __forceinline__ void cmul64(double &a, double &b, double c, double d)
{
    const double r = a * c - b * d;
    b = a * d + b * c;
    a = r;
}

// v * (c + i s) in FP64, rounded once.
__device__ __forceinline__ cx<float> mul_round(cx<float> v, double c, double s)
{
    const double re = (double)v.re * c - (double)v.im * s;
    const double im = (double)v.re * s + (double)v.im * c;
    return {(float)re, (float)im};
}

// cos(2 pi k / 16), k = 0..15 (FP64 constants of the radix-8/16 codelets).
__host__ __device__ constexpr double cos16(int k)
{
    constexpr double c[16] = {1.0,
                              0.92387953251128675613,
                              0.70710678118654752440,
                              0.38268343236508977173,
                              0.0,
                              -0.38268343236508977173,
                              -0.70710678118654752440,
                              -0.92387953251128675613,
                              -1.0,
                              -0.92387953251128675613,
                              -0.70710678118654752440,
                              -0.38268343236508977173,
                              0.0,
                              0.38268343236508977173,
                              0.70710678118654752440,
                              0.92387953251128675613};
    return c[k & 15];
}
__host__ __device__ constexpr double sin16(int k) { return cos16((k + 12) & 15); }

// a * W_NR^E for the codelet constants, W = exp(DIR 2 pi i / NR), NR | 16.
template <int DIR, int NR, int E, typename R> __device__ __forceinline__ cx<R> cmul_const(cx<R> a)
{
    constexpr int e16 = ((E * (16 / NR)) % 16 + 16) % 16;
    if constexpr (e16 == 0) {
        return a;
    } else if constexpr (e16 == 8) {
        return {-a.re, -a.im};
    } else if constexpr (e16 == 4) {
        return mul_quarter<DIR>(a);
    } else if constexpr (e16 == 12) {
        return mul_quarter<-DIR>(a);
    } else if constexpr ((e16 & 3) == 2) {
        // odd multiple of 45 degrees: W = h (sr + i si), h = sqrt(1/2), sr, si = +-1
        constexpr double sr = cos16(e16) > 0 ? 1.0 : -1.0;
        constexpr double si = (DIR < 0 ? -1.0 : 1.0) * (sin16(e16) > 0 ? 1.0 : -1.0);
        const R u = sr > 0 ? (si > 0 ? a.re - a.im : a.re + a.im) : (si > 0 ? -a.re - a.im : -a.re + a.im);
        const R w = si > 0 ? (sr > 0 ? a.re + a.im : a.re - a.im) : (sr > 0 ? -a.re + a.im : -a.re - a.im);
        constexpr double h = 0.70710678118654752440;
        if constexpr (sizeof(R) == 4) {
            constexpr float hh = (float)h, hl = (float)(h - (double)hh);
            return {__builtin_fmaf(u, hh, u * hl), __builtin_fmaf(w, hh, w * hl)};
        } else {
            return {u * h, w * h};
        }
    } else {
        constexpr double wr = cos16(e16);
        constexpr double wi = (DIR < 0 ? -1.0 : 1.0) * sin16(e16);
        if constexpr (sizeof(R) == 4) {
            constexpr float hr = (float)wr, hi = (float)wi;
            constexpr float lr = (float)(wr - (double)hr), li = (float)(wi - (double)hi);
            return cmul_hl(a, hr, hi, lr, li);
        } else {
            return cmul_d(a, wr, wi);
        }
    }
}

template <int NR, int DIR, int N1, int N2, int J2 = 0, int M1 = 0, typename R>
__device__ __forceinline__ void twiddle_grid(cx<R> (&a)[N2][N1])
{
    if constexpr (J2 < N2) {
        if constexpr (M1 < N1) {
            a[J2][M1] = cmul_const<DIR, NR, J2 * M1>(a[J2][M1]);
            twiddle_grid<NR, DIR, N1, N2, J2, M1 + 1>(a);
        } else {
            twiddle_grid<NR, DIR, N1, N2, J2 + 1, 0>(a);
        }
    }
}

// In-register DFT of size NR (1, 2, 4, 8, 16), natural order in and out:
// y_m = sum_j v_j exp(DIR 2 pi i j m / NR).  Sizes above 4 split as 4 x NR/4.
template <int NR, int DIR, typename R> __device__ __forceinline__ void dft(cx<R> *v)
{
    if constexpr (NR == 1) {
        return;
    } else if constexpr (NR == 2) {
        cx<R> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (NR == 4) {
        cx<R> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        cx<R> s13 = cadd(v[1], v[3]), d13 = mul_quarter<DIR>(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else {
        constexpr int N1 = 4, N2 = NR / 4;
        cx<R> a[N2][N1];
#pragma unroll
        for (int j2 = 0; j2 < N2; ++j2) {
#pragma unroll
            for (int j1 = 0; j1 < N1; ++j1) a[j2][j1] = v[N2 * j1 + j2];
            dft<N1, DIR>(a[j2]);
        }
        // twiddles W_NR^{j2 m1}
        twiddle_grid<NR, DIR, N1, N2>(a);
#pragma unroll
        for (int m1 = 0; m1 < N1; ++m1) {
            cx<R> b[N2];
#pragma unroll
            for (int j2 = 0; j2 < N2; ++j2) b[j2] = a[j2][m1];
            dft<N2, DIR>(b);
#pragma unroll
            for (int m2 = 0; m2 < N2; ++m2) v[m1 + N1 * m2] = b[m2];
        }
    }
}

#ifndef SFO_TW_GROUPED
#define SFO_TW_GROUPED 1
#endif

// Stage twiddles and DFT of size NR = 8 or 16 in one pass: the twiddles of
// the four inputs of each first-layer 4-point DFT are fetched and applied
// just before it, so that at most four table entries are live at a time
// instead of NR - 1 (for complex64 each entry is an FP32 hi/lo pair, four
// registers).  Same arithmetic as twiddle() followed by dft<NR>().
template <int NR, int DIR, bool PRE, typename R, typename TW>
__device__ __forceinline__ void tw_dft(cx<R> *v, const TW *__restrict__ tw, int two, int L, int k, double pwr,
                                       double pwi)
{
    constexpr int N1 = 4, N2 = NR / 4;
    cx<R> a[N2][N1];
    if constexpr (std::is_same<R, float>::value || PRE) {
        // complex64: W^k (read here, or PRE: read at the start of the pass,
        // pwr + i pwi); the factor of input j = j2 + N2 j1 is
        // W^{k j2} (W^{k N2})^{j1}, each formed by at most N2 - 1 + 3 + 3 FP64
        // products from W^k.  Complex128 with PRE (a pass that reads no table
        // during its transforms) forms its factors the same way and applies
        // them in FP64.
        double wr = pwr, wi = pwi;
        if constexpr (!PRE) {
            uint32_t kb = (uint32_t)k * (uint32_t)sizeof(TW);
            __asm__ __volatile__("" : "+v"(kb));
            twiddle_base(tw, two, kb, wr, wi);
        } else {
            // opaque copies: the factors of two transforms of the same line
            // (two states, or the forward and inverse transforms) are then
            // formed afresh in each instead of being kept live between them
            __asm__ __volatile__("" : "+v"(wr), "+v"(wi));
        }
        if (DIR > 0) wi = -wi;
        double sr = wr, si = wi;  // W^{k N2}
#pragma unroll
        for (int q = 1; q < N2; q *= 2) cmul64(sr, si, sr, si);
        double gr = 1.0, gi = 0.0;  // W^{k j2}
#pragma unroll
        for (int j2 = 0; j2 < N2; ++j2) {
            double cr = gr, ci = gi;
#pragma unroll
            for (int j1 = 0; j1 < N1; ++j1) {
                const int j = N2 * j1 + j2;
                if constexpr (std::is_same<R, float>::value)
                    a[j2][j1] = j == 0 ? v[0] : mul_round(v[j], cr, ci);
                else
                    a[j2][j1] = j == 0 ? v[0] : cmul_d(v[j], cr, ci);
                if (j1 + 1 < N1) cmul64(cr, ci, sr, si);
            }
            dft<N1, DIR>(a[j2]);
            if (j2 + 1 < N2) cmul64(gr, gi, wr, wi);
        }
    } else {
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2) {
        // an opaque copy of the index pins this group's table loads here: the
        // table is read-only, and the compiler would otherwise issue every
        // load of the transform at its start and hold them all in registers
        uint32_t kb = (uint32_t)k * (uint32_t)sizeof(TW);
        __asm__ __volatile__("" : "+v"(kb));
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) {
            const int j = N2 * j1 + j2;
            a[j2][j1] = j == 0 ? v[0] : twiddle<DIR>(v[j], tw, two + (j - 1) * L, kb);
        }
        dft<N1, DIR>(a[j2]);
    }
    }
    twiddle_grid<NR, DIR, N1, N2>(a);
#pragma unroll
    for (int m1 = 0; m1 < N1; ++m1) {
        cx<R> b[N2];
#pragma unroll
        for (int j2 = 0; j2 < N2; ++j2) b[j2] = a[j2][m1];
        dft<N2, DIR>(b);
#pragma unroll
        for (int m2 = 0; m2 < N2; ++m2) v[m1 + N1 * m2] = b[m2];
    }
}

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// LDS placement of element p of a line during an exchange.  Two kinds:
//
// Padded maps, at(p) = (p + (p >> SH)) * C (one pad slot every 2^SH
// elements; C lines interleaved, lane c at offset c).  Every Stockham access
// pattern then splits into a per-thread base and compile-time offsets:
// positions base + d with d = m L (writes: base = j0 L r + k, k < L, L and r
// powers of two) or d = m T (reads: base = t < T) satisfy
//     at(base + d) = at(base) + off(d),  off(d) = (d + (d >> SH)) * C,
// because either d is a multiple of 2^SH, or the base's low part plus d stays
// inside one block of 2^SH (L divides 2^SH and k < L).  The offsets become
// immediate fields of the LDS instructions: no address arithmetic per element.
//
// The XOR map (the default for radix-8 rows) permutes the low address bits
// inside aligned blocks of 32 and needs an address per element; its bank
// conflicts are lower for that shape.  The shifts were chosen with a 64-bank, 4-byte-word model of
// the LDS over the write and read patterns of every stage for N = 256..4096.
template <typename R, int RAD, bool PAD = (RAD == 16)> struct RowMap {
    static constexpr bool TW_AT_ONCE_FP64 = false;
    static constexpr bool AFFINE = PAD;
    static constexpr int SH = AFFINE ? (sizeof(R) == 4 ? 5 : 4) : 3;
    static constexpr int MASK = sizeof(R) == 4 ? 31 : 15;
    __device__ static int at(int p) { return AFFINE ? p + (p >> SH) : p ^ ((p >> SH) & MASK); }
    __host__ __device__ static constexpr int off(int d) { return d + (d >> SH); }
    static constexpr int slots(int N) { return AFFINE ? N + (N >> SH) : N; }
};
template <int C> struct ColMap {
    static constexpr bool AFFINE = true;
    // complex128 column transforms read all of a stage's twiddles at its start
    // (measured faster: one table latency per stage; their few waves per SIMD
    // leave the registers for it)
    static constexpr bool TW_AT_ONCE_FP64 = true;
    __device__ static int at(int p) { return (p + (p >> 3)) * C; }
    __host__ __device__ static constexpr int off(int d) { return (d + (d >> 3)) * C; }
    static constexpr int slots(int N) { return (N + N / 8) * C; }
};

// Shape of an N-point line transform with RAD values per thread.
template <int N, int RAD> struct LineShape {
    static constexpr int RV = N < RAD ? N : RAD;         // values per thread
    static constexpr int T = N / RV;                     // threads per line
    static constexpr int LOGR = ilog2(RV);
    static constexpr int NFULL = LOGR ? ilog2(N) / LOGR : 0;
    static constexpr int REM = N >> (NFULL * LOGR);      // leading small radix, 1 if none
    static constexpr int NST = NFULL + (REM > 1 ? 1 : 0);
    static constexpr int radix(int s) { return (REM > 1 && s == 0) ? REM : RV; }
    static constexpr int span(int s) { return s == 0 ? 1 : span(s - 1) * radix(s - 1); }
    // Stage twiddle table: stage s (span L > 1, radix r) stores W_{L r}^{j k} at
    // tw_offset(s) + (j - 1) L + k, j = 1..r-1, k = 0..L-1, so that the lanes of a
    // wave (consecutive k) read consecutive entries.
    static constexpr int tw_offset(int s) { return s <= 1 ? 0 : tw_offset(s - 1) + (radix(s - 1) - 1) * span(s - 1); }
    static constexpr int TW_SIZE = tw_offset(NST);
};

// W^k in FP64 of the thread's butterfly in each twiddled stage (S >= 1, one
// butterfly per thread there) of an N-point line, read once per pass so that
// the complex64 transforms of the pass read no table (see tw_dft).
template <int N, int RAD> struct TwBase {
    static constexpr int NT = LineShape<N, RAD>::NST > 1 ? LineShape<N, RAD>::NST - 1 : 1;
    double r[NT], i[NT];
};
template <int N, int RAD, int S = 1>
__device__ __forceinline__ void tw_base_load(TwBase<N, RAD> &w, const TwEntry<float> *__restrict__ tw, int t)
{
    using Sh = LineShape<N, RAD>;
    if constexpr (S < Sh::NST) {
        static_assert(Sh::RV / Sh::radix(S) == 1, "one butterfly per thread in a twiddled stage");
        // both evaluated here at compile time (as call arguments the recursive
        // constexpr functions can end up as run-time calls with a stack frame)
        constexpr int L = Sh::span(S), TWO = Sh::tw_offset(S);
        twiddle_base(tw, TWO, (uint32_t)(t & (L - 1)) * (uint32_t)sizeof(TwEntry<float>), w.r[S - 1], w.i[S - 1]);
        tw_base_load<N, RAD, S + 1>(w, tw, t);
    }
}

template <int N, int RAD, int S = 1>
__device__ __forceinline__ void tw_base_load(TwBase<N, RAD> &w, const TwEntry<double> *__restrict__ tw, int t)
{
    using Sh = LineShape<N, RAD>;
    if constexpr (S < Sh::NST) {
        static_assert(Sh::RV / Sh::radix(S) == 1, "one butterfly per thread in a twiddled stage");
        constexpr int L = Sh::span(S), TWO = Sh::tw_offset(S);  // compile time (see above)
        const TwEntry<double> e = tw[TWO + (t & (L - 1))];
        w.r[S - 1] = e.r;
        w.i[S - 1] = e.i;
        tw_base_load<N, RAD, S + 1>(w, tw, t);
    }
}

// One Stockham stage S of an N-point transform (see the file comment).
// v: the thread's RV cyclic values; sh: this line's LDS region; t: thread in
// line; tw: the stage twiddle table of this (N, RAD).
template <typename R, int N, int RAD, int DIR, int S, class MAP, bool PRE, int NV>
__device__ __forceinline__ void fft_stage(cx<R> (&v)[NV], cx<R> *sh, int t, const TwEntry<R> *__restrict__ tw,
                                          const TwBase<N, RAD> &wb, bool act = true)
{
    using Sh = LineShape<N, RAD>;
    static_assert(NV == Sh::RV, "register array size must match the line shape");
    // keep the scheduler from pulling the next stage's table loads (and their
    // registers) ahead into this one
    __builtin_amdgcn_sched_barrier(0);
    constexpr int RV = Sh::RV, T = Sh::T;
    constexpr int r = Sh::radix(S), L = Sh::span(S), NB = RV / r;
    constexpr bool last = (S == Sh::NST - 1);
    constexpr int TWO = Sh::tw_offset(S);
    // act = false: a thread beyond this line's T threads (a work-group sized for
    // a longer line) keeps step with the barriers and touches nothing
    if (act) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        cx<R> u[r];
#pragma unroll
        for (int j = 0; j < r; ++j) u[j] = v[i + j * NB];
        const int b = t + i * T;
        const int k = b & (L - 1);
        if constexpr (L > 1 && r >= 8 && SFO_TW_GROUPED &&
                      (PRE || !(MAP::TW_AT_ONCE_FP64 && std::is_same<R, double>::value))) {
            constexpr int WB = S >= 1 ? S - 1 : 0;
            tw_dft<r, DIR, PRE>(u, tw, TWO, L, k, PRE ? wb.r[WB] : 0.0, PRE ? wb.i[WB] : 0.0);
        } else {
            if constexpr (L > 1) {
                // pins the table loads to this stage (see tw_dft)
                uint32_t kb = (uint32_t)k * (uint32_t)sizeof(TwEntry<R>);
                __asm__ __volatile__("" : "+v"(kb));
                if constexpr (std::is_same<R, float>::value || PRE) {
                    // complex64 (and complex128 with PRE): W^{jk} = (W^k)^j in FP64
                    // from the one table value
                    double wr, wi;
                    if constexpr (PRE) {
                        static_assert(NB == 1, "one butterfly per thread in a twiddled stage");
                        wr = wb.r[S - 1];
                        wi = wb.i[S - 1];
                        __asm__ __volatile__("" : "+v"(wr), "+v"(wi));  // see tw_dft
                    } else {
                        twiddle_base(tw, TWO, kb, wr, wi);
                    }
                    if (DIR > 0) wi = -wi;
                    double cr = wr, ci = wi;
#pragma unroll
                    for (int j = 1; j < r; ++j) {
                        if constexpr (std::is_same<R, float>::value)
                            u[j] = mul_round(u[j], cr, ci);
                        else
                            u[j] = cmul_d(u[j], cr, ci);
                        if (j + 1 < r) cmul64(cr, ci, wr, wi);
                    }
                } else {
#pragma unroll
                    for (int j = 1; j < r; ++j) u[j] = twiddle<DIR>(u[j], tw, TWO + (j - 1) * L, kb);
                }
            }
            dft<r, DIR>(u);
        }
        if constexpr (last) {
#pragma unroll
            for (int m = 0; m < r; ++m) v[i + m * NB] = u[m];
        } else {
            const int base = (b / L) * (L * r) + k;
            if constexpr (MAP::AFFINE) {
                cx<R> *w = sh + MAP::at(base);
#pragma unroll
                for (int m = 0; m < r; ++m) w[MAP::off(m * L)] = u[m];
            } else {
#pragma unroll
                for (int m = 0; m < r; ++m) sh[MAP::at(base + m * L)] = u[m];
            }
        }
    }
    }
    if constexpr (!last) {
        __syncthreads();
        if (act) {
            if constexpr (MAP::AFFINE) {
                const cx<R> *q = sh + MAP::at(t);
#pragma unroll
                for (int m = 0; m < RV; ++m) v[m] = q[MAP::off(m * T)];
            } else {
#pragma unroll
                for (int m = 0; m < RV; ++m) v[m] = sh[MAP::at(t + m * T)];
            }
        }
        __syncthreads();
    }
}

// Full N-point transform of the thread's cyclic values (direction DIR), with
// the LDS exchanges placed by MAP (RowMap<R, RAD> or ColMap<C>).  PRE: the
// complex64 stage factors come from wb (see TwBase) instead of the table.
// HOOK: called with std::integral_constant<int, S> after stage S (work of
// the caller's placed between the stages, e.g. loads issued in parts).
struct NoStageHook {
    template <int S> __device__ __forceinline__ void operator()(std::integral_constant<int, S>) const {}
};
template <typename R, int N, int RAD, int DIR, class MAP, bool PRE, int S, int NV, class HOOK = NoStageHook>
__device__ __forceinline__ void fft_line_st(cx<R> (&v)[NV], cx<R> *sh, int t, const TwEntry<R> *__restrict__ tw,
                                            const TwBase<N, RAD> &wb, bool act, const HOOK &hook = HOOK{})
{
    if constexpr (S < LineShape<N, RAD>::NST) {
        fft_stage<R, N, RAD, DIR, S, MAP, PRE>(v, sh, t, tw, wb, act);
        hook(std::integral_constant<int, S>{});
        fft_line_st<R, N, RAD, DIR, MAP, PRE, S + 1>(v, sh, t, tw, wb, act, hook);
    }
}

template <typename R, int N, int RAD, int DIR, class MAP, bool PRE, int NV, class HOOK = NoStageHook>
__device__ __forceinline__ void fft_line_impl(cx<R> (&v)[NV], cx<R> *sh, int t, const TwEntry<R> *__restrict__ tw,
                                              const TwBase<N, RAD> &wb, bool act, const HOOK &hook = HOOK{})
{
    // a fresh copy of the thread index per transform: the exchange
    // addresses of two transforms in a row are then not shared (and kept
    // live) between them
    int tt = t;
    __asm__ __volatile__("" : "+v"(tt));
    fft_line_st<R, N, RAD, DIR, MAP, PRE, 0>(v, sh, tt, tw, wb, act, hook);
}

template <typename R, int N, int RAD, int DIR, class MAP, int NV>
__device__ __forceinline__ void fft_line(cx<R> (&v)[NV], cx<R> *sh, int t, const TwEntry<R> *__restrict__ tw,
                                         bool act = true)
{
    TwBase<N, RAD> unused;
    fft_line_impl<R, N, RAD, DIR, MAP, false>(v, sh, t, tw, unused, act);
}

// Either precision with the stage factors formed from wb (PRE): the
// transforms read no table.
template <typename R, int N, int RAD, int DIR, class MAP, int NV, class HOOK = NoStageHook>
__device__ __forceinline__ void fft_line_pre(cx<R> (&v)[NV], cx<R> *sh, int t, const TwEntry<R> *__restrict__ tw,
                                             const TwBase<N, RAD> &wb, const HOOK &hook = HOOK{})
{
    fft_line_impl<R, N, RAD, DIR, MAP, true>(v, sh, t, tw, wb, true, hook);
}

// The same with the stage factors of a complex64 line taken from wb.
template <typename R, int N, int RAD, int DIR, class MAP, int NV>
__device__ __forceinline__ void fft_line(cx<R> (&v)[NV], cx<R> *sh, int t, const TwEntry<R> *__restrict__ tw,
                                         const TwBase<N, RAD> &wb, bool act = true)
{
    fft_line_impl<R, N, RAD, DIR, MAP, std::is_same<R, float>::value>(v, sh, t, tw, wb, act);
}

// ---------------------------------------------------------------- phases --
// exp(-i theta) with theta in FP64.  Range reduction by quadrant with a
// two-term (Cody-Waite) pi/2 and one FMA, then the Taylor series of sin and
// cos on [-pi/4, pi/4] to degree 15/16 (truncation below 5e-17), then the
// quadrant's swap and signs.  Accurate to a few ulp of FP64 for
// |theta| < 1e6, far beyond the phases of a step.
__device__ __forceinline__ void sincos_fp64(double x, double &s, double &c)
{
    const double two_over_pi = 0.63661977236758134308;
    const double pio2_hi = 1.5707963267948966192;     // pi/2 rounded to FP64
    const double pio2_lo = 6.1232339957367658e-17;    // pi/2 - pio2_hi
    const double q = rint(x * two_over_pi);
    const double r = __builtin_fma(-q, pio2_lo, __builtin_fma(-q, pio2_hi, x));
    const double r2 = r * r;
    double ps = -7.6471637318198164759e-13;           // -1/15!
    ps = __builtin_fma(ps, r2, 1.6059043836821614599e-10);  // 1/13!
    ps = __builtin_fma(ps, r2, -2.5052108385441718775e-08); // -1/11!
    ps = __builtin_fma(ps, r2, 2.7557319223985890653e-06);  // 1/9!
    ps = __builtin_fma(ps, r2, -1.9841269841269841270e-04); // -1/7!
    ps = __builtin_fma(ps, r2, 8.3333333333333333333e-03);  // 1/5!
    ps = __builtin_fma(ps, r2, -1.6666666666666666667e-01); // -1/3!
    const double sr = __builtin_fma(ps * r2, r, r);
    double pc = 4.7794773323873852974e-14;            // 1/16!
    pc = __builtin_fma(pc, r2, -1.1470745597729724714e-11); // -1/14!
    pc = __builtin_fma(pc, r2, 2.0876756987868098979e-09);  // 1/12!
    pc = __builtin_fma(pc, r2, -2.7557319223985890653e-07); // -1/10!
    pc = __builtin_fma(pc, r2, 2.4801587301587301587e-05);  // 1/8!
    pc = __builtin_fma(pc, r2, -1.3888888888888888889e-03); // -1/6!
    pc = __builtin_fma(pc, r2, 4.1666666666666666667e-02);  // 1/4!
    pc = __builtin_fma(pc, r2, -0.5);
    const double cr = __builtin_fma(pc, r2, 1.0);
    // quadrant q mod 4 without branches: odd quadrants swap sin and cos,
    // quadrants 2 and 3 negate sin, quadrants 1 and 2 negate cos
    const int quad = (int)q & 3;
    const double ss = (quad & 1) ? cr : sr;
    const double cc = (quad & 1) ? sr : cr;
    s = (quad & 2) ? -ss : ss;
    c = ((quad + 1) & 2) ? -cc : cc;
}

template <typename R> __device__ __forceinline__ cx<R> mul_phase(cx<R> v, double c, double s)
{
    // v * (c + i s) in FP64, rounded once
    double re = (double)v.re * c - (double)v.im * s;
    double im = (double)v.re * s + (double)v.im * c;
    return {(R)re, (R)im};
}

template <typename R> __device__ __forceinline__ cx<R> mul_expmi(cx<R> v, double th)
{
    double s, c;
    sincos_fp64(th, s, c);
    return mul_phase(v, c, -s);
}

}  // namespace sfo
