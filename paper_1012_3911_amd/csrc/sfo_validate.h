// Argument validation of the C ABI: plain host C++ (no HIP), so that the
// checks the library applies before it touches a device or replaces a table
// can also be built and exercised on their own (under the address and
// undefined-behaviour sanitizers, tests/test_sanitizers.py).  Each check
// returns SFO_OK or the status the ABI reports, with the reason in *why.
#pragma once
#include <stdint.h>

#include <cmath>
#include <cstdio>
#include <string>

#include "sfo.h"

namespace sfo {

// Line lengths of the row/column passes and of the whole-run 1-D kernels.
constexpr int kMaxPassN = 4096;
constexpr int kMax1DN = 8192;
constexpr int kMinN = 64;

// Longest field or vector-potential table a grid accepts, in steps, and the
// largest host table (bytes) the vector tables may take.
constexpr int64_t kMaxTableSteps = int64_t(1) << 28;
constexpr double kMaxTableBytes = double(int64_t(1) << 30);

// Largest state component the passes address (32-bit byte offsets from a
// scalar base: at most N / 8 lines of stride <= plane / N apart stay below
// 2^32 for a plane of at most 2^35 bytes).
constexpr int64_t kMaxPlaneBytes = int64_t(1) << 35;

namespace check {

inline bool is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

inline sfo_status fail(std::string *why, sfo_status s, const char *fmt, long long a = 0, long long b = 0,
                       long long c = 0)
{
    if (why) {
        char buf[256];
        std::snprintf(buf, sizeof buf, fmt, a, b, c);
        *why = buf;
    }
    return s;
}

// sfo_create_grid's descriptor: everything it checks before it asks for a
// device.  *ntot_out (if not null) receives the number of grid points.
inline sfo_status grid_desc(const sfo_grid_desc *desc, std::string *why, int64_t *ntot_out = nullptr)
{
    if (!desc) return fail(why, SFO_E_INVALID, "null descriptor");
    const sfo_grid_desc &d = *desc;
    if (d.ndim < 1 || d.ndim > 3) return fail(why, SFO_E_INVALID, "ndim must be 1, 2 or 3 (got %lld)", d.ndim);
    if (d.equation != SFO_SCHRODINGER && d.equation != SFO_DIRAC)
        return fail(why, SFO_E_INVALID, "unknown equation %lld", d.equation);
    if (d.dtype != SFO_C64 && d.dtype != SFO_C128) return fail(why, SFO_E_INVALID, "unknown dtype %lld", d.dtype);
    if (!(d.dt > 0) || !std::isfinite(d.dt)) return fail(why, SFO_E_INVALID, "dt must be positive and finite");
    if (!(d.hbar > 0) || !(d.mass > 0) || !std::isfinite(d.hbar) || !std::isfinite(d.mass))
        return fail(why, SFO_E_INVALID, "hbar and mass must be positive and finite");
    if (!std::isfinite(d.charge)) return fail(why, SFO_E_INVALID, "charge must be finite");
    if (d.equation == SFO_DIRAC && (d.ndim > 2 || !(d.c > 0) || !std::isfinite(d.c)))
        return fail(why, SFO_E_INVALID, "Dirac needs ndim 1 or 2 and a finite c > 0");
    int64_t ntot = 1;
    for (int a = 0; a < d.ndim; ++a) {
        if (!is_pow2(d.n[a]))
            return fail(why, SFO_E_INVALID, "n[%lld] = %lld is not a power of two", a, (long long)d.n[a]);
        if (!(d.xmax[a] > d.xmin[a]) || !std::isfinite(d.xmin[a]) || !std::isfinite(d.xmax[a]) ||
            !std::isfinite(d.xmax[a] - d.xmin[a]))
            return fail(why, SFO_E_INVALID, "axis %lld: need finite xmin < xmax", a);
        const int64_t maxn = d.ndim == 1 ? kMax1DN : kMaxPassN;
        if (d.n[a] < kMinN || d.n[a] > maxn)
            return fail(why, SFO_E_UNSUPPORTED, "n[%lld] = %lld outside the supported 64..%lld", a,
                        (long long)d.n[a], (long long)maxn);
        ntot *= d.n[a];  // at most 4096^3: no overflow
    }
    const int64_t plane_bytes = ntot * (d.dtype == SFO_C128 ? 16 : 8);
    if (plane_bytes > kMaxPlaneBytes)
        return fail(why, SFO_E_UNSUPPORTED, "a state of %lld bytes per component exceeds the 32 GiB the passes address",
                    (long long)plane_bytes);
    if (ntot_out) *ntot_out = ntot;
    return SFO_OK;
}

// A per-step host table of nsteps x per_step finite doubles (nsteps = 0
// clears; host may then be null), of at most kMaxTableSteps steps and, when
// max_bytes > 0, at most max_bytes of per-step entries of entry_bytes each.
inline sfo_status step_table(const double *host, int64_t nsteps, int64_t per_step, double entry_bytes,
                             double max_bytes, const char *what, std::string *why)
{
    if (nsteps < 0 || per_step < 1 || (nsteps > 0 && !host))
        return fail(why, SFO_E_INVALID, "bad table (steps %lld, entries per step %lld)", (long long)nsteps,
                    (long long)per_step);
    if (nsteps > kMaxTableSteps ||
        (max_bytes > 0 && (double)nsteps * (double)per_step * entry_bytes > max_bytes)) {
        std::string w = std::string(what) + " tables of %lld steps are beyond the supported size";
        return fail(why, SFO_E_UNSUPPORTED, w.c_str(), (long long)nsteps);
    }
    const int64_t count = nsteps * per_step;  // below 2^28 * 2^13 * 3: no overflow
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(host[i])) {
            std::string w = std::string(what) + " table holds a non-finite value at entry %lld";
            return fail(why, SFO_E_INVALID, w.c_str(), (long long)i);
        }
    return SFO_OK;
}

// Steps step0 .. step0 + nsteps - 1 against a table of table_steps steps
// (0: no table, every step allowed).
inline sfo_status step_range(int64_t step0, int64_t nsteps, int64_t table_steps, const char *what, std::string *why)
{
    if (step0 < 0 || nsteps < 0) return fail(why, SFO_E_INVALID, "negative step index or count");
    if (table_steps > 0 && (step0 > table_steps || nsteps > table_steps - step0)) {
        std::string w = std::string("steps %lld.. (%lld of them) exceed the ") + what + " table (%lld steps)";
        return fail(why, SFO_E_INVALID, w.c_str(), (long long)step0, (long long)nsteps, (long long)table_steps);
    }
    return SFO_OK;
}

}  // namespace check
}  // namespace sfo
