// Instantiations of the row (x) pass for complex64 and complex128.
#include <type_traits>

#include "pass_kernels.h"

namespace sfo {

template <typename R>
hipError_t launch_xpass(int variant, int N, int ns, const StatePtrs<R> &S, int64_t nrows, int ny, const void *V0,
                        const void *const *tw, const PhaseArgs &ph, const GradArgs &ga, int mode, hipStream_t st,
                        const GroupArgs<R> &grp, int ngroup, const hipEvent_t *ev)
{
    if (ns == 2) {
#define CALL(n)                                                                             \
    row_dispatch<R, n, 2>(variant, S, nrows, ny, V0, tw, ph, ga, mode, st, grp, ngroup, ev, \
                          std::make_index_sequence<kNumRowVariants>{})
        SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
    }
#define CALL(n)                                                                             \
    row_dispatch<R, n, 1>(variant, S, nrows, ny, V0, tw, ph, ga, mode, st, grp, ngroup, ev, \
                          std::make_index_sequence<kNumRowVariants>{})
    SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
}

template <typename R, int N, size_t... I> bool row_ok_n(int v, std::index_sequence<I...>)
{
    bool ok = false;
    ((v == (int)I ? (ok = row_variant_ok<R, N, (int)I>(), 0) : 0), ...);
    return ok;
}

template <typename R> bool xpass_variant_ok(int variant, int N)
{
    if (variant < 0 || variant >= kNumRowVariants) return false;
    switch (N) {
#define CASE(n) case n: return row_ok_n<R, n>(variant, std::make_index_sequence<kNumRowVariants>{});
    CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096)
#undef CASE
    default: return false;
    }
}

// Scratch bytes per lane of the kernel a row shape launches with ns states
// (the compiler's private segment: register spills), -1 if there is none.
template <typename R, int N, int NS, size_t... I> int row_scratch_n(int v, std::index_sequence<I...>)
{
    int bytes = -1;
    auto one = [&](auto vi) {
        constexpr int V = decltype(vi)::value;
        if constexpr (row_variant_ok<R, N, V>()) {
            constexpr RowVariant rv = kRowVariants[V];
            hipFuncAttributes a{};
            if (hipFuncGetAttributes(&a, (const void *)k_xpass<R, N, rv.rad, rv.threads, rv.wpe, NS, rv.pad, rv.late,
                                                                 rv.pre && sizeof(R) == 8>) == hipSuccess)
                bytes = (int)a.localSizeBytes;
        }
    };
    ((v == (int)I ? (one(std::integral_constant<int, (int)I>{}), 0) : 0), ...);
    return bytes;
}

template <typename R> int xpass_scratch(int variant, int N, int ns)
{
    if (variant < 0 || variant >= kNumRowVariants) return -1;
    switch (N) {
#define CASE(n)                                                                                   \
    case n:                                                                                       \
        return ns == 2 ? row_scratch_n<R, n, 2>(variant, std::make_index_sequence<kNumRowVariants>{}) \
                       : row_scratch_n<R, n, 1>(variant, std::make_index_sequence<kNumRowVariants>{});
    CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096)
#undef CASE
    default: return -1;
    }
}

template int xpass_scratch<float>(int, int, int);
template int xpass_scratch<double>(int, int, int);

template <typename R, int N, size_t... I> int row_groups_n(int v, int64_t nrows, std::index_sequence<I...>)
{
    int g = -1;
    auto one = [&](auto vi) {
        constexpr int V = decltype(vi)::value;
        if constexpr (row_variant_ok<R, N, V>()) {
            constexpr RowVariant rv = kRowVariants[V];
            using Tl = RowTile<N, rv.rad, rv.threads>;
            g = (int)(nrows % Tl::ROWS ? nrows : nrows / Tl::ROWS);
        }
    };
    ((v == (int)I ? (one(std::integral_constant<int, (int)I>{}), 0) : 0), ...);
    return g;
}

template <typename R> int xpass_groups(int variant, int N, int64_t nrows)
{
    if (variant < 0 || variant >= kNumRowVariants) return -1;
    switch (N) {
#define CASE(n) case n: return row_groups_n<R, n>(variant, nrows, std::make_index_sequence<kNumRowVariants>{});
    CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096)
#undef CASE
    default: return -1;
    }
}

template int xpass_groups<float>(int, int, int64_t);
template int xpass_groups<double>(int, int, int64_t);
template bool xpass_variant_ok<float>(int, int);
template bool xpass_variant_ok<double>(int, int);

template hipError_t launch_xpass<float>(int, int, int, const StatePtrs<float> &, int64_t, int, const void *,
                                        const void *const *, const PhaseArgs &, const GradArgs &, int, hipStream_t,
                                        const GroupArgs<float> &, int, const hipEvent_t *);
template hipError_t launch_xpass<double>(int, int, int, const StatePtrs<double> &, int64_t, int, const void *,
                                         const void *const *, const PhaseArgs &, const GradArgs &, int, hipStream_t,
                                         const GroupArgs<double> &, int, const hipEvent_t *);

}  // namespace sfo
