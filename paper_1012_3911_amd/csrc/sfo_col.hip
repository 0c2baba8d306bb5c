// Instantiations of the strided column passes for complex64 and complex128.
#include "pass_kernels.h"

namespace sfo {

template <typename R>
hipError_t launch_colpass(int variant, int N, int ns, const StatePtrs<R> &S, int64_t ncols, int64_t stride, int nslab,
                          int64_t slab_stride, const void *const *tw, const KinArgs &kin, int mode, hipStream_t st,
                          const GroupArgs<R> &grp, int ngroup, const hipEvent_t *ev)
{
    if (ns == 2) {
#define CALL(n)                                                                                       \
    col_dispatch<R, n, 2>(variant, S, ncols, stride, nslab, slab_stride, tw, kin, mode, st, grp, ngroup, ev, \
                          std::make_index_sequence<kNumColVariants>{})
        SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
    }
#define CALL(n)                                                                                       \
    col_dispatch<R, n, 1>(variant, S, ncols, stride, nslab, slab_stride, tw, kin, mode, st, grp, ngroup, ev, \
                          std::make_index_sequence<kNumColVariants>{})
    SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
}

template <typename R, int N, size_t... I> bool col_ok_n(int v, std::index_sequence<I...>)
{
    bool ok = false;
    ((v == (int)I ? (ok = col_variant_ok<R, N, (int)I>(), 0) : 0), ...);
    return ok;
}

template <typename R> bool colpass_variant_ok(int variant, int N, int64_t ncols, int ns)
{
    if (variant < 0 || variant >= kNumColVariants) return false;
    if (ncols % kColVariants[variant].cols) return false;
    (void)ns;
    switch (N) {
#define CASE(n) case n: return col_ok_n<R, n>(variant, std::make_index_sequence<kNumColVariants>{});
    CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096)
#undef CASE
    default: return false;
    }
}

// Scratch bytes per lane of the kernel a column shape launches for a step's
// k-space pass (ns = 1: the pipelined kernel where the shape has one, else
// the plain one) or the reverse sweep's (ns = 2), -1 if there is none.
template <typename R, int N, int NS, size_t... I> int col_scratch_n(int v, std::index_sequence<I...>)
{
    int bytes = -1;
    auto one = [&](auto vi) {
        constexpr int V = decltype(vi)::value;
        if constexpr (col_variant_ok<R, N, V>()) {
            constexpr ColVariant cv = kColVariants[V];
            const void *k = nullptr;
            if constexpr (cv.pipe > 0 && NS == 1)
                k = (const void *)k_colpipe<R, N, cv.rad, cv.cols, cv.wpe, cv.order>;
            else if constexpr (cv.pre)
                k = (const void *)k_colpass<R, N, cv.rad, cv.cols, cv.wpe, NS, false, false, true>;
            else
                k = (const void *)k_colpass<R, N, cv.rad, cv.cols, cv.wpe, NS>;
            hipFuncAttributes a{};
            if (hipFuncGetAttributes(&a, k) == hipSuccess) bytes = (int)a.localSizeBytes;
        }
    };
    ((v == (int)I ? (one(std::integral_constant<int, (int)I>{}), 0) : 0), ...);
    return bytes;
}

template <typename R> int colpass_scratch(int variant, int N, int ns)
{
    if (variant < 0 || variant >= kNumColVariants) return -1;
    switch (N) {
#define CASE(n)                                                                                   \
    case n:                                                                                       \
        return ns == 2 ? col_scratch_n<R, n, 2>(variant, std::make_index_sequence<kNumColVariants>{}) \
                       : col_scratch_n<R, n, 1>(variant, std::make_index_sequence<kNumColVariants>{});
    CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096)
#undef CASE
    default: return -1;
    }
}

template int colpass_scratch<float>(int, int, int);
template int colpass_scratch<double>(int, int, int);

template bool colpass_variant_ok<float>(int, int, int64_t, int);
template bool colpass_variant_ok<double>(int, int, int64_t, int);

template hipError_t launch_colpass<float>(int, int, int, const StatePtrs<float> &, int64_t, int64_t, int, int64_t,
                                          const void *const *, const KinArgs &, int, hipStream_t,
                                          const GroupArgs<float> &, int, const hipEvent_t *);
template hipError_t launch_colpass<double>(int, int, int, const StatePtrs<double> &, int64_t, int64_t, int, int64_t,
                                           const void *const *, const KinArgs &, int, hipStream_t,
                                           const GroupArgs<double> &, int, const hipEvent_t *);

}  // namespace sfo
