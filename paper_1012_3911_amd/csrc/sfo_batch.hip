// Batched runs: many independent Schroedinger problems of uneven sizes.
//
// Problems are grouped by grid shape.  One launch of a line pass covers every
// problem of a group, the problem index being a grid dimension (see
// GroupArgs), so that a 400-step run of a batch costs a few launches per step
// in all, not a few per problem; the whole sequence is captured in a HIP
// graph by the host (sfo_api.hip).  This file holds the small kernel that
// only batches need.
#include <algorithm>

#include "sfo_batch.h"

namespace sfo {

// dL/dEbar[s][a] = (M[s+1][a] + M[s][a]) / (2 hbar), M summed over each
// problem's partial slots in slot order; one grid row per problem.
template <typename R> __global__ void k_batch_ebar_grad(const BatchProb<R> *__restrict__ probs, int64_t nsteps)
{
    const BatchProb<R> &P = probs[blockIdx.y];
    if (!P.dE) return;
    const int nd = P.ndim, ns = P.gslots;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nsteps * nd;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / nd;
        const int a = (int)(i % nd);
        double m1 = 0.0, m0 = 0.0;
        for (int k = 0; k < ns; ++k) {
            m1 += P.part[((s + 1) * ns + k) * 3 + a];
            m0 += P.part[(s * ns + k) * 3 + a];
        }
        P.dE[i] = (m1 + m0) * P.inv_2hbar;
    }
}

template <typename R>
hipError_t launch_batch_ebar_grad(const BatchProb<R> *probs, int nprob, int64_t nsteps, hipStream_t st)
{
    if (nprob == 0 || nsteps == 0) return hipSuccess;
    const unsigned bx = (unsigned)std::min<int64_t>(64, (nsteps * 3 + 255) / 256);
    hipLaunchKernelGGL(k_batch_ebar_grad<R>, dim3(bx, (unsigned)nprob), dim3(256), 0, st, probs, nsteps);
    return hipGetLastError();
}

template hipError_t launch_batch_ebar_grad<float>(const BatchProb<float> *, int, int64_t, hipStream_t);
template hipError_t launch_batch_ebar_grad<double>(const BatchProb<double> *, int, int64_t, hipStream_t);

}  // namespace sfo
