// Internal interface of the batched runs (sfo_batch.hip, sfo_api.hip).
#pragma once
#include "sfo_impl.h"

namespace sfo {

// Zeroes the per-problem reduction counters of a reverse sweep (a fill
// kernel rather than a memset, so that it can sit in a captured graph).
hipError_t launch_batch_reset(unsigned *count, int n, hipStream_t st);

// dL/dEbar of every problem of a reverse sweep from its boundary moments.
template <typename R>
hipError_t launch_batch_ebar_grad(const BatchProb<R> *probs, int nprob, int64_t nsteps, hipStream_t st);

}  // namespace sfo
