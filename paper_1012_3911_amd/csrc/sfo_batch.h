// Internal interface of the batched runs (sfo_batch.hip, sfo_api.hip).
#pragma once
#include "sfo_impl.h"

namespace sfo {

// dL/dEbar of every problem of a reverse sweep from its boundary moments.
template <typename R>
hipError_t launch_batch_ebar_grad(const BatchProb<R> *probs, int nprob, int64_t nsteps, hipStream_t st);

}  // namespace sfo
