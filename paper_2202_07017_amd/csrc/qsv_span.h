// Span passes for expectation values: launch of the kernels
// (kernels_span.hip); descriptors and planner in qsv_span_plan.h.
#pragma once

#include "qsv_internal.h"
#include "qsv_span_plan.h"

namespace qsv {

// Adds the pass's part of <psi|H|psi> to partials[b] (b < nslots, one slot
// per block; the imaginary slots partials[nslots + b] get 0: every Hermitian
// pair is summed once, so the imaginary part vanishes identically), or writes
// it when accumulate is 0 (then slots beyond the grid are zeroed too).
hipError_t launch_span_pass(const SpanPassK& a, const void* psi, int dt, double* partials, int nslots,
                            int accumulate, hipStream_t s);

}  // namespace qsv
