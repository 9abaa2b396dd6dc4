// Two-level agg_i (per-case top lists, then the top of their collection).
#pragma once

#include "dcflow_internal.h"

namespace dcflow {

// cases of a plan: the N-0 case, the contingency columns (branches, generators),
// the multi-outage cases
int per_case_slots(const dcflow_plan *p);

hipError_t launch_worst_per_case(dcflow_batch *bt, const void *flows, int nvar, int prec,
                                 const dcflow_score *scores, int per_case, int top_k, void *ws,
                                 dcflow_case *out, hipStream_t s);

}  // namespace dcflow
