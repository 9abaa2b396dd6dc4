// Two-level agg_i (per-case top lists, then the top of their collection).
#pragma once

#include "dcflow_internal.h"

namespace dcflow {

// cases of a plan: the N-0 case, the contingency columns (branches, generators),
// the multi-outage cases
int per_case_slots(const dcflow_plan *p);
// device bytes of the two-level pass: the per-case lists, then (when one row band
// covers the monitored rows) the winners' case maxima used to prune the cases
size_t per_case_workspace(const dcflow_batch *bt, int per_case);

hipError_t launch_worst_per_case(dcflow_batch *bt, const void *flows, int nvar, int prec,
                                 const dcflow_score *scores, int per_case, int top_k, void *ws,
                                 dcflow_case *out, hipStream_t s);

}  // namespace dcflow
