// dd_tune.hpp -- the process-wide tuning table: schedules measured by the
// tuner (dd_tune.cpp) for plain plans, keyed by (N, alpha, input dtype,
// batch size class), and for the batch kernel, keyed by (N, alpha).
#pragma once

#include <cstdint>

#include "../../include/dense_dft.h"

namespace dd {

struct Sched;

// Batch size class of a plain plan: floor(log2(batch)), at most 12.
int tune_batch_class(int64_t batch);

bool tune_lookup_plan(int64_t N, int alpha, int dtype, int64_t batch, dd_sched* out);
void tune_store_plan(int64_t N, int alpha, int dtype, int64_t batch, const dd_sched& s, float ms);
bool tune_lookup_batch(int64_t N, int alpha, dd_sched* out);
void tune_store_batch(int64_t N, int alpha, const dd_sched& s, float ms);

// Batch plan whose kernel signals all take the schedule `force` (the tuner's
// candidates); NULL: as dense_dft_batch_plan.
dd_status batch_plan_forced(dd_batch_t* out, const dd_desc* descs, int32_t count, uint32_t flags,
                            const Sched* force);

}  // namespace dd
