// amy_tune.hpp -- autotuner cache (internal).
#pragma once
#include "amy_host.hpp"

BatchTune amy_tune_lookup_batch(const amy_problem* probs, int32_t count, const BatchPlan& bp);
// AMY_VARIANT_AUTO when the shape class has not been tuned.
int amy_tune_lookup_variant(const Plan& pl, const amy_problem* p);
