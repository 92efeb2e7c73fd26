// jk_tune.hpp -- the recorded-plan table shared by the build orchestration
// (jk_api.hip) and the table code (jk_tune.hip).
#pragma once
#include "../../include/jk_tune.h"

namespace jk {
// The recorded plan for p's shape class, or the default {0, 1024}.
jk_tuning tuning_for(const jk_problem *p);
void tuning_record(const jk_problem *p, const jk_tuning &t);
} // namespace jk
