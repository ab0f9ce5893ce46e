// step_f32.hip -- step-kernel instances for float storage, float arithmetic.
#define VANSE_S float
#define VANSE_T float
#define VANSE_SHIFT false
#define VANSE_FUSED2_NT 256
#define VANSE_FUSED2_BATCH_MAX 256
#include "step_inst.hpp"
