// step_f32s.hip -- step-kernel instances for float storage, float arithmetic, shifted storage.
#define VANSE_S float
#define VANSE_T float
#define VANSE_SHIFT true
#define VANSE_FUSED2_NT 256
#define VANSE_FUSED2_BATCH_MAX 256
#include "step_inst.hpp"
