// step_f32.hip -- step-kernel instances for float storage, float arithmetic.
#define VANSE_S float
#define VANSE_T float
#define VANSE_SHIFT false
#include "step_inst.hpp"
