// step_f32s.hip -- step-kernel instances for float storage, float arithmetic, shifted storage.
#define VANSE_S float
#define VANSE_T float
#define VANSE_SHIFT true
#include "step_inst.hpp"
