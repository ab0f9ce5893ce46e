// step_f16s.hip -- step-kernel instances for _Float16 storage, float arithmetic, shifted storage.
#define VANSE_S _Float16
#define VANSE_T float
#define VANSE_SHIFT true
#include "step_inst.hpp"
