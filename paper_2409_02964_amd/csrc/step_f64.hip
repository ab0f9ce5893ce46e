// step_f64.hip -- step-kernel instances for double storage, double arithmetic.
#define VANSE_S double
#define VANSE_T double
#define VANSE_SHIFT false
#include "step_inst.hpp"
