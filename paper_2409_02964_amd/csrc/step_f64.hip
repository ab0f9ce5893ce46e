// step_f64.hip -- step-kernel instances for double storage, double arithmetic.
#define VANSE_S double
#define VANSE_T double
#define VANSE_SHIFT false
#define VANSE_FUSED2_NT 128
#define VANSE_FUSED2_BATCH_MAX 128
#include "step_inst.hpp"
