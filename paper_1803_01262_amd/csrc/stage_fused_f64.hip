// FP64 instantiations of the fused two-stage sweeps.
#include "pf_fused_launch.h"

PF_FUSED_INST(double, 32, 16, 32, false)
PF_FUSED_INST(double, 32, 16, 64, false)
PF_FUSED_INST(double, 32, 16, 0, false)
PF_FUSED_INST(double, 64, 8, 32, false)
PF_FUSED_INST(double, 64, 8, 64, false)
PF_FUSED_INST(double, 64, 8, 0, false)
PF_FUSED_INST(double, 64, 8, 32, true)
