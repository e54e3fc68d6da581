// FP32 instantiations of the fused two-stage sweeps.
#include "pf_fused_launch.h"

PF_FUSED_INST(float, 64, 8, 32, false)
PF_FUSED_INST(float, 64, 8, 64, false)
PF_FUSED_INST(float, 64, 8, 0, false)
PF_FUSED_INST(float, 64, 16, 32, false)
PF_FUSED_INST(float, 64, 16, 64, false)
PF_FUSED_INST(float, 128, 8, 32, false)
PF_FUSED_INST(float, 32, 16, 32, false)
PF_FUSED_INST(float, 32, 16, 64, false)
PF_FUSED_INST(float, 32, 16, 0, false)
PF_FUSED_INST(float, 64, 8, 32, true)
