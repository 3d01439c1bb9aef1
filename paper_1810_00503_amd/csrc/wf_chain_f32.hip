// Transform-chain kernels, float32 instantiations.
#define WF_T float
#define WF_LAUNCH_NAME chain_launch_f32
#define WF_PREP_NAME chain_prepare_f32
#include "wf_chain_inst.hpp"
