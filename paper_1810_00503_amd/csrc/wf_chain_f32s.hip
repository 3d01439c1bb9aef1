// Transform-chain kernels, float32, grid sides 8..96, with tile variants.
#define WF_T float
#define WF_VARIANTS 1
#define WF_SIZES(X) X(8) X(16) X(24) X(32) X(48) X(64) X(96)
#define WF_LAUNCH_NAME chain_launch_f32_s
#define WF_PREP_NAME chain_prepare_f32_s
#include "wf_chain_inst.hpp"
