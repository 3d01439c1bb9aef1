// Transform-chain kernels, float32, grid sides 128..1024, with tile variants.
#define WF_T float
#define WF_VARIANTS 1
#define WF_SIZES(X) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)
#define WF_LAUNCH_NAME chain_launch_f32_l
#define WF_PREP_NAME chain_prepare_f32_l
#include "wf_chain_inst.hpp"
