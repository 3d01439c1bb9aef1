// Transform-chain kernels, float64 instantiations.
#define WF_T double
#define WF_LAUNCH_NAME chain_launch_f64
#define WF_PREP_NAME chain_prepare_f64
#include "wf_chain_inst.hpp"
