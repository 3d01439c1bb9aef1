// Transform-chain kernels, float64 (default tiles only).
#define WF_T double
#define WF_VARIANTS 0
#define WF_SIZES(X) X(8) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)
#define WF_LAUNCH_NAME chain_launch_f64
#define WF_PREP_NAME chain_prepare_f64
#include "wf_chain_inst.hpp"
