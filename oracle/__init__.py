"""Plain FP64 CPU oracle for the Wiener-filter-as-MAP method (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The library's product path never imports, links or executes it, and
it shares no code with the HIP kernels: it is written directly from the paper's
equations (sections 2.2-2.4, appendices A and C) with numpy, one library FFT per
transform and no blocking, fusion or reordering beyond what the equations state.

Parity status of each function is listed in the module docstrings.
"""
from .wf_oracle import *  # noqa: F401,F403
from .philox import philox4x32_10, normals_for_sim  # noqa: F401
