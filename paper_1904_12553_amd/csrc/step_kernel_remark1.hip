// step_kernel_remark1.hip -- the step kernel instantiated for the force
// distribution of Remark 1 (Sec. 3.1) with the central stencils of eq:N31a
// (see step_kernel.hip), compiled as its own translation unit.
#define NPL_GS 2
#include "step_kernel.hip"
