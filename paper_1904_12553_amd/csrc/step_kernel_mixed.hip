// step_kernel_mixed.hip -- the step kernel instantiated for the isotropic
// mixed gradient scheme of eq:N40 (see step_kernel.hip), compiled as its own
// translation unit.
#define NPL_GS 1
#include "step_kernel.hip"
