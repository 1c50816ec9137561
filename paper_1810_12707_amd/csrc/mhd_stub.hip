// Empty registration for a grid size left out of a partial build.
#include "mhd_registry.h"

namespace mhd {
#define MHD_CAT2(a, b) a##b
#define MHD_CAT(a, b) MHD_CAT2(a, b)
#if MHD_SCHED == 1
void MHD_CAT(register_s1_, MHD_N)(Registry&) {}
#else
void MHD_CAT(register_, MHD_N)(Registry&) {}
#endif
}  // namespace mhd
