// Empty registration for a grid size left out of a partial build.
#include "mhd_registry.h"

namespace mhd {
#define MHD_CAT2(a, b) a##b
#define MHD_CAT(a, b) MHD_CAT2(a, b)
void MHD_CAT(register_, MHD_N)(Registry&) {}
}  // namespace mhd
