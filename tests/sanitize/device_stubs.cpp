// Stand-ins for the GPU half of the library, so that the host half
// (automaton.cpp, api.cpp) can be built with the host compiler's sanitizers
// and driven without a GPU.  Dictionaries in the sanitizer build are host-only: they
// never reach upload_dict, and release_dict has nothing to free.
#include "../../paper_1403_7294_amd/csrc/internal.h"

namespace acx {
int upload_dict(ac_dict *) { return AC_E_NO_DEVICE; }
void release_dict(ac_dict *) {}
int device_limits(uint32_t *, uint32_t *) { return AC_E_HIP; }
}  // namespace acx
