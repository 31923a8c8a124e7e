// Kernel instantiations for nx = 32 (see dmpc_device.h).  Rows of S^ and
// Phi^-1 are read from the workspace (3 x 32 coefficients per row do not fit
// in registers next to the PCG vectors); the iterate, QP solution and
// line-search region of long horizons live in the workspace too.
#include "dmpc_device.h"

namespace dmpc {

#define DMPC_K(NX, SL, MB, RG) \
  {NX, SL, MB, RG, forward_kernel<NX, SL, MB, RG>, backward_kernel<NX, SL, MB, RG>}

// (values per thread, launch bound, mode: 0 rows read from the workspace,
// 1 rows in registers, 2 rows in registers in the wave-block layout)
static const KEntry kEntries[] = {
    DMPC_K(32, 2, 1024, 0), DMPC_K(32, 4, 1024, 0), DMPC_K(32, 8, 1024, 0),
    DMPC_K(32, 12, 1024, 0),
};

const KEntry* kernel_entries_nx32(int* n) {
  *n = (int)(sizeof(kEntries) / sizeof(kEntries[0]));
  return kEntries;
}

}  // namespace dmpc
