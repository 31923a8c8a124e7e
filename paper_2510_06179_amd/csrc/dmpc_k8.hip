// Kernel instantiations for nx = 8 (see dmpc_device.h).
#include "dmpc_device.h"

namespace dmpc {

#define DMPC_K(NX, SL, MB, RG) \
  {NX, SL, MB, RG, forward_kernel<NX, SL, MB, RG>, backward_kernel<NX, SL, MB, RG>}

// (values per thread, launch bound, mode: 0 rows read from the workspace,
// 1 rows in registers, 2 rows in registers in the wave-block layout)
static const KEntry kEntries[] = {
    DMPC_K(8, 1, 64, 1), DMPC_K(8, 2, 64, 1), DMPC_K(8, 4, 64, 1),
    DMPC_K(8, 1, 128, 1), DMPC_K(8, 2, 128, 1), DMPC_K(8, 4, 128, 1),
    DMPC_K(8, 1, 256, 1), DMPC_K(8, 2, 256, 1), DMPC_K(8, 4, 256, 1), DMPC_K(8, 1, 512, 1), DMPC_K(8, 2, 512, 1),
    DMPC_K(8, 1, 1024, 1), DMPC_K(8, 3, 512, 1), DMPC_K(8, 2, 1024, 1),
    DMPC_K(8, 4, 256, 0), DMPC_K(8, 8, 256, 0), DMPC_K(8, 8, 512, 0),
    DMPC_K(8, 8, 64, 2),
    DMPC_K(8, 3, 384, 5), DMPC_K(8, 2, 320, 5), DMPC_K(8, 2, 128, 5), DMPC_K(8, 3, 192, 5),
    DMPC_K(8, 5, 256, 5), DMPC_K(8, 3, 128, 5),
};

const KEntry* kernel_entries_nx8(int* n) {
  *n = (int)(sizeof(kEntries) / sizeof(kEntries[0]));
  return kEntries;
}

}  // namespace dmpc
