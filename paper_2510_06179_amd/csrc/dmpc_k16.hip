// Kernel instantiations for nx = 16 (see dmpc_device.h).
#include "dmpc_device.h"

namespace dmpc {

#define DMPC_K(NX, SL, MB, RG) \
  {NX, SL, MB, RG, forward_kernel<NX, SL, MB, RG>, backward_kernel<NX, SL, MB, RG>}

// (values per thread, launch bound, mode: 0 rows read from the workspace,
// 1 rows in registers, 2 rows in registers in the wave-block layout, 3 Schur
// rows in registers and the inverted diagonal blocks in LDS, 4 as 3 with the
// last slot's rows in LDS, 5 the Cholesky-scaled system: rows of its two
// off-diagonal blocks in registers)
static const KEntry kEntries[] = {
    DMPC_K(16, 1, 64, 1), DMPC_K(16, 2, 64, 1), DMPC_K(16, 1, 128, 1), DMPC_K(16, 2, 128, 1),
    DMPC_K(16, 1, 256, 1), DMPC_K(16, 2, 256, 1), DMPC_K(16, 1, 512, 1), DMPC_K(16, 2, 512, 1),
    DMPC_K(16, 1, 1024, 1),
    DMPC_K(16, 4, 256, 0), DMPC_K(16, 8, 256, 0), DMPC_K(16, 8, 512, 0), DMPC_K(16, 4, 1024, 0),
    DMPC_K(16, 2, 640, 3), DMPC_K(16, 2, 1024, 3), DMPC_K(16, 5, 512, 4), DMPC_K(16, 3, 512, 4), DMPC_K(16, 2, 512, 4),
    DMPC_K(16, 5, 512, 5), DMPC_K(16, 3, 512, 5), DMPC_K(16, 2, 512, 5), DMPC_K(16, 2, 320, 5),
    DMPC_K(16, 1, 320, 5), DMPC_K(16, 5, 256, 5), DMPC_K(16, 3, 192, 5), DMPC_K(16, 9, 256, 5),
    DMPC_K(16, 2, 192, 5), DMPC_K(16, 3, 384, 5),
};

const KEntry* kernel_entries_nx16(int* n) {
  *n = (int)(sizeof(kEntries) / sizeof(kEntries[0]));
  return kEntries;
}

}  // namespace dmpc
