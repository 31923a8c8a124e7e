// Kernel instantiations for nx = 12 (see dmpc_device.h).
#include "dmpc_device.h"

namespace dmpc {

#define DMPC_K(NX, SL, MB, RG) \
  {NX, SL, MB, RG, forward_kernel<NX, SL, MB, RG>, backward_kernel<NX, SL, MB, RG>}

// (values per thread, launch bound, mode: 0 rows read from the workspace,
// 1 rows in registers, 2 rows in registers in the wave-block layout, 3 Schur
// rows in registers and the inverted diagonal blocks in LDS, 4 as 3 with the
// last slot's rows in LDS, 5 the Cholesky-scaled system: rows of its two
// off-diagonal blocks in registers; launched with whole stages per group of
// block_threads rows)
static const KEntry kEntries[] = {
    DMPC_K(12, 1, 64, 1), DMPC_K(12, 2, 64, 1), DMPC_K(12, 1, 128, 1), DMPC_K(12, 2, 128, 1),
    DMPC_K(12, 1, 256, 1), DMPC_K(12, 2, 256, 1), DMPC_K(12, 1, 512, 1), DMPC_K(12, 2, 512, 1),
    DMPC_K(12, 1, 1024, 1),
    DMPC_K(12, 4, 256, 0), DMPC_K(12, 8, 256, 0), DMPC_K(12, 8, 512, 0),
    DMPC_K(12, 2, 1024, 3), DMPC_K(12, 4, 512, 4),
    DMPC_K(12, 5, 384, 5), DMPC_K(12, 3, 576, 5), DMPC_K(12, 5, 192, 5), DMPC_K(12, 3, 384, 5),
    DMPC_K(12, 3, 192, 5), DMPC_K(12, 2, 192, 5),
};

const KEntry* kernel_entries_nx12(int* n) {
  *n = (int)(sizeof(kEntries) / sizeof(kEntries[0]));
  return kEntries;
}

}  // namespace dmpc
