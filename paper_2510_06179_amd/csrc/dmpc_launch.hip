// Kernel lookup and launch for the host runtime.
#include <hip/hip_runtime.h>

#include "dmpc_internal.h"

namespace dmpc {

typedef void (*KernelFn)(KArgs);
struct KEntry {
  int nx, slots, maxbt, reg;
  KernelFn fwd, bwd;
};

#define DMPC_DECL(NX) const KEntry* kernel_entries_nx##NX(int* n);
DMPC_DECL(2)
DMPC_DECL(3)
DMPC_DECL(4)
DMPC_DECL(8)
DMPC_DECL(12)
DMPC_DECL(16)
DMPC_DECL(32)

static const KEntry* find_entry(int nx, int slots, int maxbt, int reg) {
  typedef const KEntry* (*Getter)(int*);
  static const Getter getters[] = {kernel_entries_nx2, kernel_entries_nx3, kernel_entries_nx4,
                                   kernel_entries_nx8, kernel_entries_nx12, kernel_entries_nx16,
                                   kernel_entries_nx32};
  for (Getter g : getters) {
    int n = 0;
    const KEntry* e = g(&n);
    for (int i = 0; i < n; ++i)
      if (e[i].nx == nx && e[i].slots == slots && e[i].maxbt == maxbt && e[i].reg == reg)
        return &e[i];
  }
  return nullptr;
}

bool kernel_available(int nx, int slots, int maxbt, int reg) {
  return find_entry(nx, slots, maxbt, reg) != nullptr;
}

static int launch(const LaunchCfg& c, const KArgs& a, void* stream, bool fwd) {
  const KEntry* e = find_entry(c.nx, c.slots, c.maxbt, c.reg);
  if (!e) return -1;
  KernelFn fn = fwd ? e->fwd : e->bwd;
  if (c.lds_bytes > 64 * 1024 &&
      hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)c.lds_bytes) != hipSuccess)
    return -2;
  hipLaunchKernelGGL(fn, dim3(c.grid), dim3(c.bt), c.lds_bytes, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

const void* kernel_function(const LaunchCfg& c, bool fwd) {
  const KEntry* e = find_entry(c.nx, c.slots, c.maxbt, c.reg);
  if (!e) return nullptr;
  KernelFn fn = fwd ? e->fwd : e->bwd;
  if (c.lds_bytes > 64 * 1024 &&
      hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)c.lds_bytes) != hipSuccess)
    return nullptr;
  return (const void*)fn;
}

int launch_forward(const LaunchCfg& c, const KArgs& a, void* stream) { return launch(c, a, stream, true); }
int launch_backward(const LaunchCfg& c, const KArgs& a, void* stream) { return launch(c, a, stream, false); }

}  // namespace dmpc
