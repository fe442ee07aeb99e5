// MFMA direct DST-7/DCT-8 kernels (filled in below).
#include "kernels.hpp"

namespace ta {
const KernelEntry* mfma_kernels(int* count) {
  *count = 0;
  return nullptr;
}
}  // namespace ta
