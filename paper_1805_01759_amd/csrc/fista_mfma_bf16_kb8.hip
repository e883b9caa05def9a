// Instantiations of the split-BF16 iteration kernel with 8 blocks of 16 unknowns
// per wave (256 < L <= 512), its bf16 planes of A read from L2.
#include "fista_mfma.h"

namespace l1ls {
template hipError_t launch_mfma_one<1, 8, false, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<2, 8, false, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<3, 8, false, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<4, 8, false, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
}  // namespace l1ls
