// Instantiations of the split-BF16 iteration kernel with 4 blocks of 16 unknowns
// per wave (bf16 planes of A in LDS, or from L2 above 32 rows), and the host-side
// plane size.
#include "fista_mfma.h"

namespace l1ls {
size_t fm_bf_planes_bytes_host(int rows, int l_pad) { return fm_bf_planes_bytes(rows, l_pad); }
template hipError_t launch_mfma_one<1, 4, true, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<2, 4, true, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<3, 4, true, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<4, 4, true, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<1, 4, false, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<2, 4, false, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<3, 4, false, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<4, 4, false, L1LS_SPLIT_BF16, 4>(const StackTable &, int, hipStream_t);
}  // namespace l1ls
