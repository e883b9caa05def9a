// Instantiations of the FP32 iteration kernel: 4 blocks of 16 unknowns per wave.
#include "fista_mfma.h"

namespace l1ls {
template hipError_t launch_mfma_one<1, 4, true, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<1, 4, false, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<2, 4, true, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<2, 4, false, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<3, 4, true, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<3, 4, false, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<4, 4, true, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<4, 4, false, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
}  // namespace l1ls
