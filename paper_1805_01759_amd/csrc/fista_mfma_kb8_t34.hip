// Instantiations of the FP32 iteration kernel: 8 blocks of 16 unknowns per wave, 48 and 64 rows
// (a unit of its own so that the two halves compile in parallel).
#include "fista_mfma.h"

namespace l1ls {
template hipError_t launch_mfma_one<3, 8, true, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<3, 8, false, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<4, 8, true, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<4, 8, false, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
}  // namespace l1ls
