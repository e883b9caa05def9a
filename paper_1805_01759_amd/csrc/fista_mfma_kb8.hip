// Instantiations of the FP32 iteration kernel: 8 blocks of 16 unknowns per wave, 16 and 32 rows.
#include "fista_mfma.h"

namespace l1ls {
template hipError_t launch_mfma_one<1, 8, true, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<1, 8, false, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<2, 8, true, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<2, 8, false, L1LS_FP32, 4>(const StackTable &, int, hipStream_t);
}  // namespace l1ls
