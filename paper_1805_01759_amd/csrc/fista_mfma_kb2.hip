// Instantiations of the FP32 MFMA iteration kernel with 32 unknowns per wave and
// up to eight waves (two per SIMD), for L <= 256 and N <= 32.
#include "fista_mfma.h"

namespace l1ls {
template hipError_t launch_mfma_one<1, 2, true, L1LS_FP32, 8>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<1, 2, false, L1LS_FP32, 8>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<2, 2, true, L1LS_FP32, 8>(const StackTable &, int, hipStream_t);
template hipError_t launch_mfma_one<2, 2, false, L1LS_FP32, 8>(const StackTable &, int, hipStream_t);
}  // namespace l1ls
