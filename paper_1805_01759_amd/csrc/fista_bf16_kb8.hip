// Instantiations of the persistent iteration kernel: bf16, 8 row blocks per wave.
#include "fista_impl.h"

namespace l1ls {
template hipError_t launch_one<1, 8, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<1, 8, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<2, 8, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<2, 8, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<3, 8, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<3, 8, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<4, 8, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<4, 8, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<5, 8, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<5, 8, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<6, 8, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<6, 8, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<7, 8, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<7, 8, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<8, 8, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<8, 8, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
}  // namespace l1ls
