// Instantiations of the persistent iteration kernel: bf16, 16 row blocks per wave.
#include "fista_impl.h"

namespace l1ls {
template hipError_t launch_one<1, 16, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<1, 16, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<2, 16, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<2, 16, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<3, 16, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<3, 16, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<4, 16, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<4, 16, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<5, 16, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<5, 16, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<6, 16, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<6, 16, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<7, 16, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<7, 16, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<8, 16, true, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
template hipError_t launch_one<8, 16, false, L1LS_SPLIT_BF16>(const FistaArgs &, int, hipStream_t);
}  // namespace l1ls
