// Split-BF16 instantiations of the streamed MFMA tile.
#include "fista_stream.h"

namespace l1ls {
template hipError_t launch_stream_t<1, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
template hipError_t launch_stream_t<2, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
template hipError_t launch_stream_t<3, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
template hipError_t launch_stream_t<4, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
template hipError_t launch_stream_t<5, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
template hipError_t launch_stream_t<6, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
template hipError_t launch_stream_t<7, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
template hipError_t launch_stream_t<8, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
}  // namespace l1ls
