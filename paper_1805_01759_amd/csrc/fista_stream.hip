// FP32 instantiations of the streamed MFMA tile, its LDS size and the launch
// dispatch over row blocks and precision.
#include "fista_stream.h"

namespace l1ls {

size_t fista_stream_lds_bytes(int T) { return fista_stream_lds_bytes_t(T); }

// split-BF16 instantiations (fista_stream_bf16.hip)
extern template hipError_t launch_stream_t<1, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
extern template hipError_t launch_stream_t<2, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
extern template hipError_t launch_stream_t<3, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
extern template hipError_t launch_stream_t<4, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
extern template hipError_t launch_stream_t<5, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
extern template hipError_t launch_stream_t<6, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
extern template hipError_t launch_stream_t<7, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);
extern template hipError_t launch_stream_t<8, L1LS_SPLIT_BF16>(const StackTable &, hipStream_t);

template <int PREC>
static hipError_t launch_stream_p(const StackTable &t, int T, hipStream_t s)
{
    switch (T) {
    case 1: return launch_stream_t<1, PREC>(t, s);
    case 2: return launch_stream_t<2, PREC>(t, s);
    case 3: return launch_stream_t<3, PREC>(t, s);
    case 4: return launch_stream_t<4, PREC>(t, s);
    case 5: return launch_stream_t<5, PREC>(t, s);
    case 6: return launch_stream_t<6, PREC>(t, s);
    case 7: return launch_stream_t<7, PREC>(t, s);
    case 8: return launch_stream_t<8, PREC>(t, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stream_table(const StackTable &t, int T, int precision, hipStream_t s)
{
    return precision == L1LS_SPLIT_BF16 ? launch_stream_p<L1LS_SPLIT_BF16>(t, T, s)
                                        : launch_stream_p<L1LS_FP32>(t, T, s);
}

}  // namespace l1ls
