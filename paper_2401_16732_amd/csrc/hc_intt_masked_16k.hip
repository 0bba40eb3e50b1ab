// Masked inverse NTT instances for N = 16384.
#define HC_INTT_MASKED_IMPL
#include "hc_intt_masked.h"

namespace hc {
template hipError_t intt_masked_logn<14>(const ConvGeom &, uint32_t, uint32_t, uint32_t, const uint32_t *,
                                            const uint32_t *, uint32_t *, uint32_t *, uint32_t,
                                            const LimbConsts &, const Twiddles &, const OutPtrs &, hipStream_t, bool);
}  // namespace hc
