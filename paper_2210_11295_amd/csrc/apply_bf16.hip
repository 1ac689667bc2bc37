// Split-BF16 matrix-core form of the block SRHT apply (placeholder until the
// MFMA kernel lands): reports BSRHT_EUNSUPPORTED.
#include "common.h"

namespace bsrht {

size_t apply_split_bf16_ws_bytes(const bsrht_plan_s *, int64_t) { return 0; }

int apply_split_bf16(const bsrht_plan_s *, const float *, int64_t, int64_t, float *,
                     int64_t, void *, size_t, hipStream_t) {
  return BSRHT_EUNSUPPORTED;
}

}  // namespace bsrht
