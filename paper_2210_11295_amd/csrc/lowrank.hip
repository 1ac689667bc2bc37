// Randomized SVD (Algorithm 1) and Nystrom (Algorithm 2) drivers.
// Placeholder entry points: report BSRHT_EUNSUPPORTED until the FP64 dense
// kernels are in place.
#include "common.h"

extern "C" {

size_t rsvd_workspace(bsrht_plan_t, int64_t, int64_t) { return 0; }

int rsvd(bsrht_plan_t, const float *, int64_t, int64_t, int64_t, float *, double *, float *,
         int32_t *, void *, size_t, void *) {
  return BSRHT_EUNSUPPORTED;
}

size_t nystrom_workspace(bsrht_plan_t, int64_t) { return 0; }

int nystrom(bsrht_plan_t, const float *, int64_t, int64_t, float *, double *, int32_t *, void *,
            size_t, void *) {
  return BSRHT_EUNSUPPORTED;
}

}  // extern "C"
