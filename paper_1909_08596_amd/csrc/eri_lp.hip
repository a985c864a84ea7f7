// Reduced-precision forms of the embedding-ERI transformation (placeholder
// until the FP32-3M and split-BF16x3 kernels land).
#include "common.h"
#include "eri.h"

namespace dmet {

size_t eri_lp_workspace(const EriPlan& p) { return 256; }

dmet_status eri_lp(const EriPlan& p, const void*, const double*, double*, double*, double*, void*, size_t,
                   hipStream_t) {
    return fail(DMET_E_UNSUPPORTED, "reduced-precision forms are not built yet");
}

}  // namespace dmet
