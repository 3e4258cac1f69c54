// Reduced-precision dot-product filter (work in progress).
#include "query_kernels.h"
extern "C" int isax_filter_scores(isax_index*, const float*, int64_t, int32_t, float*, float*) {
    isax::set_error(ISAX_EINVAL, "reduced-precision filter not available in this build");
    return ISAX_EINVAL;
}
