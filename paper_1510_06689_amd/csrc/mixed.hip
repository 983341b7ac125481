// Mixed-precision (split-bf16) Gram and bf16 TTM kernels.
#include "tk_common.hpp"

namespace tk {

GramPlan plan_gram_mixed(const ModeView& v) {
    (void)v;
    GramPlan pl{};
    return pl;
}

int launch_gram_mixed(const float* y, const ModeView& v, const GramPlan& pl, double* partial,
                      hipStream_t st) {
    (void)y; (void)v; (void)pl; (void)partial; (void)st;
    return fail(TK_ERR_UNSUPPORTED, "split-bf16 Gram not built");
}

int launch_ttm_mixed(const float* y, const ModeView& v, const double* m, int64_t K, int64_t ldm,
                     int transpose, int precision, float* z, hipStream_t st) {
    (void)y; (void)v; (void)m; (void)K; (void)ldm; (void)transpose; (void)precision; (void)z;
    (void)st;
    return fail(TK_ERR_UNSUPPORTED, "bf16 TTM not built");
}

}  // namespace tk
