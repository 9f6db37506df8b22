// placeholder, replaced below
#include "afd_internal.h"
namespace afd {
int launch_apply_mfma(const MatvecArgs&, const double*, int, const double*, double*, hipStream_t) {
    set_error("apply_K_mfma: not available");
    return AFD_E_INVALID_ARG;
}
}  // namespace afd
