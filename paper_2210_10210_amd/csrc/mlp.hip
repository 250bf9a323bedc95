// Preconditioner network kernels (placeholder until the MFMA kernels land).
#include "efgp_internal.h"

namespace efgp {

void mlp_forward(const float*, int64_t, const float*, float*, hipStream_t) {
    throw StatusError{EFGP_EMODEL, "network kernels not built"};
}
void mlp_loss_grad(const float*, int64_t, const float*, const float*, const float*, float*, double*, hipStream_t) {
    throw StatusError{EFGP_EMODEL, "network kernels not built"};
}
void mlp_adam(float*, const float*, float*, float*, int64_t, float, float, float, float, hipStream_t) {
    throw StatusError{EFGP_EMODEL, "network kernels not built"};
}
void mlp_precond(const float*, const Plan&, void*, hipStream_t) {
    throw StatusError{EFGP_EMODEL, "network kernels not built"};
}

}  // namespace efgp
