// Setup stage instantiated for d = 1 (see setup_impl.h).
#include "setup_impl.h"

namespace efgp {
template void setup_typed<float, 1>(Plan&, const efgp_problem&, hipStream_t);
template void setup_typed<double, 1>(Plan&, const efgp_problem&, hipStream_t);
template void vhat64_typed<1>(Plan&, hipStream_t);
}  // namespace efgp
