// Setup stage instantiated for d = 3 (see setup_impl.h).
#include "setup_impl.h"

namespace efgp {
template void setup_typed<float, 3>(Plan&, const efgp_problem&, hipStream_t);
template void setup_typed<double, 3>(Plan&, const efgp_problem&, hipStream_t);
template void vhat64_typed<3>(Plan&, hipStream_t);
}  // namespace efgp
