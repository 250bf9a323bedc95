// Setup-stage dispatch; the kernels and the per-dimension orchestration are
// in setup_impl.h and instantiated once per dimension (setup_d1/2/3.hip).
#include "efgp_internal.h"

namespace efgp {

template <typename T, int DIM> void setup_typed(Plan& P, const efgp_problem& pr, hipStream_t s);

void run_setup(Plan& P, const efgp_problem& pr, hipStream_t s) {
    if (P.precision == 32) {
        if (P.dim == 1) setup_typed<float, 1>(P, pr, s);
        else if (P.dim == 2) setup_typed<float, 2>(P, pr, s);
        else setup_typed<float, 3>(P, pr, s);
    } else {
        if (P.dim == 1) setup_typed<double, 1>(P, pr, s);
        else if (P.dim == 2) setup_typed<double, 2>(P, pr, s);
        else setup_typed<double, 3>(P, pr, s);
    }
}

}  // namespace efgp
