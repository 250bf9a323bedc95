// Setup-stage dispatch; the kernels and the per-dimension orchestration are
// in setup_impl.h and instantiated once per dimension (setup_d1/2/3.hip).
#include "efgp_internal.h"

namespace efgp {

template <typename T, int DIM> void setup_typed(Plan& P, const efgp_problem& pr, hipStream_t s);
template <int DIM> void vhat64_typed(Plan& P, hipStream_t s);

void build_vhat64(Plan& P, hipStream_t s) {
    if (P.dim == 1) vhat64_typed<1>(P, s);
    else if (P.dim == 2) vhat64_typed<2>(P, s);
    else vhat64_typed<3>(P, s);
}

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
