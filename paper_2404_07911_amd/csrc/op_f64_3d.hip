// Operator kernels instantiated for double, dim = 3.
#include "kernels_impl.hpp"

namespace ufem {

template <>
hipError_t launch_operator_dim<double, 3>(const DevArgs<double>& a, int degree, const double* x, const double* y, double* v,
                                       double* dk, bool adj, hipStream_t s) {
  return kern::launch_d<3>(a, degree, x, y, v, dk, adj, s);
}

}  // namespace ufem
