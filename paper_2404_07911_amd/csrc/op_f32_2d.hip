// Operator kernels instantiated for float, dim = 2.
#include "kernels_impl.hpp"

namespace ufem {

template <>
hipError_t launch_operator_dim<float, 2>(const DevArgs<float>& a, int degree, const float* x, const float* y, float* v,
                                       float* dk, bool adj, hipStream_t s) {
  return kern::launch_d<2>(a, degree, x, y, v, dk, adj, s);
}

}  // namespace ufem
