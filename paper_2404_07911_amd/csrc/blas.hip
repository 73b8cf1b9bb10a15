// Solver BLAS-1 kernels and the operator dispatch by dimension.
#include <algorithm>

#include "device.hpp"

namespace ufem {
namespace {

// ---------------------------------------------------------------- BLAS-1
template <typename T>
__global__ void __launch_bounds__(256) dot_kernel(int64_t n, const T* __restrict__ x, const T* __restrict__ y,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)x[i] * (double)y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

__global__ void zero1_kernel(double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = 0.0;
}

template <typename T>
__global__ void __launch_bounds__(256) axpby_kernel(int64_t n, T a, const T* __restrict__ x, T b, T* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) cast_kernel(int64_t n, const TI* __restrict__ x, TO* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (TO)x[i];
}

template <typename T>
__global__ void __launch_bounds__(256) zero_kernel(int64_t n, T* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = T(0);
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }
// kernels that end in one atomic add per block onto one address: a grid of
// at most 1024 blocks (four per compute unit, enough to stream the vectors
// at full bandwidth) keeps the atomics on the one cache line few (8192 of
// them cost more than the streaming itself)
int grid_red(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024)); }

// ------------------------------------------------- conjugate gradients
// Device-resident CG: the scalars live in device memory, scal = [r.r, p.Ap,
// new r.r, breakdown flag]; p.Ap and the new r.r are accumulated in FP64 by
// block sums and one atomic add per block, and cleared again by cg_roll.
__device__ __forceinline__ double block_sum(double s) {
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// r -= alpha Ap, new r.r; alpha = r.r / p.Ap (x is updated with the old p
// by the direction kernel, which reads p anyway)
template <typename T>
__global__ void __launch_bounds__(256) cg_update_kernel(int64_t n, T* __restrict__ r, const T* __restrict__ ap,
                                                        double* __restrict__ scal) {
  const double pap = scal[1];
  if (scal[3] != 0.0 || !(pap > 0.0)) return;
  const T alpha = (T)(scal[0] / pap);
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T ri = r[i] - alpha * ap[i];
    r[i] = ri;
    s += (double)ri * (double)ri;
  }
  const double bs = block_sum(s);
  if (threadIdx.x == 0) atomicAdd(scal + 2, bs);
}

// x += alpha p, then p = r + beta p; beta = new r.r / r.r
template <typename T>
__global__ void __launch_bounds__(256) cg_direction_kernel(int64_t n, T* __restrict__ x, const T* __restrict__ r,
                                                           T* __restrict__ p, const double* __restrict__ scal) {
  if (scal[3] != 0.0 || !(scal[1] > 0.0)) return;
  const T alpha = (T)(scal[0] / scal[1]);
  const T beta = (T)(scal[2] / scal[0]);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T pi = p[i];
    x[i] += alpha * pi;
    p[i] = r[i] + beta * pi;
  }
}

// next iteration's scalars (one thread); a non-positive p.Ap stops the loop
__global__ void cg_roll_kernel(double* scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (scal[3] == 0.0) {
    if (!(scal[1] > 0.0)) scal[3] = 1.0;
    else scal[0] = scal[2];
  }
  scal[1] = 0.0;
  scal[2] = 0.0;
}

// the static-workspace CG: scalars cleared before r.r is accumulated, and
// the result (new r.r, breakdown flag) copied out at the end
__global__ void cg_clear4_kernel(double* scal) {
  if (blockIdx.x == 0 && threadIdx.x < 4) scal[threadIdx.x] = 0.0;
}

__global__ void cg_result_kernel(const double* __restrict__ scal, double* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out[0] = scal[0];
    out[1] = scal[3];
  }
}

}  // namespace

// Fixed workspace of ufem_cg_iterate_static, one copy per device for the
// life of the process: kStaticCgScalarBytes of CG scalars, then A p.  Host
// code never passes this name to a kernel: it takes the device address from
// static_scratch_address once per device (the name is a host-side stand-in).
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch_address(void** out) { return hipGetSymbolAddress(out, HIP_SYMBOL(scratch)); }

hipError_t launch_cg_static_begin(int prec, int64_t n, const void* r, double* scal, hipStream_t s) {
  cg_clear4_kernel<<<1, 64, 0, s>>>(scal);
  if (n > 0) {
    if (prec == 0)
      dot_kernel<double><<<grid_red(n), 256, 0, s>>>(n, (const double*)r, (const double*)r, scal);
    else
      dot_kernel<float><<<grid_red(n), 256, 0, s>>>(n, (const float*)r, (const float*)r, scal);
  }
  return hipGetLastError();
}

hipError_t launch_cg_static_end(const double* scal, double* out, hipStream_t s) {
  cg_result_kernel<<<1, 64, 0, s>>>(scal, out);
  return hipGetLastError();
}

hipError_t launch_cg_tail(int prec, int64_t n, void* x, void* r, void* p, const void* ap, double* scal, hipStream_t s) {
  const int g = grid_for(n), gr = grid_red(n);
  if (n > 0) {
    if (prec == 0) {
      dot_kernel<double><<<gr, 256, 0, s>>>(n, (const double*)p, (const double*)ap, scal + 1);
      cg_update_kernel<double><<<gr, 256, 0, s>>>(n, (double*)r, (const double*)ap, scal);
      cg_direction_kernel<double><<<g, 256, 0, s>>>(n, (double*)x, (const double*)r, (double*)p, scal);
    } else {
      dot_kernel<float><<<gr, 256, 0, s>>>(n, (const float*)p, (const float*)ap, scal + 1);
      cg_update_kernel<float><<<gr, 256, 0, s>>>(n, (float*)r, (const float*)ap, scal);
      cg_direction_kernel<float><<<g, 256, 0, s>>>(n, (float*)x, (const float*)r, (float*)p, scal);
    }
  }
  cg_roll_kernel<<<1, 64, 0, s>>>(scal);
  return hipGetLastError();
}


template <typename T>
hipError_t launch_operator(const DevArgs<T>& a, int dim, int degree, const T* u, T* v, const T* w_adj, T* dkappa,
                           bool adjoint, hipStream_t s) {
  // adjoint: the operator acts on w (A^T w = A w), u enters dkappa only
  const T* x = adjoint ? w_adj : u;
  const T* y = adjoint ? u : nullptr;
  if (dim == 3) return launch_operator_dim<T, 3>(a, degree, x, y, v, dkappa, adjoint, s);
  if (dim == 2) return launch_operator_dim<T, 2>(a, degree, x, y, v, dkappa, adjoint, s);
  return hipErrorInvalidValue;
}

template hipError_t launch_operator<double>(const DevArgs<double>&, int, int, const double*, double*, const double*,
                                            double*, bool, hipStream_t);
template hipError_t launch_operator<float>(const DevArgs<float>&, int, int, const float*, float*, const float*, float*,
                                           bool, hipStream_t);

hipError_t launch_dot(int prec, int64_t n, const void* x, const void* y, double* out, hipStream_t s) {
  zero1_kernel<<<1, 64, 0, s>>>(out);
  if (n > 0) {
    if (prec == 0)
      dot_kernel<double><<<grid_red(n), 256, 0, s>>>(n, (const double*)x, (const double*)y, out);
    else
      dot_kernel<float><<<grid_red(n), 256, 0, s>>>(n, (const float*)x, (const float*)y, out);
  }
  return hipGetLastError();
}

hipError_t launch_axpby(int prec, int64_t n, double a, const void* x, double b, void* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (prec == 0)
    axpby_kernel<double><<<grid_for(n), 256, 0, s>>>(n, a, (const double*)x, b, (double*)y);
  else
    axpby_kernel<float><<<grid_for(n), 256, 0, s>>>(n, (float)a, (const float*)x, (float)b, (float*)y);
  return hipGetLastError();
}

hipError_t launch_cast(int pin, int pout, int64_t n, const void* x, void* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int g = grid_for(n);
  if (pin == 0 && pout == 1) cast_kernel<double, float><<<g, 256, 0, s>>>(n, (const double*)x, (float*)y);
  else if (pin == 1 && pout == 0) cast_kernel<float, double><<<g, 256, 0, s>>>(n, (const float*)x, (double*)y);
  else if (pin == 0) cast_kernel<double, double><<<g, 256, 0, s>>>(n, (const double*)x, (double*)y);
  else cast_kernel<float, float><<<g, 256, 0, s>>>(n, (const float*)x, (float*)y);
  return hipGetLastError();
}

hipError_t launch_zero(int prec, int64_t n, void* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (prec == 0) zero_kernel<double><<<grid_for(n), 256, 0, s>>>(n, (double*)y);
  else zero_kernel<float><<<grid_for(n), 256, 0, s>>>(n, (float*)y);
  return hipGetLastError();
}

}  // namespace ufem

// ------------------------------------------- mixed evaluation set-up
namespace ufem {
namespace {

template <typename T>
__global__ void __launch_bounds__(256) unit_rows_kernel(int64_t n_dofs, int nd, int n_cut,
                                                        const int32_t* __restrict__ cut_rank, int j, T* __restrict__ x) {
  // zero everywhere, then 1 at local index j of every cut cell
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_dofs; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = T(0);
}

template <typename T>
__global__ void __launch_bounds__(256) unit_rows_set_kernel(int nd, int n_cut, const int32_t* __restrict__ cut_rank,
                                                            int j, T* __restrict__ x) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n_cut; c += gridDim.x * blockDim.x)
    x[(int64_t)cut_rank[c] * nd + j] = T(1);
}

template <typename T>
__global__ void __launch_bounds__(256) matrix_column_kernel(int nd, int n_cut, const int32_t* __restrict__ cut_rank,
                                                            int j, const T* __restrict__ v, T* __restrict__ mat) {
  const int64_t total = (int64_t)n_cut * nd;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / nd;
    const int i = (int)(idx % nd);
    mat[c * nd * (int64_t)nd + (int64_t)j * nd + i] = v[(int64_t)cut_rank[c] * nd + i];
  }
}

__global__ void __launch_bounds__(256) matrix_cast_kernel(int64_t n, const double* __restrict__ in,
                                                          float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

int grid_for2(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

}  // namespace

hipError_t launch_unit_rows(int prec, int64_t n_dofs, int nd, int n_cut, const int32_t* cut_rank, int j, void* x,
                            hipStream_t s) {
  if (prec == 0) {
    unit_rows_kernel<double><<<grid_for2(n_dofs), 256, 0, s>>>(n_dofs, nd, n_cut, cut_rank, j, (double*)x);
    if (n_cut > 0) unit_rows_set_kernel<double><<<grid_for2(n_cut), 256, 0, s>>>(nd, n_cut, cut_rank, j, (double*)x);
  } else {
    unit_rows_kernel<float><<<grid_for2(n_dofs), 256, 0, s>>>(n_dofs, nd, n_cut, cut_rank, j, (float*)x);
    if (n_cut > 0) unit_rows_set_kernel<float><<<grid_for2(n_cut), 256, 0, s>>>(nd, n_cut, cut_rank, j, (float*)x);
  }
  return hipGetLastError();
}

hipError_t launch_matrix_column(int prec, int nd, int n_cut, const int32_t* cut_rank, int j, const void* v, void* mat,
                                hipStream_t s) {
  if (n_cut <= 0) return hipSuccess;
  const int g = grid_for2((int64_t)n_cut * nd);
  if (prec == 0)
    matrix_column_kernel<double><<<g, 256, 0, s>>>(nd, n_cut, cut_rank, j, (const double*)v, (double*)mat);
  else
    matrix_column_kernel<float><<<g, 256, 0, s>>>(nd, n_cut, cut_rank, j, (const float*)v, (float*)mat);
  return hipGetLastError();
}

hipError_t launch_matrix_cast(int64_t n, const double* in, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  matrix_cast_kernel<<<grid_for2(n), 256, 0, s>>>(n, in, out);
  return hipGetLastError();
}

}  // namespace ufem

// ------------------------------------------- continuous space: P and P^T
namespace ufem {
namespace {

template <typename T>
__global__ void __launch_bounds__(256) gather_kernel(int64_t n_cell, const int32_t* __restrict__ cell_node,
                                                     const T* __restrict__ u, T* __restrict__ ucell) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_cell; i += (int64_t)gridDim.x * blockDim.x)
    ucell[i] = u[cell_node[i]];
}

// every node sums its cells' contributions in the fixed order of node_src
// (no atomics: repeated applies are bit-identical).  A lattice node lies in
// at most 2^3 cells: all its source indices are loaded at once, then all
// values, so that a node costs two dependent memory round trips.
constexpr int kMaxNodeCells = 8;
template <typename T>
__global__ void __launch_bounds__(256) scatter_kernel(int64_t n_nodes, const int64_t* __restrict__ node_ptr,
                                                      const int32_t* __restrict__ node_src,
                                                      const T* __restrict__ vcell, T* __restrict__ v) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_nodes; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = node_ptr[j];
    const int n = (int)(node_ptr[j + 1] - b);
    int src[kMaxNodeCells];
#pragma unroll
    for (int k = 0; k < kMaxNodeCells; ++k) src[k] = k < n ? node_src[b + k] : 0;
    T val[kMaxNodeCells];
#pragma unroll
    for (int k = 0; k < kMaxNodeCells; ++k) val[k] = k < n ? vcell[src[k]] : T(0);
    T s = 0;
#pragma unroll
    for (int k = 0; k < kMaxNodeCells; ++k)
      if (k < n) s += val[k];
    v[j] = s;
  }
}

int grid_for3(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

}  // namespace

hipError_t launch_gather(int prec, int64_t n_cell, const int32_t* cell_node, const void* u, void* ucell,
                         hipStream_t s) {
  if (n_cell <= 0) return hipSuccess;
  if (prec == 0)
    gather_kernel<double><<<grid_for3(n_cell), 256, 0, s>>>(n_cell, cell_node, (const double*)u, (double*)ucell);
  else
    gather_kernel<float><<<grid_for3(n_cell), 256, 0, s>>>(n_cell, cell_node, (const float*)u, (float*)ucell);
  return hipGetLastError();
}

hipError_t launch_scatter(int prec, int64_t n_nodes, const int64_t* node_ptr, const int32_t* node_src,
                          const void* vcell, void* v, hipStream_t s) {
  if (n_nodes <= 0) return hipSuccess;
  if (prec == 0)
    scatter_kernel<double><<<grid_for3(n_nodes), 256, 0, s>>>(n_nodes, node_ptr, node_src, (const double*)vcell,
                                                               (double*)v);
  else
    scatter_kernel<float><<<grid_for3(n_nodes), 256, 0, s>>>(n_nodes, node_ptr, node_src, (const float*)vcell,
                                                              (float*)v);
  return hipGetLastError();
}

}  // namespace ufem
