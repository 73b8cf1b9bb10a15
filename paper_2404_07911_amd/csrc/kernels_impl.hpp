// HIP kernels of the matrix-free unfitted DG operator (gfx950).
//
// Cell-centric schedule: every row of v belongs to one cell and is written
// by the wave that owns the cell in each stage, so no global atomics and no
// colouring are needed; each interior face flux is computed from both sides.
//
//  * structured terms (Section 3.2, structured quadrature evaluation): with
//    kappa = 1 the cell operator is a sum of Kronecker products of the 1D
//    mass and stiffness matrices plus face terms at the Gauss-Lobatto face
//    nodes (inside_kron_kernel, one lane per 1D line); with a kappa field
//    the same line passes go through the k^d Gauss points, where the kappa
//    of each point weights the integrand (kappa_struct_kernel);
//  * cut cells (Section 3.2, unstructured quadrature evaluation): the points
//    of the dimension-reduction quadrature lie on lines along one axis, so
//    per line the d-1 off-axis 1D Lagrange factors are fixed and only the
//    on-axis one changes from point to point (cut_batch_kernel for volume
//    and interface lines, cut_face_kernel for the lines of the cut faces,
//    whose face-normal traces are interpolated structurally first);
//  * dL/dkappa (the adjoint pass): the same evaluations with both arguments,
//    one value per quadrature point (inside_dk, face_dk, cut_dk,
//    cut_face_dk kernels).
#pragma once
#include <algorithm>

#include "device.hpp"

namespace ufem {
namespace kern {

constexpr __host__ __device__ int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

__device__ __forceinline__ void sync() { __syncthreads(); }

// Workgroups are handed to the 8 XCDs round robin, each XCD with its own L2.
// xcd_block renumbers them so that each XCD works on one contiguous range of
// block indices (a contiguous range of cells), which keeps the neighbours a
// cell reads in the L2 that read them first.  A bijection of [0, gridDim.x).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  if (nb < kXcds) return b;
  const int q = nb / kXcds, r = nb % kXcds, x = b % kXcds, i = b / kXcds;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// 1D GLL Lagrange values and first derivatives at t: L_i = ID_i prod_{j != i}
// (t - X_j).  Up to K = 4 each i takes its own product (K independent
// chains); from K = 5 on the products over j < i and j > i are formed once
// as prefix and suffix products with their derivatives (about 10 K instead
// of 2 K^2 operations: 76 against 136 at K = 8).
template <int K, typename T>
__device__ __forceinline__ void lagrange1d(const T* __restrict__ X, const T* __restrict__ ID, T t, T* L, T* dL) {
  if constexpr (K <= 4) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      T prod = 1, dsum = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (j == i) continue;
        const T f = t - X[j];
        dsum = dsum * f + prod;
        prod = prod * f;
      }
      L[i] = prod * ID[i];
      dL[i] = dsum * ID[i];
    }
  } else {
    T f[K], P[K], dP[K];
#pragma unroll
    for (int j = 0; j < K; ++j) f[j] = t - X[j];
    P[0] = 1;
    dP[0] = 0;
#pragma unroll
    for (int i = 1; i < K; ++i) {
      dP[i] = dP[i - 1] * f[i - 1] + P[i - 1];
      P[i] = P[i - 1] * f[i - 1];
    }
    T S = 1, dS = 0;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
      L[i] = P[i] * S * ID[i];
      dL[i] = (dP[i] * S + P[i] * dS) * ID[i];
      dS = dS * f[i] + S;
      S = S * f[i];
    }
  }
}

// cell index of in-face node f at layer l along `axis`
template <int K, int D>
__device__ __forceinline__ int cell_index(int axis, int f, int l) {
  if constexpr (D == 2) {
    return axis == 0 ? (l + K * f) : (f + K * l);
  } else {
    const int f0 = f % K, f1 = f / K;
    if (axis == 0) return l + K * f0 + K * K * f1;
    if (axis == 1) return f0 + K * l + K * K * f1;
    return f0 + K * f1 + K * K * l;
  }
}

// ------------------------------------------------ inside cells, kappa = 1
// With a constant coefficient, exact Gauss integration and the Cartesian
// metric, the operator restricted to an inside cell is a sum of Kronecker
// products of the 1D GLL mass M and stiffness KS (the structured cell
// evaluation of Section 3.2 with the quadrature folded into the 1D
// matrices):
//   v = hs [ M_z (M_y R_x + M_x R_y) + M_x M_y R_z ],
//   R_a = KS_a u + sum over the two faces normal to a of C_a,
// where C_a[layer l, face node f] collects the face terms at the
// Gauss-Lobatto face nodes: SIPG  e_l sigma (gamma [u] - {d_n u}) - g_l [u] / 2
// and ghost penalty  sum_j gamma_j E^j_l (d^j u_own - d^j u_nb)
// (e, g, E^j: value, first and j-th derivative of the own basis at the face);
// the in-face mass M (x) M of the face integrals is applied by the
// subsequent passes.  One lane per 1D line, CK cells per workgroup.
template <int K, int D>
struct KronShape {
  static constexpr int ND = ipow(K, D);
  static constexpr int NL = ipow(K, D - 1);           // lines per direction
  static constexpr int C = 64 / NL;                   // cells per wave
  static constexpr int NT = 64;
  // the Kronecker kernel's workgroup: two waves at K = 5, 6, where one wave
  // holds 2 / 1 cells (50 / 36 of its 64 lanes busy) and two hold 5 / 3
  // (structured stage -5 % / -20 % measured; the other degrees lose)
  static constexpr int NTK = K == 5 || K == 6 ? 128 : 64;
  static constexpr int CK = NTK / NL;
};

// LDS layout of a cell tensor in the Kronecker kernel: element (i0, i1, i2)
// at ((i0 + i2) mod K) + K ((i1 + i2) mod K) + K^2 i2 (3D), (i0 + i1) mod K +
// K i1 (2D).  The lanes of a cell (one per line) then hit distinct banks in
// the passes along every axis, and the cell stride (NDP, = 16 mod 32
// elements) separates the cells of a wave.
template <int K, int D>
struct KronLayout {
  static constexpr int ND = ipow(K, D);
  static constexpr int NDP = ND + (16 - ND % 32 + 32) % 32;
  static __device__ __forceinline__ int at(int i0, int i1, int i2) {
    if constexpr (D == 3) return (i0 + i2) % K + K * ((i1 + i2) % K) + K * K * i2;
    else return (i0 + i1) % K + K * i1;
  }
  // the K LDS positions of line l along axis AX
  template <int AX>
  static __device__ __forceinline__ void line(int l, int* pos) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      if constexpr (D == 2) pos[q] = AX == 0 ? at(q, l, 0) : at(l, q, 0);
      else {
        const int a = l % K, b = l / K;
        pos[q] = AX == 0 ? at(q, a, b) : (AX == 1 ? at(a, q, b) : at(a, b, q));
      }
    }
  }
};

template <int K, int D, typename T>
struct KronWork {
  static constexpr int NDP = KronLayout<K, D>::NDP, C = KronShape<K, D>::CK;
  T A[C][NDP];
  T Cc[C][NDP];
  T U[C][NDP];
};

// waves per SIMD the Kronecker kernel asks the compiler for (the register
// budget 512 / W; 1: no request).  Three at K = 7 in double (a few spilled
// registers, the structured stage -11 % at p = 6); the other requests
// measured (five at K = 4, 5, four at K = 6, three at K = 8 in double, five
// at K = 7, 8 in float) spilled more and were slower)
template <int K, typename T>
struct KronOcc {
  static constexpr int W = sizeof(T) == 8 && K == 7 ? 3 : 1;
};

template <int K, typename T>
__device__ __forceinline__ void kl_load(const T* arr, const int* pos, T* v) {
#pragma unroll
  for (int q = 0; q < K; ++q) v[q] = arr[pos[q]];
}
template <int K, typename T>
__device__ __forceinline__ void kl_store(T* arr, const int* pos, const T* v) {
#pragma unroll
  for (int q = 0; q < K; ++q) arr[pos[q]] = v[q];
}

// element stride of the lines along axis ax, and the first element of line l
template <int K, int D, int AX>
__device__ __forceinline__ constexpr int line_stride() {
  return ipow(K, AX);
}
template <int K, int D, int AX>
__device__ __forceinline__ int line_base(int l) {
  if constexpr (D == 2) return AX == 0 ? K * l : l;
  else {
    const int a = l % K, b = l / K;
    if constexpr (AX == 0) return K * a + K * K * b;
    else if constexpr (AX == 1) return a + K * K * b;
    else return a + K * b;
  }
}

// y = M x along a line (M row-major K x K, uniform across the wave)
template <int K, typename T>
__device__ __forceinline__ void line_mat(const T* __restrict__ M, const T* x, T* y) {
#pragma unroll
  for (int r = 0; r < K; ++r) {
    T s = 0;
#pragma unroll
    for (int q = 0; q < K; ++q) s += M[r * K + q] * x[q];
    y[r] = s;
  }
}

// SIPG and ghost-penalty face terms of the two faces normal to the line
// axis, added to the line of R (own line uo, neighbour lines nlo / nhi)
template <int K, typename T>
__device__ __forceinline__ void line_faces(const T* __restrict__ tab, const DevArgs<T>& a, int fl, int ax,
                                           const T* uo, const T* nlo, const T* nhi, T* R) {
  const bool ghost = (a.terms & 8) != 0, sipg = (a.terms & 2) != 0;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int s = 2 * ax + side;
    const bool fs = sipg && ((fl >> (kFlagStr + s)) & 1);
    const bool fg = ghost && ((fl >> (kFlagGP + s)) & 1);
    if (!fs && !fg) continue;
    const T* Eo = tab + (side ? TabOff::E1(K) : TabOff::E0(K));
    const T* En = tab + (side ? TabOff::E0(K) : TabOff::E1(K));
    const T* un = side ? nhi : nlo;
    const T sigma = side ? T(1) : T(-1);
    if (fs) {
      // the basis is nodal on Gauss-Lobatto points, so a line's value at a
      // face is its end-point DoF (own: node io, neighbour: node in) and
      // the value test functions of the face are the unit vector at io
      const int io = side ? K - 1 : 0, in = side ? 0 : K - 1;
      T od = 0, nd = 0;
#pragma unroll
      for (int l = 0; l < K; ++l) {
        od += Eo[K + l] * uo[l];
        nd += En[K + l] * un[l];
      }
      const T J = sigma * (uo[io] - un[in]);
      const T Av = T(0.5) * (od + nd);
      const T cv = sigma * (a.gamma * J - Av);
      const T cd = T(-0.5) * J;
#pragma unroll
      for (int l = 0; l < K; ++l) R[l] += Eo[K + l] * cd;
      R[io] += cv;
    }
    if (fg) {
      // face ghost penalty: sum_j gamma_j E^j_l (d^j u_own - d^j u_nb),
      // folded into two K x K matrices on the host; volume ghost penalty:
      // tau_v times the patch mass products along the line (the in-face
      // mass follows in the later passes)
      const T* Go = tab + TabOff::GP(K) + 2 * side * K * K;
      const T* Gn = Go + K * K;
#pragma unroll
      for (int l = 0; l < K; ++l) {
        T r = R[l];
#pragma unroll
        for (int m = 0; m < K; ++m) {
          r += Go[l * K + m] * uo[m];
          r -= Gn[l * K + m] * un[m];
        }
        R[l] = r;
      }
    }
  }
}

template <int K, int D, int AX, typename T>
__device__ __forceinline__ void glb_line_load(const T* __restrict__ src, int base, T* v) {
#pragma unroll
  for (int q = 0; q < K; ++q) v[q] = src[base + q * line_stride<K, D, AX>()];
}

// One wave handles C inside cells; each lane owns one 1D line of its cell
// in every pass (x-, y-, z-lines in turn), so a contraction costs K loads,
// K^2 FMAs and K stores per lane and the 1D matrices are wave-uniform:
//   v = hs [ M_z (M_y R_x + M_x R_y) + M_y M_x R_z ]
template <int K, int D, typename T>
__global__ void __launch_bounds__((KronShape<K, D>::NTK)) __attribute__((amdgpu_waves_per_eu(KronOcc<K, T>::W))) inside_kron_kernel(DevArgs<T> a, const T* __restrict__ x, T* __restrict__ v,
                                                         const int32_t* __restrict__ kinfo, int n_list, int with_volume) {
  constexpr int ND = KronShape<K, D>::ND, NL = KronShape<K, D>::NL, C = KronShape<K, D>::CK;
  __shared__ KronWork<K, D, T> W;
  const T* __restrict__ tab = a.tab;
  const T* M = tab + TabOff::M(K);
  const T* KS = tab + TabOff::KS(K);
  const int lane = threadIdx.x;
  const int c = lane / NL, l = lane % NL;
  const bool active = c < C;
  // cells flagged kFlagNoVolume (cut cells in the combined list) take the
  // faces only
  const bool vol_all = with_volume && (a.terms & 1) != 0;
  for (int c0 = xcd_block() * C; c0 < n_list; c0 += gridDim.x * C) {
    const int ci = c0 + c;
    const bool valid = active && ci < n_list;
    // the cell's rank, flags and neighbours in one load, then every global
    // read of the cell at once: own x-line and the neighbours' lines through
    // this lane's face nodes of the x-, y- and z-faces
    int4 k0 = make_int4(0, 0, 0, 0), k1 = make_int4(0, 0, 0, 0);
    if (valid) {
      k0 = reinterpret_cast<const int4*>(kinfo)[2 * ci];
      k1 = reinterpret_cast<const int4*>(kinfo)[2 * ci + 1];
    }
    const int r = k0.x, fl = k0.y;
    const bool vol = vol_all && !((fl >> kFlagNoVolume) & 1);
    const int nbr[6] = {k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
    T ux[K], nb[2 * D][K];
    const int bx = line_base<K, D, 0>(l), by = line_base<K, D, 1>(l);
    const int bz = D == 3 ? line_base<K, D, 2>(l) : 0;
    if (valid) {
      glb_line_load<K, D, 0>(x + (int64_t)r * ND, bx, ux);
#pragma unroll
      for (int s = 0; s < 2 * D; ++s) {
        if (!((((fl >> (kFlagStr + s)) & (a.terms >> 1)) | ((fl >> (kFlagGP + s)) & (a.terms >> 3))) & 1)) continue;
        const T* un = x + (int64_t)nbr[s] * ND;
        const int ax = s >> 1;
        if (ax == 0) glb_line_load<K, D, 0>(un, bx, nb[s]);
        else if (ax == 1) glb_line_load<K, D, 1>(un, by, nb[s]);
        else if constexpr (D == 3) glb_line_load<K, D, 2>(un, bz, nb[s]);
      }
    }
    T* U = W.U[active ? c : 0];
    T* A = W.A[active ? c : 0];
    T* Cc = W.Cc[active ? c : 0];
    T t0[K], t1[K], t2[K];
    int px[K], py[K], pz[K];
    KronLayout<K, D>::template line<0>(l, px);
    KronLayout<K, D>::template line<1>(l, py);
    if constexpr (D == 3) KronLayout<K, D>::template line<2>(l, pz);
    // Three cell tensors in LDS (A, Cc, U); each pass reads and writes only
    // its own lanes' lines, so the updates in place need no extra array.
    // pass x1: R_x = KS u + x-faces -> A ; u -> U
    if (valid) {
      kl_store<K>(U, px, ux);
      if (vol) line_mat<K>(KS, ux, t0);
      else {
#pragma unroll
        for (int q = 0; q < K; ++q) t0[q] = 0;
      }
      line_faces<K>(tab, a, fl, 0, ux, nb[0], nb[1], t0);
      kl_store<K>(A, px, t0);
    }
    sync();
    // pass y1: R_y = KS u + y-faces -> Cc ; A = M_y R_x (in place)
    if (valid) {
      kl_load<K>(U, py, t1);
      if (vol) line_mat<K>(KS, t1, t0);
      else {
#pragma unroll
        for (int q = 0; q < K; ++q) t0[q] = 0;
      }
      line_faces<K>(tab, a, fl, 1, t1, nb[2], nb[3], t0);
      kl_store<K>(Cc, py, t0);
      kl_load<K>(A, py, t1);
      line_mat<K>(M, t1, t2);
      kl_store<K>(A, py, t2);
    }
    sync();
    if constexpr (D == 3) {
      // pass z1: R_z = KS u + z-faces -> U (in place)
      if (valid) {
        kl_load<K>(U, pz, t1);
        if (vol) line_mat<K>(KS, t1, t0);
        else {
#pragma unroll
          for (int q = 0; q < K; ++q) t0[q] = 0;
        }
        line_faces<K>(tab, a, fl, 2, t1, nb[4], nb[5], t0);
        kl_store<K>(U, pz, t0);
      }
      sync();
      // pass x2: S = M_y R_x + M_x R_y -> A ; M_x R_z -> Cc
      if (valid) {
        kl_load<K>(Cc, px, t1);
        line_mat<K>(M, t1, t2);
        kl_load<K>(A, px, t1);
#pragma unroll
        for (int q = 0; q < K; ++q) t2[q] += t1[q];
        kl_store<K>(A, px, t2);
        kl_load<K>(U, px, t1);
        line_mat<K>(M, t1, t2);
        kl_store<K>(Cc, px, t2);
      }
      sync();
      // pass z2: M_z S -> U
      if (valid) {
        kl_load<K>(A, pz, t1);
        line_mat<K>(M, t1, t2);
        kl_store<K>(U, pz, t2);
      }
      sync();
      // pass y2: v = hs (M_z S + M_y M_x R_z)
      if (valid) {
        kl_load<K>(Cc, py, t1);
        line_mat<K>(M, t1, t2);
        kl_load<K>(U, py, t1);
        T* out = v + (int64_t)r * ND;
#pragma unroll
        for (int q = 0; q < K; ++q) out[by + q * K] = a.hs * (t2[q] + t1[q]);
      }
    } else {
      // pass x2: v = hs (M_y R_x + M_x R_y)
      if (valid) {
        kl_load<K>(Cc, px, t1);
        line_mat<K>(M, t1, t2);
        kl_load<K>(A, px, t1);
        T* out = v + (int64_t)r * ND;
#pragma unroll
        for (int q = 0; q < K; ++q) out[bx + q] = a.hs * (t2[q] + t1[q]);
      }
    }
    sync();
  }
}

// ------------------------------------------------ structured terms with kappa
// One wave handles C cells (inside cells with their volume term, or cut
// cells for their structured faces and ghost penalty), one lane per 1D line
// as in the Kronecker kernel.  Volume: the reference gradient at the k^d
// Gauss points by three line passes (S: GLL basis at the Gauss points, DS:
// its derivative), times w_q kappa_q h^(d-2), and the transposed passes back
// to the nodes (the paper's structured evaluation, Section 3.2).  Faces
// (Gauss-Lobatto node grid of the face = the lines along the normal axis):
// SIPG from the value and normal-derivative traces of both sides,
// interpolated to the face Gauss points, weighted by w_q kappa_q h^(d-2) and
// integrated back; ghost penalty from the derivative jumps of every order
// times the exact in-face mass matrices (no kappa).  Rows are overwritten.
template <int K, int D, typename T>
struct KappaWork {
  static constexpr int NDP = KronLayout<K, D>::NDP, C = KronShape<K, D>::C, NF = ipow(K, D - 1);
  T A[C][NDP];
  T B[C][NDP];
  T Cc[C][NDP];
  T U[C][NDP];
  T OUT[C][NDP];
  T F0[C][NF];
  T F1[C][NF];
  T FJ[C][K][NF];  // derivative jumps of every order (ghost penalty)
};

// y = M^T x along a line (M row-major K x K, uniform across the wave)
template <int K, typename T>
__device__ __forceinline__ void line_matT(const T* __restrict__ M, const T* x, T* y) {
#pragma unroll
  for (int r = 0; r < K; ++r) {
    T s = 0;
#pragma unroll
    for (int q = 0; q < K; ++q) s += M[q * K + r] * x[q];
    y[r] = s;
  }
}

// in-face transform of a node field F (K^(D-1) values, lower in-face axis
// fastest) by M1 x M1 (M1 row-major K x K; TR: transposed), value at this
// lane's node f
template <int K, int D, bool TR, typename T>
__device__ __forceinline__ T face_transform(const T* __restrict__ M1, const T* F, int f) {
  if constexpr (D == 2) {
    T s = 0;
#pragma unroll
    for (int g = 0; g < K; ++g) s += (TR ? M1[g * K + f] : M1[f * K + g]) * F[g];
    return s;
  } else {
    const int f0 = f % K, f1 = f / K;
    T s = 0;
#pragma unroll
    for (int g1 = 0; g1 < K; ++g1) {
      T t = 0;
#pragma unroll
      for (int g0 = 0; g0 < K; ++g0) t += (TR ? M1[g0 * K + f0] : M1[f0 * K + g0]) * F[g0 + K * g1];
      s += (TR ? M1[g1 * K + f1] : M1[f1 * K + g1]) * t;
    }
    return s;
  }
}

// (up to K = 5 the kernel fits two waves per SIMD, in double with at most a
// couple of spilled registers; beyond, the spills would cost more)
template <int K, int D, typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(K <= 5 ? 2 : 1))) kappa_struct_kernel(DevArgs<T> a, const T* __restrict__ x, T* __restrict__ v,
                                                          const int32_t* __restrict__ kinfo,
                                                          const int64_t* __restrict__ kface, int n_list,
                                                          int with_volume) {
  constexpr int ND = KronShape<K, D>::ND, NL = KronShape<K, D>::NL, C = KronShape<K, D>::C;
  // the face loop skips its barriers on wave votes (no lane of the wave has
  // the face): correct only while a workgroup is one wave
  static_assert(KronShape<K, D>::NT == 64, "one-wave workgroups");
  __shared__ KappaWork<K, D, T> W;
  const T* __restrict__ tab = a.tab;
  const T* S = tab + TabOff::S(K);
  const T* DS = tab + TabOff::DS(K);
  const T* M = tab + TabOff::M(K);
  const T* Wg = tab + TabOff::W(K);
  const T* GW = tab + TabOff::GW(K);
  const int lane = threadIdx.x;
  const int c = lane / NL, l = lane % NL;
  const bool active = c < C;
  const int cc = active ? c : 0;
  const bool vol_on = with_volume && (a.terms & 1) != 0;
  const bool sipg_on = (a.terms & 2) != 0, gp_on = (a.terms & 8) != 0;
  int pos[D][K];
  KronLayout<K, D>::template line<0>(l, pos[0]);
  KronLayout<K, D>::template line<1>(l, pos[1]);
  if constexpr (D == 3) KronLayout<K, D>::template line<2>(l, pos[2]);
  for (int c0 = xcd_block() * C; c0 < n_list; c0 += gridDim.x * C) {
    const int ci = c0 + c;
    const bool valid = active && ci < n_list;
    int4 k0 = make_int4(0, 0, 0, 0), k1 = make_int4(0, 0, 0, 0);
    if (valid) {
      k0 = reinterpret_cast<const int4*>(kinfo)[2 * ci];
      k1 = reinterpret_cast<const int4*>(kinfo)[2 * ci + 1];
    }
    const int r = k0.x, fl = k0.y;
    const int nbr[6] = {k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
    const int bx = line_base<K, D, 0>(l), by = line_base<K, D, 1>(l);
    const int bz = D == 3 ? line_base<K, D, 2>(l) : 0;
    T ux[K];
    // float: every neighbour line and face offset loaded up front (enough
    // registers); double: one normal axis at a time in the face loop
    constexpr bool kRoll = sizeof(T) == 8;
    T nball[kRoll ? 1 : 2 * D][K];
    int64_t fkall[kRoll ? 1 : 2 * D];
    if (valid) {
      glb_line_load<K, D, 0>(x + (int64_t)r * ND, bx, ux);
      if constexpr (!kRoll) {
#pragma unroll
        for (int s = 0; s < 2 * D; ++s) {
          fkall[s] = kface[(int64_t)ci * 2 * D + s];
          if (!((((fl >> (kFlagStr + s)) & (a.terms >> 1)) | ((fl >> (kFlagGP + s)) & (a.terms >> 3))) & 1)) continue;
          const T* un = x + (int64_t)nbr[s] * ND;
          const int ax = s >> 1;
          if (ax == 0) glb_line_load<K, D, 0>(un, bx, nball[s]);
          else if (ax == 1) glb_line_load<K, D, 1>(un, by, nball[s]);
          else if constexpr (D == 3) glb_line_load<K, D, 2>(un, bz, nball[s]);
        }
      }
    }
    T* U = W.U[cc];
    T* A = W.A[cc];
    T* B = W.B[cc];
    T* Cc = W.Cc[cc];
    T* OUT = W.OUT[cc];
    T t0[K], t1[K], t2[K], t3[K];
    if (valid) {
      kl_store<K>(U, pos[0], ux);
#pragma unroll
      for (int q = 0; q < K; ++q) t0[q] = 0;
      kl_store<K>(OUT, pos[0], t0);
    }
    sync();
    // ---- volume
    const bool vol = vol_on && valid;
    if constexpr (D == 3) {
      if (vol) {
        line_mat<K>(S, ux, t0);
        line_mat<K>(DS, ux, t1);
        kl_store<K>(A, pos[0], t0);  // S_x u
        kl_store<K>(B, pos[0], t1);  // DS_x u
      }
      sync();
      if (vol) {
        kl_load<K>(A, pos[1], t0);
        line_mat<K>(S, t0, t1);
        line_mat<K>(DS, t0, t2);
        kl_store<K>(A, pos[1], t1);   // S_y S_x u
        kl_store<K>(Cc, pos[1], t2);  // DS_y S_x u
        kl_load<K>(B, pos[1], t0);
        line_mat<K>(S, t0, t1);
        kl_store<K>(B, pos[1], t1);   // S_y DS_x u
      }
      sync();
      if (vol) {
        // this lane's z-line: Gauss indices (q0, q1) = (l % K, l / K)
        const int q0 = l % K, q1 = l / K;
        kl_load<K>(A, pos[2], t0);
        line_mat<K>(DS, t0, t3);      // d/dz
        kl_load<K>(Cc, pos[2], t0);
        line_mat<K>(S, t0, t2);       // d/dy
        kl_load<K>(B, pos[2], t0);
        line_mat<K>(S, t0, t1);       // d/dx
        const int64_t kb = a.seg[0] + (int64_t)ci * ND + q0 + K * q1;
        const T w01 = a.hs * Wg[q0] * Wg[q1];
#pragma unroll
        for (int m = 0; m < K; ++m) {
          T cq = w01 * Wg[m];
          if (a.kappa) cq *= a.kappa[kb + K * K * m];
          t1[m] *= cq;
          t2[m] *= cq;
          t3[m] *= cq;
        }
        line_matT<K>(S, t1, t0);
        kl_store<K>(A, pos[2], t0);
        line_matT<K>(S, t2, t0);
        kl_store<K>(Cc, pos[2], t0);
        line_matT<K>(DS, t3, t0);
        kl_store<K>(B, pos[2], t0);
      }
      sync();
      if (vol) {
        kl_load<K>(A, pos[1], t0);
        line_matT<K>(S, t0, t1);
        kl_store<K>(A, pos[1], t1);   // S_y^T (x-part)
        kl_load<K>(Cc, pos[1], t0);
        line_matT<K>(DS, t0, t1);
        kl_load<K>(B, pos[1], t0);
        line_matT<K>(S, t0, t2);
#pragma unroll
        for (int q = 0; q < K; ++q) t1[q] += t2[q];
        kl_store<K>(B, pos[1], t1);   // DS_y^T (y-part) + S_y^T (z-part)
      }
      sync();
      if (vol) {
        kl_load<K>(A, pos[0], t0);
        line_matT<K>(DS, t0, t1);
        kl_load<K>(B, pos[0], t0);
        line_matT<K>(S, t0, t2);
#pragma unroll
        for (int q = 0; q < K; ++q) t1[q] += t2[q];
        kl_store<K>(OUT, pos[0], t1);
      }
      sync();
    } else {
      if (vol) {
        line_mat<K>(S, ux, t0);
        line_mat<K>(DS, ux, t1);
        kl_store<K>(A, pos[0], t0);  // S_x u
        kl_store<K>(B, pos[0], t1);  // DS_x u
      }
      sync();
      if (vol) {
        // this lane's y-line: Gauss index q0 = l
        kl_load<K>(A, pos[1], t0);
        line_mat<K>(DS, t0, t2);      // d/dy
        kl_load<K>(B, pos[1], t0);
        line_mat<K>(S, t0, t1);       // d/dx
        const int64_t kb = a.seg[0] + (int64_t)ci * ND + l;
        const T w0 = a.hs * Wg[l];
#pragma unroll
        for (int m = 0; m < K; ++m) {
          T cq = w0 * Wg[m];
          if (a.kappa) cq *= a.kappa[kb + K * m];
          t1[m] *= cq;
          t2[m] *= cq;
        }
        line_matT<K>(S, t1, t0);
        kl_store<K>(A, pos[1], t0);
        line_matT<K>(DS, t2, t0);
        kl_store<K>(B, pos[1], t0);
      }
      sync();
      if (vol) {
        kl_load<K>(A, pos[0], t0);
        line_matT<K>(DS, t0, t1);
        kl_load<K>(B, pos[0], t0);
        line_matT<K>(S, t0, t2);
#pragma unroll
        for (int q = 0; q < K; ++q) t1[q] += t2[q];
        kl_store<K>(OUT, pos[0], t1);
      }
      sync();
    }
    // ---- faces, one normal axis at a time (double: a loop that is not
    // unrolled, holding one axis's neighbour lines and face terms only); lane
    // l is face node / Gauss point l of the face (lower in-face axis fastest)
#pragma unroll(kRoll ? 1 : D)
    for (int ax = 0; ax < D; ++ax) {
      // this lane's line along ax: LDS positions, global offset and stride
      int pa[K];
      {
        const int la = l % K, lb = D == 3 ? l / K : 0;
#pragma unroll
        for (int q = 0; q < K; ++q)
          pa[q] = D == 2 ? (ax == 0 ? KronLayout<K, D>::at(q, l, 0) : KronLayout<K, D>::at(l, q, 0))
                         : (ax == 0 ? KronLayout<K, D>::at(q, la, lb)
                                    : (ax == 1 ? KronLayout<K, D>::at(la, q, lb) : KronLayout<K, D>::at(la, lb, q)));
      }
      const int gbase = ax == 0 ? bx : (ax == 1 ? by : bz);
      const int gstride = ax == 0 ? 1 : (ax == 1 ? K : K * K);
      T nbl[2][K];
      int64_t fko[2];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int s = 2 * ax + side;
        if constexpr (!kRoll) {
          fko[side] = fkall[s];
#pragma unroll
          for (int q = 0; q < K; ++q) nbl[side][q] = nball[s][q];
          continue;
        }
        fko[side] = 0;
#pragma unroll
        for (int q = 0; q < K; ++q) nbl[side][q] = 0;
        if (!valid) continue;
        fko[side] = kface[(int64_t)ci * 2 * D + s];
        if (!((((fl >> (kFlagStr + s)) & (a.terms >> 1)) | ((fl >> (kFlagGP + s)) & (a.terms >> 3))) & 1)) continue;
        const int ns = s == 0 ? nbr[0] : s == 1 ? nbr[1] : s == 2 ? nbr[2] : s == 3 ? nbr[3] : s == 4 ? nbr[4] : nbr[5];
        const T* un = x + (int64_t)ns * ND + gbase;
#pragma unroll
        for (int q = 0; q < K; ++q) nbl[side][q] = un[q * gstride];
      }
      T R[K];
#pragma unroll
      for (int q = 0; q < K; ++q) R[q] = 0;
      T uo[K];
      if (valid) kl_load<K>(U, pa, uo);
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int s = 2 * ax + side;
        // wave-uniform loop bounds: every lane takes part in the syncs
        const bool fs = valid && sipg_on && ((fl >> (kFlagStr + s)) & 1);
        const bool fg = valid && gp_on && ((fl >> (kFlagGP + s)) & 1);
        const T* Eo = tab + (side ? TabOff::E1(K) : TabOff::E0(K));
        const T* En = tab + (side ? TabOff::E0(K) : TabOff::E1(K));
        const T sigma = side ? T(1) : T(-1);
        const T* un = nbl[side];
        // ghost penalty: derivative jumps of every order, exact in-face mass
        // (skipped by waves without such a face on this slot)
        if (__any(fg)) {
          // face kind: the jumps of the normal derivatives of every order,
          // FJ[j] = E^j u_own - F^j u_nb; volume kind: the line of the patch
          // mass products, FJ[j] = (Go u_own - Gn u_nb)[j] (the in-face mass
          // of the patch integral is the face transform below)
          // (the two kinds in separate loops: a select inside one loop keeps
          // both tables' products live and costs registers)
          const bool vgp = a.gp_volume != 0;
          if (fg) {
            const T* Fo = vgp ? tab + TabOff::GP(K) + 2 * side * K * K : Eo;
            const T* Fn = vgp ? Fo + K * K : En;
#pragma unroll
            for (int j = 0; j < K; ++j) {
              T dj = 0;
#pragma unroll
              for (int q = 0; q < K; ++q) dj += Fo[j * K + q] * uo[q] - Fn[j * K + q] * un[q];
              W.FJ[cc][j][l] = dj;
            }
          }
          sync();
          if (fg) {
            if (vgp) {
#pragma unroll
              for (int j = 0; j < K; ++j) R[j] += a.hs * face_transform<K, D, false>(M, W.FJ[cc][j], l);
            } else {
#pragma unroll
              for (int j = 0; j < K; ++j) {
                const T g = a.hs * face_transform<K, D, false>(M, W.FJ[cc][j], l);
#pragma unroll
                for (int q = 0; q < K; ++q) R[q] += Eo[j * K + q] * (GW[j] * g);
              }
            }
          }
          sync();
        }
        if (!__any(fs)) continue;
        // SIPG with kappa at the face Gauss points
        if (fs) {
          T ov = 0, od = 0, nv = 0, nd = 0;
#pragma unroll
          for (int q = 0; q < K; ++q) {
            ov += Eo[q] * uo[q];
            od += Eo[K + q] * uo[q];
            nv += En[q] * un[q];
            nd += En[K + q] * un[q];
          }
          W.F0[cc][l] = sigma * (ov - nv);
          W.F1[cc][l] = T(0.5) * (od + nd);
        }
        sync();
        T fv = 0, fd = 0;
        if (fs) {
          const T J = face_transform<K, D, false>(S, W.F0[cc], l);
          const T Av = face_transform<K, D, false>(S, W.F1[cc], l);
          const int q0 = l % K, q1 = D == 3 ? l / K : 0;
          T cq = a.hs * Wg[q0] * (D == 3 ? Wg[q1] : T(1));
          if (a.kappa) cq *= a.kappa[fko[side] + l];
          fv = cq * sigma * (a.gamma * J - Av);
          fd = T(-0.5) * cq * J;
        }
        sync();
        if (fs) {
          W.F0[cc][l] = fv;
          W.F1[cc][l] = fd;
        }
        sync();
        if (fs) {
          const T gv = face_transform<K, D, true>(S, W.F0[cc], l);
          const T gd = face_transform<K, D, true>(S, W.F1[cc], l);
#pragma unroll
          for (int q = 0; q < K; ++q) R[q] += Eo[q] * gv + Eo[K + q] * gd;
        }
        sync();
      }
      if (valid) {
        kl_load<K>(OUT, pa, t0);
#pragma unroll
        for (int q = 0; q < K; ++q) t0[q] += R[q];
        kl_store<K>(OUT, pa, t0);
      }
      sync();
    }
    if (valid) {
      kl_load<K>(OUT, pos[0], t0);
      T* out = v + (int64_t)r * ND;
#pragma unroll
      for (int q = 0; q < K; ++q) out[bx + q] = t0[q];
    }
    sync();
  }
}

// ------------------------------------------------ cut cells, point lines
// One wave per cut cell.  The structured faces of the cell (SIPG on faces
// inside the domain, ghost penalty) use the Kronecker face pipeline of the
// inside cells.  The unstructured points (volume, interface, cut faces) come
// in lines: runs of points that share all coordinates but one (the
// dimension-reduction rule places q Gauss points on each height line).  One
// lane per line evaluates the 1D Lagrange polynomials of the fixed
// coordinates, contracts the cell DoFs over the fixed axes once (columns
// along the line axis), and then needs only 1D sums per point (Section 3.2,
// unstructured evaluation with the per-point 1D basis reused along the
// line).  The transposed sums leave a per-line record (fixed-axis basis and
// line-axis coefficients), and one lane per DoF adds the records of a round.
template <int K, int D>
struct LineShape {
  static constexpr int ND = ipow(K, D);
  static constexpr int NT = 64;
  // line record, K-vectors [V1 | dV1 | V2 | dV2 | D0 | D1 | D2] (3D) or
  // [V1 | dV1 | D0 | D1] (2D): the line's test-function coefficient of DoF
  // (i_KA, i_O1, i_O2) is V2 (V1 D0 + dV1 D1) + V1 dV2 D2
  static constexpr int RS = D == 3 ? 7 * K : 4 * K;
  static constexpr int V1 = 0, DV1 = K, V2 = 2 * K, DV2 = 3 * K, D0 = D == 3 ? 4 * K : 2 * K,
                       D1 = D0 + K, D2 = D0 + 2 * K;
  // records are stored one after the other with this stride (= 2 mod 4
  // elements: 16-byte aligned records whose pair accesses by consecutive
  // lanes fall into distinct bank groups); at K = 5 in 3D without padding,
  // so that a batch's LDS (one cell, 64 records) stays under 20 KiB and two
  // waves fit per SIMD (volume lines 209 -> 166 us at p = 4, 2e7 DoF)
  static constexpr int RSP = (K == 5 && D == 3) ? RS : RS + ((2 - RS % 4) + 4) % 4;
};

// columns along axis KA of the DoF tensor u contracted with (V1, dV1) over
// the lower other axis and (V2, dV2) over the upper one:
//   c0 = V1 V2 u, c1 = dV1 V2 u, c2 = V1 dV2 u
template <int K, int D, int KA, typename T>
__device__ __forceinline__ void line_columns(const T* u, const T* V1, const T* dV1, const T* V2, const T* dV2, T* c0,
                                             T* c1, T* c2) {
  constexpr int O1 = KA == 0 ? 1 : 0;
  constexpr int O2 = KA == 2 ? 1 : 2;
  constexpr int SK = ipow(K, KA), S1 = ipow(K, O1), S2 = D == 3 ? ipow(K, O2) : 0;
#pragma unroll
  for (int lk = 0; lk < K; ++lk) {
    // one layer of loads at a time keeps the register footprint at K^2: the
    // empty asm at the end of a layer needs the layer's sums and keeps the
    // next layer's LDS reads behind it
    T a0 = 0, a1 = 0, a2 = 0;
    if constexpr (D == 3) {
#pragma unroll
      for (int b = 0; b < K; ++b) {
        T s = 0, t = 0;
#pragma unroll
        for (int aa = 0; aa < K; ++aa) {
          const T uu = u[lk * SK + aa * S1 + b * S2];
          s += V1[aa] * uu;
          t += dV1[aa] * uu;
        }
        a0 += V2[b] * s;
        a1 += V2[b] * t;
        a2 += dV2[b] * s;
      }
    } else {
#pragma unroll
      for (int aa = 0; aa < K; ++aa) {
        const T uu = u[lk * SK + aa * S1];
        a0 += V1[aa] * uu;
        a1 += dV1[aa] * uu;
      }
    }
    asm volatile("" : "+v"(a0), "+v"(a1), "+v"(a2)::"memory");
    c0[lk] = a0;
    c1[lk] = a1;
    c2[lk] = a2;
  }
}

// the two parts of a line record (layout of LineShape), record r of REC:
// the basis values of the fixed coordinates, and the point sums
template <int K, int D, typename T>
__device__ __forceinline__ void line_record_basis(const T* V1, const T* dV1, const T* V2, const T* dV2, T* REC, int r) {
  using LS = LineShape<K, D>;
  T* R = REC + r * LS::RSP;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    R[LS::V1 + i] = V1[i];
    R[LS::DV1 + i] = dV1[i];
    if constexpr (D == 3) {
      R[LS::V2 + i] = V2[i];
      R[LS::DV2 + i] = dV2[i];
    }
  }
}

template <int K, int D, typename T>
__device__ __forceinline__ void line_record_sums(const T* D0, const T* D1, const T* D2, T* REC, int r) {
  using LS = LineShape<K, D>;
  T* R = REC + r * LS::RSP;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    R[LS::D0 + i] = D0[i];
    R[LS::D1 + i] = D1[i];
    if constexpr (D == 3) R[LS::D2 + i] = D2[i];
  }
}

// Point data of a line, loaded ahead of the arithmetic: the two fixed
// coordinates, and for the first PB points the coordinate along the line,
// the weight (times kappa) and, on interface lines, the normal.  PB per
// degree and line kind, as measured: four points, except two for the cell
// lines at K = 2 (volume lines -10 %: the registers freed give a third
// and fourth wave per SIMD) and K for the cut-face lines at K = 2, 3 (-3 %
// and -4 %); K points at K = 3 cost the volume lines 25 %, and at K >= 5
// gain at most 2 % in one precision while losing in the other.
template <int K>
struct LinePB {
  static constexpr int CELL = K == 2 ? 2 : 4, FACE = K < 4 ? K : 4;
};
template <typename T, int PB>
struct LinePts {
  T t1, t2;
  T tk[PB], wq[PB], nk[PB], n1[PB], n2[PB];
};

// loads of points [pb, pb + PB) of a volume / interface line along cell axis
// ax (runtime) starting at point p0; fixed coordinates when pb == 0
template <int D, typename T, int PB>
__device__ __forceinline__ void line_load_cell(const DevArgs<T>& a, int info, int p0, int pb, LinePts<T, PB>& L) {
  const int n = info & 0xffff;
  const int ax = (info >> 16) & 0xf;
  const bool surf = ((info >> 20) & 0xf) == 1;
  const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
  const T* px = surf ? a.surf_x : a.vol_x;
  const int64_t stride = surf ? a.n_surf : a.n_vol;
  const T* pw = surf ? a.surf_w : a.vol_w;
  const int64_t kbase = surf ? a.seg[4] : a.seg[1];
  if (pb == 0) {
    L.t1 = px[o1 * stride + p0];
    L.t2 = D == 3 ? px[o2 * stride + p0] : T(0);
  }
#pragma unroll
  for (int i = 0; i < PB; ++i) {
    L.tk[i] = 0; L.wq[i] = 0; L.nk[i] = 0; L.n1[i] = 0; L.n2[i] = 0;
    if (pb + i < n) {
      const int64_t q = p0 + pb + i;
      L.tk[i] = px[ax * stride + q];
      L.wq[i] = pw[q];
      if (a.kappa) L.wq[i] *= a.kappa[kbase + q];
      if (surf) {
        L.nk[i] = a.surf_n[ax * stride + q];
        L.n1[i] = a.surf_n[o1 * stride + q];
        if constexpr (D == 3) L.n2[i] = a.surf_n[o2 * stride + q];
      }
    }
  }
}

// one volume or interface line of points along cell axis KA whose first
// point data are in L: evaluate, apply the point flux, integrate along the
// line; writes the line record as record r of REC.  info / p0: the line
// descriptor (count | axis << 16 | kind << 20, first point)
template <int K, int D, int KA, typename T>
__device__ __forceinline__ void line_work_cell(const T* tab, const DevArgs<T>& a, int info, int p0,
                                               LinePts<T, LinePB<K>::CELL>& L,
                                               const T* Uo, T* REC, int r) {
  const T* Xn = tab + TabOff::X(K);
  const T* ID = tab + TabOff::ID(K);
  const int n = info & 0xffff;
  const bool surf = ((info >> 20) & 0xf) == 1;
  T V1[K], dV1[K], V2[K], dV2[K];
  lagrange1d<K>(Xn, ID, L.t1, V1, dV1);
  if constexpr (D == 3) {
    lagrange1d<K>(Xn, ID, L.t2, V2, dV2);
  } else {
#pragma unroll
    for (int i = 0; i < K; ++i) { V2[i] = 1; dV2[i] = 0; }
  }
  T c0[K], c1[K], c2[K];
  line_columns<K, D, KA>(Uo, V1, dV1, V2, dV2, c0, c1, c2);
  // the basis parts of the record go out now, which frees their registers
  // for the point loop
  line_record_basis<K, D>(V1, dV1, V2, dV2, REC, r);
  T D0[K], D1[K], D2[K];
#pragma unroll
  for (int i = 0; i < K; ++i) { D0[i] = 0; D1[i] = 0; D2[i] = 0; }
  for (int pb = 0; pb < n; pb += LinePB<K>::CELL) {
    if (pb > 0) line_load_cell<D>(a, info, p0, pb, L);
#pragma unroll
    for (int i = 0; i < LinePB<K>::CELL; ++i) {
      if (pb + i >= n) break;
      T Z[K], dZ[K];
      lagrange1d<K>(Xn, ID, L.tk[i], Z, dZ);
      T val = 0, gk = 0, g1 = 0, g2 = 0;
#pragma unroll
      for (int ii = 0; ii < K; ++ii) {
        val += Z[ii] * c0[ii];
        gk += dZ[ii] * c0[ii];
        g1 += Z[ii] * c1[ii];
        g2 += Z[ii] * c2[ii];
      }
      const T c = a.hs * L.wq[i];
      T f0, fk, f1, f2;
      if (surf) {
        // Nitsche: tau u v - d_n u v - u d_n v
        const T dn = L.nk[i] * gk + L.n1[i] * g1 + L.n2[i] * g2;
        f0 = c * (a.tau * val - dn);
        fk = -c * val * L.nk[i];
        f1 = -c * val * L.n1[i];
        f2 = -c * val * L.n2[i];
      } else {
        f0 = 0;
        fk = c * gk;
        f1 = c * g1;
        f2 = c * g2;
      }
#pragma unroll
      for (int ii = 0; ii < K; ++ii) {
        D0[ii] += Z[ii] * f0 + dZ[ii] * fk;
        D1[ii] += Z[ii] * f1;
        D2[ii] += Z[ii] * f2;
      }
    }
  }
  line_record_sums<K, D>(D0, D1, D2, REC, r);
}

// Batched line kernels: one wave per batch of cut cells whose lines fit in
// one round (or one cell with several rounds).  The result is added to v.
// Each lane keeps the sums of its DoFs for every entry of the batch in
// registers; the records of a round pass through LDS, and as the lines of
// an entry come ordered by axis, the reduction reads them with fixed index
// patterns.  The grid is persistent: while a wave works on one batch, the
// batch record and the first-round line descriptors of its next batch are
// already in flight, and the point data of a round are loaded together with
// the cell DoFs.
template <int K, int D>
struct BatchShape {
  static constexpr int ND = ipow(K, D);
  static constexpr int NT = kBatchLines;
  static constexpr int NPL = (ND + NT - 1) / NT;  // DoFs per lane
  static constexpr int RP = NT + 1;               // record component pitch
};

// tensor index of the lane's DoFs
template <int K, int D, int NPL>
__device__ __forceinline__ void lane_dofs(int (*dof_i)[3]) {
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int l = min((int)threadIdx.x + kBatchLines * j, ipow(K, D) - 1);
    dof_i[j][0] = l % K;
    dof_i[j][1] = (l / K) % K;
    dof_i[j][2] = D == 3 ? l / (K * K) : 0;
  }
}

// the batch's entries: sums of the lane's DoFs start from v's row for the
// first entry of a cell; at the end the entries of a cell go out once
template <int K, int D, int ME, int NPL, typename T>
__device__ __forceinline__ void batch_acc_init(const T* __restrict__ v, const int* rank, int ne, T (*acc)[NPL]) {
  constexpr int ND = ipow(K, D);
#pragma unroll
  for (int e = 0; e < ME; ++e) {
    const bool first = e < ne && (e == 0 || rank[e - 1] != rank[e]);
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
      const int l = threadIdx.x + kBatchLines * j;
      acc[e][j] = (first && l < ND) ? v[(int64_t)rank[e] * ND + l] : T(0);
    }
  }
}

template <int K, int D, int ME, int NPL, typename T>
__device__ __forceinline__ void batch_acc_store(T* __restrict__ v, const int* rank, int ne, T (*acc)[NPL]) {
  constexpr int ND = ipow(K, D);
#pragma unroll
  for (int e = 0; e < ME; ++e) {
    if (e < ne && (e == 0 || rank[e - 1] != rank[e])) {
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        T s = acc[e][j];
#pragma unroll
        for (int e2 = e + 1; e2 < ME; ++e2)
          if (e2 < ne && rank[e2] == rank[e]) s += acc[e2][j];
        const int l = threadIdx.x + kBatchLines * j;
        if (l < ND) v[(int64_t)rank[e] * ND + l] = s;
      }
    }
  }
}

// the batch record (header and entries, batch_record_ints(ME) ints at a
// fixed stride) and the lane's first-round line descriptor
struct BatchFetch {
  int2 rec;  // record int t (.x), or ints 2t, 2t + 1 for records longer than kBatchLines ints
  int2 hd;
};

template <int ME>
__device__ __forceinline__ BatchFetch batch_fetch(const int32_t* __restrict__ brec, const int32_t* __restrict__ desc,
                                                  int b, int n_batches) {
  constexpr int NR = batch_record_ints(ME);
  static_assert(NR % 2 == 0 && NR <= 2 * kBatchLines, "batch records are fetched as ints or int pairs");
  BatchFetch f{make_int2(0, 0), make_int2(0, 0)};
  if (b < n_batches) {
    const int t = threadIdx.x;
    if constexpr (NR <= kBatchLines) {
      if (t < NR) f.rec.x = brec[(int64_t)b * NR + t];
    } else {
      if (2 * t < NR) f.rec = *reinterpret_cast<const int2*>(brec + (int64_t)b * NR + 2 * t);
    }
    f.hd = *reinterpret_cast<const int2*>(desc + 2 * ((int64_t)b * kBatchLines + t));
  }
  return f;
}

// the fetched record into LDS (rec: batch_record_ints(ME) ints)
template <int ME>
__device__ __forceinline__ void batch_record_store(int* rec, const BatchFetch& f) {
  constexpr int NR = batch_record_ints(ME);
  const int t = threadIdx.x;
  if constexpr (NR <= kBatchLines) {
    if (t < NR) rec[t] = f.rec.x;
  } else {
    if (2 * t < NR) {
      rec[2 * t] = f.rec.x;
      rec[2 * t + 1] = f.rec.y;
    }
  }
}

// line descriptor of in-batch line g >= kBatchLines
__device__ __forceinline__ int2 batch_desc(const int32_t* __restrict__ desc, int n_batches, int ovf, int g) {
  return *reinterpret_cast<const int2*>(desc + 2 * ((int64_t)n_batches * kBatchLines + ovf + g - kBatchLines));
}

// ---- volume and interface lines
// Every entry of a volume batch is one cut cell.  In 3D the records of a
// round are reduced by groups of lanes: lane (ik, tile) of a group owns the
// DoFs (ik, i1, i2) with i1 in its tile of the i1 range and all i2; per
// record it forms P = V1[i1] D0[ik] + dV1[i1] D1[ik] and Q = V1[i1] D2[ik]
// for its i1 and adds V2[i2] P + dV2[i2] Q to its DoFs.  The G groups take
// every G-th record and are added into the cell's LDS row with LDS atomics;
// group g visits its i1 and i2 in an order rotated by g, so that the groups'
// atomic adds of one instruction go to distinct addresses.  The rows are kept
// in double for both precisions: LDS atomic adds of doubles are native and
// cheap on gfx950, those of floats cost several times more (measured), and
// the float operator's lines stay in float up to that last sum.  (2D: one
// lane per DoF.)
template <int K>
struct ReduceShape {
  // i1 tile: at most 32 / K rows, so that a lane holds at most 32 sums; at
  // K = 4 two rows (eight groups of eight lanes, each with more records per
  // round) beat four rows (sixteen groups of four): volume lines -4 % in
  // double, -15 % in float, measured; the other degrees lose with it
  static constexpr int AMAX = K == 4 ? 2 : (K < 32 / K ? K : 32 / K);
  static constexpr int NTL = (K + AMAX - 1) / AMAX;  // tiles
  static constexpr int A = (K + NTL - 1) / NTL;      // rows per tile
  static constexpr int LPG = K * NTL;                // lanes per group
  static constexpr int G = kBatchLines / LPG;        // groups
};

template <int K, int D, typename T>
struct BatchWork {
  static constexpr int ND = BatchShape<K, D>::ND, ME = batch_max_entries(ipow(K, D), false, sizeof(T) == 4),
                       RS = LineShape<K, D>::RS, RP = BatchShape<K, D>::RP;
  T U[ME][ND];
  double OUT[ME][ND];  // the cells' rows of v (double also for T = float)
  T REC[kBatchLines * LineShape<K, D>::RSP];  // the round's records
  int rec[batch_record_ints(ME)];
};

// 2D: acc += the records [lo, hi) of the round, all along axis KA
template <int K, int KA, int NPL, typename T>
__device__ __forceinline__ void reduce_axis_2d(const T* REC, int lo, int hi, const int (*dof_i)[3], T* acc) {
  using LS = LineShape<K, 2>;
  constexpr int O1 = KA == 0 ? 1 : 0;
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int ik = dof_i[j][KA], i1 = dof_i[j][O1];
    T s = 0;
    for (int r = lo; r < hi; ++r) {
      const T* R = REC + r * LS::RSP;
      s += R[LS::V1 + i1] * R[LS::D0 + ik] + R[LS::DV1 + i1] * R[LS::D1 + ik];
    }
    acc[j] += s;
  }
}

// 3D: OUT += the records [lo, hi) of the round, all along axis KA (group
// reduction described above)
template <int K, int KA, typename T>
__device__ __forceinline__ void reduce_axis_3d(const T* REC, int lo, int hi, double* OUT) {
  using LS = LineShape<K, 3>;
  using RS = ReduceShape<K>;
  constexpr int A = RS::A, G = RS::G, LPG = RS::LPG;
  constexpr int O1 = KA == 0 ? 1 : 0;
  constexpr int O2 = KA == 2 ? 1 : 2;
  constexpr int SK = ipow(K, KA), S1 = ipow(K, O1), S2 = ipow(K, O2);
  const int t = threadIdx.x, grp = t / LPG, m = t % LPG, ik = m % K, i1b = (m / K) * A;
  if (grp >= G || lo + grp >= hi) return;
  // rows of the lane's tile (the last tile may be short) and the rotations
  const int na = RS::NTL == 1 ? A : min(A, K - i1b);
  const int rot2 = grp % K, rot1 = RS::NTL == 1 ? (grp / K) % A : 0;
  int o1[A], o2[K];
#pragma unroll
  for (int s1 = 0; s1 < A; ++s1) o1[s1] = i1b + (s1 + rot1 < A ? s1 + rot1 : s1 + rot1 - A);
#pragma unroll
  for (int s2 = 0; s2 < K; ++s2) o2[s2] = s2 + rot2 < K ? s2 + rot2 : s2 + rot2 - K;
  T acc[A][K];
#pragma unroll
  for (int s1 = 0; s1 < A; ++s1)
#pragma unroll
    for (int s2 = 0; s2 < K; ++s2) acc[s1][s2] = 0;
  for (int r = lo + grp; r < hi; r += G) {
    const T* R = REC + r * LS::RSP;
    const T d0 = R[LS::D0 + ik], d1 = R[LS::D1 + ik], d2 = R[LS::D2 + ik];
    T v2[K], w2[K];
#pragma unroll
    for (int s2 = 0; s2 < K; ++s2) {
      v2[s2] = R[LS::V2 + o2[s2]];
      w2[s2] = R[LS::DV2 + o2[s2]];
    }
#pragma unroll
    for (int s1 = 0; s1 < A; ++s1) {
      if (RS::NTL > 1 && s1 >= na) break;
      const T v1 = R[LS::V1 + o1[s1]];
      const T pp = v1 * d0 + R[LS::DV1 + o1[s1]] * d1;
      const T qq = v1 * d2;
#pragma unroll
      for (int s2 = 0; s2 < K; ++s2) {
        acc[s1][s2] += v2[s2] * pp;
        acc[s1][s2] += w2[s2] * qq;
      }
    }
  }
#pragma unroll
  for (int s1 = 0; s1 < A; ++s1) {
    if (RS::NTL > 1 && s1 >= na) break;
    double* row = OUT + ik * SK + o1[s1] * S1;
#pragma unroll
    for (int s2 = 0; s2 < K; ++s2) {
      if constexpr (G == 1) row[o2[s2] * S2] += acc[s1][s2];
      else atomicAdd(row + o2[s2] * S2, (double)acc[s1][s2]);
    }
  }
}

// (K = 5, 6: two waves per SIMD at the price of a few spilled registers is
// faster than one wave without, by 6 and 10 % measured; for K >= 7 the
// spills outweigh it)
template <int K, int D, typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(K == 5 || K == 6 ? 2 : 1))) cut_batch_kernel(DevArgs<T> a, const T* __restrict__ x, T* __restrict__ v,
                                                       const int32_t* __restrict__ brec,
                                                       const int32_t* __restrict__ desc, int n_batches) {
  using BW = BatchWork<K, D, T>;
  constexpr int ND = BW::ND, ME = BW::ME, RS = BW::RS, RP = BW::RP, NT = BatchShape<K, D>::NT,
                NPL = BatchShape<K, D>::NPL, NR = batch_record_ints(ME);
  constexpr int OFS = (1 << kBatchOffsetBits) - 1;
  __shared__ BW W;
  const int t = threadIdx.x;
  const bool do_vol = (a.terms & 1) != 0, do_surf = (a.terms & 4) != 0;
  int dof_i[NPL][3];
  lane_dofs<K, D, NPL>(dof_i);
  BatchFetch nxt = batch_fetch<ME>(brec, desc, blockIdx.x, n_batches);
  for (int b = blockIdx.x; b < n_batches; b += gridDim.x) {
    const BatchFetch cur = nxt;
    batch_record_store<ME>(W.rec, cur);
    sync();
    nxt = batch_fetch<ME>(brec, desc, b + gridDim.x, n_batches);
    const int ne = W.rec[0], total = W.rec[1], ovf = W.rec[2];
    const int* ent = W.rec + 4;
    // point data of the first round, DoFs and rows of v in one round trip
    int2 hd = cur.hd;
    LinePts<T, LinePB<K>::CELL> L;
    if (t < total) line_load_cell<D>(a, hd.y & 0xffffff, hd.x, 0, L);
    // (a loop of fixed trip count: every load is issued before the first
    // LDS store waits for one)
    // (indices clamped into the batch, so that the loads need no guard)
#pragma unroll
    for (int it = 0; it < (ME * ND + NT - 1) / NT; ++it) {
      if (NT * it >= ne * ND) break;  // uniform
      const int idx = min(t + NT * it, ne * ND - 1);
      const int e = idx / ND, l = idx % ND;
      const int64_t ro = (int64_t)ent[4 * e] * ND + l;
      const T xu = x[ro], xv = v[ro];
      W.U[e][l] = xu;
      W.OUT[e][l] = xv;
    }
    sync();
    for (int base = 0; base < total; base += NT) {
      const int g = base + t;
      bool done = false;
      if (g < total) {
        if (base > 0) {
          hd = batch_desc(desc, n_batches, ovf, g);
          line_load_cell<D>(a, hd.y & 0xffffff, hd.x, 0, L);
        }
        const int info = hd.y & 0xffffff, e = hd.y >> 24;
        const int kind = (info >> 20) & 0xf;
        const int ax = (info >> 16) & 0xf;
        const T* Uo = &W.U[0][0] + e * ND;
        if (kind == 0 ? do_vol : do_surf) {
          done = true;
          if (ax == 0) line_work_cell<K, D, 0>(a.tab, a, info, hd.x, L, Uo, W.REC, t);
          else if (ax == 1 || D == 2) line_work_cell<K, D, 1>(a.tab, a, info, hd.x, L, Uo, W.REC, t);
          else if constexpr (D == 3) line_work_cell<K, D, 2>(a.tab, a, info, hd.x, L, Uo, W.REC, t);
        }
      }
      if (g < total && !done) {  // a line of a switched-off term (records past total are not read)
#pragma unroll
        for (int c = 0; c < RS; ++c) W.REC[t * LineShape<K, D>::RSP + c] = 0;
      }
      sync();
      const int r1 = min(total, base + NT);
      for (int e = 0; e < ne; ++e) {
        const int a0 = ent[4 * e + 2] & OFS, a3 = e + 1 < ne ? (ent[4 * (e + 1) + 2] & OFS) : total;
        if (a0 >= r1 || a3 <= base) continue;
        const int a1 = a0 + (ent[4 * e + 1] & 0xffff), a2 = a1 + ((ent[4 * e + 1] >> 16) & 0xffff);
        double* out = &W.OUT[0][0] + e * ND;
        if constexpr (D == 3) {
          reduce_axis_3d<K, 0>(W.REC, max(a0, base) - base, min(a1, r1) - base, out);
          reduce_axis_3d<K, 1>(W.REC, max(a1, base) - base, min(a2, r1) - base, out);
          reduce_axis_3d<K, 2>(W.REC, max(a2, base) - base, min(a3, r1) - base, out);
        } else {
          T acc[NPL];
#pragma unroll
          for (int j = 0; j < NPL; ++j) acc[j] = 0;
          reduce_axis_2d<K, 0, NPL>(W.REC, max(a0, base) - base, min(a1, r1) - base, dof_i, acc);
          reduce_axis_2d<K, 1, NPL>(W.REC, max(a1, base) - base, min(a3, r1) - base, dof_i, acc);
#pragma unroll
          for (int j = 0; j < NPL; ++j)
            if (t + NT * j < ND) out[t + NT * j] += acc[j];
        }
      }
      sync();
    }
    for (int idx = t; idx < ne * ND; idx += NT) {
      const int e = idx / ND, l = idx % ND;
      v[(int64_t)ent[4 * e] * ND + l] = (T)W.OUT[e][l];
    }
  }
}

// ---- cut-face lines
// Each entry is one cut face of a cut cell (slot s = 2 N + side, N the
// normal axis).  Only the traces enter the SIPG flux: in the batch prologue
// the value and the normal derivative of both sides are formed on the face's
// K^(D-1) node grid (in-face axes A < B, the other cell axes; the normal-axis
// contraction with the tabulated end-point values E, E' of either side).  A
// line along A or B then contracts the other in-face axis with the Lagrange
// values of its coordinate (one code path for both), evaluates at its
// points, and leaves the record [VF | D0 | DN] (3D) or [D0 | DN] (2D): the
// test-function coefficient of DoF (i_line, i_N, i_F) is
// VF[i_F] (E[i_N] D0[i_line] + E'[i_N] DN[i_line]) with E the own side's
// end-point values.  Sums are kept per cell (up to batch_max_cells cells).
template <int K, int D>
struct FaceShape {
  static constexpr int NF = ipow(K, D - 1);
  static constexpr int RS = D == 3 ? 3 * K : 2 * K;
  static constexpr int VF = 0, D0 = D == 3 ? K : 0, DN = D0 + K;
};

template <int K, int D, typename T>
struct FaceWork {
  static constexpr int NF = FaceShape<K, D>::NF, ME = batch_max_entries(ipow(K, D), true),
                       RS = FaceShape<K, D>::RS, RP = BatchShape<K, D>::RP;
  T tab[TabOff::lds_size(K)];
  T TR[ME][4][NF];  // own value, own normal derivative, neighbour value, neighbour normal derivative
  T REC[RS * RP];
  int rec[batch_record_ints(ME)];
};

// point data of a cut-face line: the coordinate along the other in-face
// axis, and for points [pb, pb + PB) the coordinate along the line and the
// weight (times kappa)
template <int D, typename T, int PB>
__device__ __forceinline__ void line_load_face(const DevArgs<T>& a, int info, int p0, int pb, LinePts<T, PB>& L) {
  const int n = info & 0xffff;
  const int fk = (info >> 16) & 0xf;  // in-face axis of the line
  const int64_t stride = a.n_fcut;
  if (pb == 0) L.t1 = D == 3 ? a.fcut_x[(1 - fk) * stride + p0] : T(0);
#pragma unroll
  for (int i = 0; i < PB; ++i) {
    L.tk[i] = 0; L.wq[i] = 0;
    if (pb + i < n) {
      const int64_t q = p0 + pb + i;
      L.tk[i] = a.fcut_x[fk * stride + q];
      L.wq[i] = a.fcut_w[q];
      if (a.kappa) L.wq[i] *= a.kappa[a.seg[3] + q];
    }
  }
}

// one cut-face line, along in-face axis A (alongB false) or B; TR: the
// entry's traces
template <int K, int D, int RP, typename T>
__device__ __forceinline__ void line_work_face(const T* tab, const DevArgs<T>& a, int info, int p0, int slot,
                                               LinePts<T, LinePB<K>::FACE>& L, const T (*TR)[FaceShape<K, D>::NF], T* REC,
                                               int r) {
  using FS = FaceShape<K, D>;
  const T* Xn = tab + TabOff::X(K);
  const T* ID = tab + TabOff::ID(K);
  const int n = info & 0xffff;
  const bool alongB = ((info >> 16) & 0xf) == 1;
  const T sigma = (slot & 1) ? T(1) : T(-1);
  T F[K], dF[K];
  if constexpr (D == 3) {
    lagrange1d<K>(Xn, ID, L.t1, F, dF);
  } else {
#pragma unroll
    for (int i = 0; i < K; ++i) F[i] = 1;
  }
  // columns along the line: value and normal derivative, own and neighbour
  T c0[K], cn[K], m0[K], mn[K];
#pragma unroll
  for (int lk = 0; lk < K; ++lk) {
    T a0 = 0, a1 = 0, b0 = 0, b1 = 0;
#pragma unroll
    for (int f = 0; f < (D == 3 ? K : 1); ++f) {
      // along A the line index is the A index (stride K), along B the B index
      const int o = D == 3 ? (alongB ? lk + f * K : lk * K + f) : lk;
      a0 += F[f] * TR[0][o];
      a1 += F[f] * TR[1][o];
      b0 += F[f] * TR[2][o];
      b1 += F[f] * TR[3][o];
    }
    c0[lk] = a0;
    cn[lk] = a1;
    m0[lk] = b0;
    mn[lk] = b1;
  }
  T D0[K], DN[K];
#pragma unroll
  for (int i = 0; i < K; ++i) { D0[i] = 0; DN[i] = 0; }
  for (int pb = 0; pb < n; pb += LinePB<K>::FACE) {
    if (pb > 0) line_load_face<D>(a, info, p0, pb, L);
#pragma unroll
    for (int i = 0; i < LinePB<K>::FACE; ++i) {
      if (pb + i >= n) break;
      T Z[K], dZ[K];
      lagrange1d<K>(Xn, ID, L.tk[i], Z, dZ);
      T val = 0, go = 0, vn = 0, gn = 0;
#pragma unroll
      for (int ii = 0; ii < K; ++ii) {
        val += Z[ii] * c0[ii];
        go += Z[ii] * cn[ii];
        vn += Z[ii] * m0[ii];
        gn += Z[ii] * mn[ii];
      }
      // SIPG: jump sigma (u_own - u_nbr), average of the normal derivative
      const T c = a.hs * L.wq[i];
      const T J = sigma * (val - vn);
      const T A = T(0.5) * (go + gn);
      const T f0 = c * sigma * (a.gamma * J - A);
      const T fn = T(-0.5) * c * J;
#pragma unroll
      for (int ii = 0; ii < K; ++ii) {
        D0[ii] += Z[ii] * f0;
        DN[ii] += Z[ii] * fn;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < K; ++i) {
    if constexpr (D == 3) REC[(FS::VF + i) * RP + r] = F[i];
    REC[(FS::D0 + i) * RP + r] = D0[i];
    REC[(FS::DN + i) * RP + r] = DN[i];
  }
}

// (double, K >= 7: two waves per SIMD with a few spilled registers beat one
// wave, 18 % at K = 7 measured; float, K = 4: five waves instead of four,
// 6 % measured; K = 2: with the batches of up to 6 cells four waves in
// double, six in float, 7 % and 4 % measured; K = 3: four and six, 9 % and
// 5 % measured; float, K = 5: four, 3 % measured)
template <int K, int D, typename T>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 && K >= 7 ? 2 : (sizeof(T) == 4 && (K == 4 || K == 5) ? (K == 4 ? 5 : 4) : (K <= 3 ? (sizeof(T) == 8 ? 4 : 6) : 1)))))
cut_face_kernel(DevArgs<T> a, const T* __restrict__ x, T* __restrict__ v,
                                                      const int32_t* __restrict__ brec,
                                                      const int32_t* __restrict__ desc, int n_batches) {
  using FW = FaceWork<K, D, T>;
  using FS = FaceShape<K, D>;
  constexpr int ND = BatchShape<K, D>::ND, ME = FW::ME, RS = FW::RS, RP = FW::RP, NT = BatchShape<K, D>::NT,
                NPL = BatchShape<K, D>::NPL, NF = FS::NF, NR = batch_record_ints(ME),
                MC = batch_max_cells(ipow(K, D), true);
  constexpr int OFS = (1 << kBatchOffsetBits) - 1;
  __shared__ FW W;
  const int t = threadIdx.x;
  for (int i = t; i < TabOff::lds_size(K); i += NT) W.tab[i] = a.tab[i];
  int dof_i[NPL][3];
  lane_dofs<K, D, NPL>(dof_i);
  BatchFetch nxt = batch_fetch<ME>(brec, desc, blockIdx.x, n_batches);
  for (int b = blockIdx.x; b < n_batches; b += gridDim.x) {
    const BatchFetch cur = nxt;
    batch_record_store<ME>(W.rec, cur);
    sync();
    nxt = batch_fetch<ME>(brec, desc, b + gridDim.x, n_batches);
    const int ne = W.rec[0], total = W.rec[1], ovf = W.rec[2];
    const int* ent = W.rec + 4;
    int2 hd = cur.hd;
    LinePts<T, LinePB<K>::FACE> L;
    if (t < total) line_load_face<D>(a, hd.y & 0xffffff, hd.x, 0, L);
    // traces of cell and neighbour on the face node grid (A, B); a loop of
    // fixed trip count, so that all loads are issued before the first wait
#pragma unroll
    for (int it = 0; it < (ME * NF + NT - 1) / NT; ++it) {
      const int idx = min(t + NT * it, ne * NF - 1);  // clamped: unguarded loads
      const int e = idx / NF, o = idx % NF;
      const int sl = ent[4 * e + 2] >> kBatchOffsetBits, N = sl >> 1;
      const int ia = o / (D == 3 ? K : 1), ib = D == 3 ? o % K : 0;
      // physical stride of the normal axis and offset of the in-face node
      int sN, off;
      if constexpr (D == 3) {
        sN = N == 0 ? 1 : (N == 1 ? K : K * K);
        off = N == 0 ? ia * K + ib * K * K : (N == 1 ? ia + ib * K * K : ia + ib * K);
      } else {
        sN = N == 0 ? 1 : K;
        off = N == 0 ? ia * K : ia;
      }
      const T* Eo = W.tab + ((sl & 1) ? TabOff::E1(K) : TabOff::E0(K));
      const T* En = W.tab + ((sl & 1) ? TabOff::E0(K) : TabOff::E1(K));
      const T* uo = x + (int64_t)ent[4 * e] * ND + off;
      const T* un = x + (int64_t)ent[4 * e + 3] * ND + off;
      T o0 = 0, o1 = 0, n0 = 0, n1 = 0;
#pragma unroll
      for (int nn = 0; nn < K; ++nn) {
        const T a0 = uo[nn * sN], b0 = un[nn * sN];
        o0 += Eo[nn] * a0;
        o1 += Eo[K + nn] * a0;
        n0 += En[nn] * b0;
        n1 += En[K + nn] * b0;
      }
      W.TR[e][0][o] = o0;
      W.TR[e][1][o] = o1;
      W.TR[e][2][o] = n0;
      W.TR[e][3][o] = n1;
    }
    // per-cell sums of the lane's DoFs, starting from v's rows
    int crank[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) crank[c] = -1;
    {
      int c = -1, prev = -1;
      for (int e = 0; e < ne; ++e) {
        const int r = ent[4 * e];
        if (r != prev) {
          ++c;
          prev = r;
#pragma unroll
          for (int cc = 0; cc < MC; ++cc)
            if (cc == c) crank[cc] = r;
        }
      }
    }
    T acc[MC][NPL];
#pragma unroll
    for (int c = 0; c < MC; ++c)
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        const int l = t + NT * j;
        acc[c][j] = (crank[c] >= 0 && l < ND) ? v[(int64_t)crank[c] * ND + l] : T(0);
      }
    sync();
    for (int base = 0; base < total; base += NT) {
      const int g = base + t;
      if (g < total) {
        if (base > 0) {
          hd = batch_desc(desc, n_batches, ovf, g);
          line_load_face<D>(a, hd.y & 0xffffff, hd.x, 0, L);
        }
        const int info = hd.y & 0xffffff, e = hd.y >> 24;
        const int slot = ent[4 * e + 2] >> kBatchOffsetBits;
        line_work_face<K, D, RP>(a.tab, a, info, hd.x, slot, L, W.TR[e], W.REC, t);
      }  // (records past total are not read)
      sync();
      const int r1 = min(total, base + NT);
      // per entry, the test coefficients of its lines in this round on the
      // face-node grid f = iA + K iB: P0 (value) and P1 (normal derivative),
      // P0[f] = sum over lines along A of VF[iB] D0[iA] + along B of VF[iA]
      // D0[iB] (P1 with DN); lane (slot, f), SL entries per pass
      constexpr int SL = NT / NF, NPS = (ME + SL - 1) / SL;
      static_assert(2 * ME * NF <= RS * RP, "entry matrices must fit in the record area");
      T p0[NPS], p1[NPS];
      {
        const int sl = t / NF, f = t % NF, fa = f % K, fb = D == 3 ? f / K : 0;
#pragma unroll
        for (int ps = 0; ps < NPS; ++ps) {
          p0[ps] = 0;
          p1[ps] = 0;
          const int e = ps * SL + sl;
          if (sl >= SL || e >= ne) continue;
          const int lo0 = ent[4 * e + 2] & OFS;
          const int hi1 = e + 1 < ne ? (ent[4 * (e + 1) + 2] & OFS) : total;
          const int nA = ent[4 * e + 1] & 0xffff;
#pragma unroll
          for (int grp = 0; grp < (D == 3 ? 2 : 1); ++grp) {
            const int lo = grp == 0 ? lo0 : lo0 + nA;
            const int hi = grp == 0 ? lo0 + nA : hi1;
            const int rlo = max(lo, base) - base, rhi = min(hi, r1) - base;
            const int il = grp == 0 ? fa : fb, iF = grp == 0 ? fb : fa;
            const T* Rv = W.REC + (FS::VF + iF) * RP;
            const T* R0 = W.REC + (FS::D0 + il) * RP;
            const T* Rn = W.REC + (FS::DN + il) * RP;
            for (int rr = rlo; rr < rhi; ++rr) {
              const T vf = D == 3 ? Rv[rr] : T(1);
              p0[ps] += vf * R0[rr];
              p1[ps] += vf * Rn[rr];
            }
          }
        }
      }
      sync();  // the records are read: the matrices go into their place
      T* PM = W.REC;  // [entry][2][NF]
      {
        const int sl = t / NF, f = t % NF;
#pragma unroll
        for (int ps = 0; ps < NPS; ++ps) {
          const int e = ps * SL + sl;
          if (sl < SL && e < ne) {
            PM[(2 * e) * NF + f] = p0[ps];
            PM[(2 * e + 1) * NF + f] = p1[ps];
          }
        }
      }
      sync();
      // each lane adds E[iN] P0[f] + E'[iN] P1[f] to its DoFs (iN, iA, iB)
      int c = -1, prev = -1;
      for (int e = 0; e < ne; ++e) {
        const int rank = ent[4 * e];
        if (rank != prev) {
          ++c;
          prev = rank;
        }
        const int lo0 = ent[4 * e + 2] & OFS;
        const int hi1 = e + 1 < ne ? (ent[4 * (e + 1) + 2] & OFS) : total;
        if (lo0 >= r1 || hi1 <= base) continue;
        const int sl = ent[4 * e + 2] >> kBatchOffsetBits, N = sl >> 1;
        const int A = N == 0 ? 1 : 0, B = N == 2 ? 1 : 2;
        const T* E = W.tab + ((sl & 1) ? TabOff::E1(K) : TabOff::E0(K));
        const T* P0 = PM + (2 * e) * NF;
        const T* P1 = P0 + NF;
        T s[NPL];
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
          auto pick = [&](int ax) { return ax == 0 ? dof_i[j][0] : (ax == 1 ? dof_i[j][1] : dof_i[j][2]); };
          const int iN = pick(N), f = pick(A) + (D == 3 ? K * pick(B) : 0);
          s[j] = E[iN] * P0[f] + E[K + iN] * P1[f];
        }
#pragma unroll
        for (int cc = 0; cc < MC; ++cc)
          if (cc == c)
#pragma unroll
            for (int j = 0; j < NPL; ++j) acc[cc][j] += s[j];
      }
      sync();
    }
#pragma unroll
    for (int c = 0; c < MC; ++c)
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        const int l = t + NT * j;
        if (crank[c] >= 0 && l < ND) v[(int64_t)crank[c] * ND + l] = acc[c][j];
      }
  }
}


// ------------------------------------------------ dL/dkappa, kappa = 1 path
// dkappa_q = a_q(w, u): the kappa-weighted integrand at quadrature point q
// evaluated with both arguments (volume: grad w . grad u; SIPG face:
// -{d_n w}[u] - [w]{d_n u} + gamma [w][u]; interface: -d_n w u - w d_n u +
// tau w u), times the point's weight and h^(d-2).

// inside cells: reference gradients of w and u at the k^d Gauss points by
// sum factorisation (one lane per 1D line, as in the Kronecker kernel)
template <int K, int D, typename T>
struct DkWork {
  // K = 3, 4: cell tensors in the skewed, padded layout of the Kronecker
  // kernel (their plain layout had 17 bank conflicts per LDS instruction at
  // K = 4); other K: the plain layout (K = 2: the padding would double the
  // LDS of 16 cells per wave; K >= 5: the skew measured slower)
  static constexpr bool SKEW = K == 3 || K == 4;
  static constexpr int NDP = SKEW ? KronLayout<K, D>::NDP : KronLayout<K, D>::ND, C = KronShape<K, D>::C;
  T A[2][C][NDP];
  T B[2][C][NDP];
  T E[2][C][NDP];
};

template <int K, int D, typename T>
__global__ void __launch_bounds__(64) inside_dk_kernel(DevArgs<T> a, const T* __restrict__ w, const T* __restrict__ u,
                                                       T* __restrict__ dk) {
  constexpr int ND = KronShape<K, D>::ND, NL = KronShape<K, D>::NL, C = KronShape<K, D>::C;
  __shared__ DkWork<K, D, T> W;
  const T* __restrict__ tab = a.tab;
  const T* S = tab + TabOff::S(K);
  const T* DS = tab + TabOff::DS(K);
  const T* Wt = tab + TabOff::W(K);
  const int lane = threadIdx.x;
  const int c = lane / NL, l = lane % NL;
  const bool active = c < C;
  const int cc = active ? c : 0;
  const bool vol_on = (a.terms & 1) != 0;  // the term mask: switched-off terms give 0
  for (int c0 = xcd_block() * C; c0 < a.n_inside; c0 += gridDim.x * C) {
    const int ci = c0 + c;
    const bool valid = active && ci < a.n_inside;
    const int r = valid ? a.inside[ci] : 0;
    const int bx = line_base<K, D, 0>(l), by = line_base<K, D, 1>(l);
    const int bz = D == 3 ? line_base<K, D, 2>(l) : 0;
    int px[K], py[K], pz[K];
    if constexpr (DkWork<K, D, T>::SKEW) {
      KronLayout<K, D>::template line<0>(l, px);
      KronLayout<K, D>::template line<1>(l, py);
      if constexpr (D == 3) KronLayout<K, D>::template line<2>(l, pz);
    } else {
#pragma unroll
      for (int q = 0; q < K; ++q) {
        px[q] = bx + q * line_stride<K, D, 0>();
        py[q] = by + q * line_stride<K, D, 1>();
        pz[q] = D == 3 ? bz + q * line_stride<K, D, 2>() : 0;
      }
    }
    T t0[K], t1[K], t2[K];
    if (valid) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        glb_line_load<K, D, 0>((f ? u : w) + (int64_t)r * ND, bx, t0);
        line_mat<K>(S, t0, t1);
        line_mat<K>(DS, t0, t2);
        kl_store<K>(W.A[f][cc], px, t1);
        kl_store<K>(W.B[f][cc], px, t2);
      }
    }
    sync();
    if constexpr (D == 3) {
      if (valid) {
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          kl_load<K>(W.A[f][cc], py, t0);
          line_mat<K>(S, t0, t1);
          line_mat<K>(DS, t0, t2);
          kl_store<K>(W.A[f][cc], py, t1);  // S S u
          kl_store<K>(W.E[f][cc], py, t2);  // DS_y S_x u
          kl_load<K>(W.B[f][cc], py, t0);
          line_mat<K>(S, t0, t1);
          kl_store<K>(W.B[f][cc], py, t1);  // S_y DS_x u
        }
      }
      sync();
      if (valid) {
        T g[2][3][K];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          kl_load<K>(W.A[f][cc], pz, t0);
          line_mat<K>(DS, t0, g[f][2]);
          kl_load<K>(W.E[f][cc], pz, t0);
          line_mat<K>(S, t0, g[f][1]);
          kl_load<K>(W.B[f][cc], pz, t0);
          line_mat<K>(S, t0, g[f][0]);
        }
        const int qx = bz % K, qy = bz / K;
        T* out = dk + a.seg[0] + (int64_t)ci * ND;
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const T wq = a.hs * Wt[qx] * Wt[qy] * Wt[q];
          out[bz + q * K * K] = vol_on ? wq * (g[0][0][q] * g[1][0][q] + g[0][1][q] * g[1][1][q] + g[0][2][q] * g[1][2][q]) : T(0);
        }
      }
    } else {
      if (valid) {
        T g[2][2][K];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          kl_load<K>(W.A[f][cc], py, t0);
          line_mat<K>(DS, t0, g[f][1]);
          kl_load<K>(W.B[f][cc], py, t0);
          line_mat<K>(S, t0, g[f][0]);
        }
        const int qx = by;
        T* out = dk + a.seg[0] + (int64_t)ci * ND;
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const T wq = a.hs * Wt[qx] * Wt[q];
          out[by + q * K] = vol_on ? wq * (g[0][0][q] * g[1][0][q] + g[0][1][q] * g[1][1][q]) : T(0);
        }
      }
    }
    sync();
  }
}

// Structured SIPG faces of dL/dkappa, by groups of C consecutive active
// cells (rank order): each cell takes its structured upper faces (slots
// 2 ax + 1).  The group's DoFs of w and u are staged in LDS once and serve
// the faces along every axis and, where a face's upper cell is in the group
// (mostly the x neighbour), its other side too; other neighbours' lines
// normal to the face come from memory.  Lane (c, f): cell c, face node f.
// Per face: value jumps and normal-derivative averages of w and u on the
// Gauss-Lobatto face nodes (the value trace is the end-point DoF of the
// nodal basis), interpolated to the face Gauss points, and
//   dk_q = w_q h^(d-2) (-{d_n w}[u] - [w]{d_n u} + gamma [w][u]).
// The faces of a cell are consecutive in kappa order, by axis, from
// sf_first[cell].
template <int K, int D>
struct FaceDkShape {
  static constexpr int NF = ipow(K, D - 1);
  static constexpr int C = 64 / NF;
};

template <int K, int D, typename T>
__global__ void __launch_bounds__(64) face_dk_kernel(DevArgs<T> a, const T* __restrict__ w, const T* __restrict__ u,
                                                     T* __restrict__ dk) {
  constexpr int ND = ipow(K, D), NF = FaceDkShape<K, D>::NF, C = FaceDkShape<K, D>::C;
  __shared__ T X[C][2][ND];
  __shared__ T F[C][4][NF];
  const T* __restrict__ tab = a.tab;
  const T* S = tab + TabOff::S(K);
  const T* Wt = tab + TabOff::W(K);
  const T* E0 = tab + TabOff::E0(K);
  const T* E1 = tab + TabOff::E1(K);
  const int lane = threadIdx.x;
  const int c = lane / NF, f = lane % NF;
  const bool active = c < C;
  const int cc = active ? c : 0;
  const bool sipg = (a.terms & 2) != 0;
  for (int g0 = xcd_block() * C; g0 < a.n_active; g0 += gridDim.x * C) {
    const int ci = g0 + c;
    const bool valid = active && ci < a.n_active;
    int4 k0 = make_int4(0, 0, 0, 0), k1 = make_int4(-1, -1, -1, -1);
    int first = 0;
    if (valid) {
      k0 = reinterpret_cast<const int4*>(a.kinfo_all)[2 * ci];
      k1 = reinterpret_cast<const int4*>(a.kinfo_all)[2 * ci + 1];
      first = a.sf_first[ci];
      // the cell's DoFs of w and u: lane f loads DoFs [f K, f K + K)
      // (without the SIPG term the face points get zeros: nothing to load)
      if (sipg) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
          X[cc][0][f * K + q] = w[(int64_t)ci * ND + f * K + q];
          X[cc][1][f * K + q] = u[(int64_t)ci * ND + f * K + q];
        }
      }
    }
    const int fl = k0.y;
    const int up[3] = {k0.w, k1.y, k1.w};  // upper neighbours (slots 1, 3, 5)
    sync();
    int nf_before = 0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      const bool has = valid && ((fl >> (kFlagStr + 2 * ax + 1)) & 1);
      if (has && sipg) {
        const int nr = up[ax];
        const bool in_group = nr >= g0 && nr < g0 + C;
#pragma unroll
        for (int fld = 0; fld < 2; ++fld) {
          T xm[K], xp[K];
#pragma unroll
          for (int l = 0; l < K; ++l) xm[l] = X[cc][fld][cell_index<K, D>(ax, f, l)];
          if (in_group) {
#pragma unroll
            for (int l = 0; l < K; ++l) xp[l] = X[nr - g0][fld][cell_index<K, D>(ax, f, l)];
          } else {
            const T* src = fld ? u : w;
#pragma unroll
            for (int l = 0; l < K; ++l) xp[l] = src[(int64_t)nr * ND + cell_index<K, D>(ax, f, l)];
          }
          T dm = 0, dp = 0;
#pragma unroll
          for (int l = 0; l < K; ++l) {
            dm += E1[K + l] * xm[l];
            dp += E0[K + l] * xp[l];
          }
          F[cc][2 * fld][f] = xm[K - 1] - xp[0];
          F[cc][2 * fld + 1][f] = T(0.5) * (dm + dp);
        }
      }
      sync();
      if (has) {
        T r = 0;
        if (sipg) {
          T g[4];
          const int q0 = f % K, q1 = f / K;
#pragma unroll
          for (int k2 = 0; k2 < 4; ++k2) {
            T s2 = 0;
            if constexpr (D == 3) {
#pragma unroll
              for (int b = 0; b < K; ++b) {
                T s1 = 0;
#pragma unroll
                for (int a2 = 0; a2 < K; ++a2) s1 += S[q0 * K + a2] * F[cc][k2][a2 + K * b];
                s2 += S[q1 * K + b] * s1;
              }
            } else {
#pragma unroll
              for (int a2 = 0; a2 < K; ++a2) s2 += S[q0 * K + a2] * F[cc][k2][a2];
            }
            g[k2] = s2;
          }
          const T wq = a.hs * (D == 3 ? Wt[q0] * Wt[q1] : Wt[q0]);
          r = wq * (-g[1] * g[2] - g[0] * g[3] + a.gamma * g[0] * g[2]);
        }
        dk[a.seg[2] + (int64_t)(first + nf_before) * NF + f] = r;
        ++nf_before;
      }
      sync();
    }
  }
}

// cut cells: the point lines of the volume and interface rules, with both
// arguments evaluated at every point
template <int K, int D, int KA, typename T>
__device__ __forceinline__ void line_dk(const T* tab, const DevArgs<T>& a, int info, int p0, const T* Wo,
                                        const T* Yo, T* __restrict__ dk) {
  constexpr int O1 = KA == 0 ? 1 : 0;
  constexpr int O2 = KA == 2 ? 1 : 2;
  const T* Xn = tab + TabOff::X(K);
  const T* ID = tab + TabOff::ID(K);
  const int n = info & 0xffff;
  const bool surf = ((info >> 20) & 0xf) == 1;
  const T* px = surf ? a.surf_x : a.vol_x;
  const int64_t stride = surf ? a.n_surf : a.n_vol;
  const T* pw = surf ? a.surf_w : a.vol_w;
  const int64_t kbase = surf ? a.seg[4] : a.seg[1];
  // the term mask: points of a switched-off term get 0
  const bool on = (a.terms & (surf ? 4 : 1)) != 0;
  T V1[K], dV1[K], V2[K], dV2[K];
  lagrange1d<K>(Xn, ID, px[O1 * stride + p0], V1, dV1);
  if constexpr (D == 3) {
    lagrange1d<K>(Xn, ID, px[O2 * stride + p0], V2, dV2);
  } else {
#pragma unroll
    for (int i = 0; i < K; ++i) { V2[i] = 1; dV2[i] = 0; }
  }
  // columns of w and u: [value, d_o1, d_o2][K]
  T cw[3][K], cu[3][K];
  line_columns<K, D, KA>(Wo, V1, dV1, V2, dV2, cw[0], cw[1], cw[2]);
  line_columns<K, D, KA>(Yo, V1, dV1, V2, dV2, cu[0], cu[1], cu[2]);
  for (int pi = 0; pi < n; ++pi) {
    const int64_t q = p0 + pi;
    T Z[K], dZ[K];
    lagrange1d<K>(Xn, ID, px[KA * stride + q], Z, dZ);
    T ew[4] = {0, 0, 0, 0}, eu[4] = {0, 0, 0, 0};  // value, d_k, d_o1, d_o2
#pragma unroll
    for (int i = 0; i < K; ++i) {
      ew[0] += Z[i] * cw[0][i];
      ew[1] += dZ[i] * cw[0][i];
      ew[2] += Z[i] * cw[1][i];
      ew[3] += Z[i] * cw[2][i];
      eu[0] += Z[i] * cu[0][i];
      eu[1] += dZ[i] * cu[0][i];
      eu[2] += Z[i] * cu[1][i];
      eu[3] += Z[i] * cu[2][i];
    }
    const T c = a.hs * pw[q];
    T val;
    if (surf) {
      const T nk = a.surf_n[KA * stride + q], n1v = a.surf_n[O1 * stride + q];
      const T n2v = D == 3 ? a.surf_n[O2 * stride + q] : T(0);
      const T dnw = nk * ew[1] + n1v * ew[2] + n2v * ew[3];
      const T dnu = nk * eu[1] + n1v * eu[2] + n2v * eu[3];
      val = -dnw * eu[0] - ew[0] * dnu + a.tau * ew[0] * eu[0];
    } else {
      val = ew[1] * eu[1] + ew[2] * eu[2] + ew[3] * eu[3];
    }
    dk[kbase + q] = on ? c * val : T(0);
  }
}

template <int K, int D, typename T>
struct DkBatchWork {
  static constexpr int ND = BatchShape<K, D>::ND, ME = batch_max_entries(ipow(K, D), false, sizeof(T) == 4);
  T tab[TabOff::lds_size(K)];
  T Wo[ME][ND];
  T Yo[ME][ND];
  int rec[batch_record_ints(ME)];
};

template <int K, int D, typename T>
__global__ void __launch_bounds__(64) cut_dk_kernel(DevArgs<T> a, const T* __restrict__ w, const T* __restrict__ u,
                                                    T* __restrict__ dk, const int32_t* __restrict__ brec,
                                                    const int32_t* __restrict__ desc, int n_batches) {
  using BW = DkBatchWork<K, D, T>;
  constexpr int ND = BW::ND, ME = BW::ME, NT = 64, NR = batch_record_ints(ME);
  __shared__ BW W;
  for (int i = threadIdx.x; i < TabOff::lds_size(K); i += NT) W.tab[i] = a.tab[i];
  const int t = threadIdx.x;
  for (int b = blockIdx.x; b < n_batches; b += gridDim.x) {
    for (int i = t; i < NR; i += NT) W.rec[i] = brec[(int64_t)b * NR + i];
    sync();
    const int ne = W.rec[0], total = W.rec[1], ovf = W.rec[2];
    const int* ent = W.rec + 4;
    for (int idx = t; idx < ne * ND; idx += NT) {
      const int e = idx / ND, l = idx % ND;
      const int64_t ro = (int64_t)ent[4 * e] * ND + l;
      W.Wo[e][l] = w[ro];
      W.Yo[e][l] = u[ro];
    }
    sync();
    for (int g = t; g < total; g += NT) {
      const int2 hd = g < kBatchLines ? *reinterpret_cast<const int2*>(desc + 2 * ((int64_t)b * kBatchLines + g))
                                      : batch_desc(desc, n_batches, ovf, g);
      const int info = hd.y & 0xffffff, e = hd.y >> 24;
      const int ax = (info >> 16) & 0xf;
      if (ax == 0) line_dk<K, D, 0>(W.tab, a, info, hd.x, W.Wo[e], W.Yo[e], dk);
      else if (ax == 1 || D == 2) line_dk<K, D, 1>(W.tab, a, info, hd.x, W.Wo[e], W.Yo[e], dk);
      else if constexpr (D == 3) line_dk<K, D, 2>(W.tab, a, info, hd.x, W.Wo[e], W.Yo[e], dk);
    }
    sync();
  }
}

// cut faces, dL/dkappa: per face entry whose cell is the face's lower cell
// (each point written once), the value and normal-derivative traces of w and
// u on both sides on the face-node grid (as in cut_face_kernel), then per
// line the in-face contraction, per point the SIPG integrand of (w, u)
template <int K, int D, typename T>
struct FaceDkWork {
  static constexpr int NF = ipow(K, D - 1), ME = batch_max_entries(ipow(K, D), true);
  T TR[ME][8][NF];  // w: own value, own d_n, nbr value, nbr d_n; then u
  int rec[batch_record_ints(ME)];
};

// (double, K = 8: two waves per SIMD at the price of a few spilled registers)
template <int K, int D, typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 && K == 8 ? 2 : 1)))
cut_face_dk_kernel(DevArgs<T> a, const T* __restrict__ w,
                                                         const T* __restrict__ u, T* __restrict__ dk,
                                                         const int32_t* __restrict__ brec,
                                                         const int32_t* __restrict__ desc, int n_batches) {
  using FW = FaceDkWork<K, D, T>;
  constexpr int ND = ipow(K, D), NF = FW::NF, ME = FW::ME, NT = kBatchLines, NR = batch_record_ints(ME);
  __shared__ FW W;
  const T* tab = a.tab;
  const T* Xn = tab + TabOff::X(K);
  const T* ID = tab + TabOff::ID(K);
  const int t = threadIdx.x;
  for (int b = blockIdx.x; b < n_batches; b += gridDim.x) {
    for (int i = t; i < NR; i += NT) W.rec[i] = brec[(int64_t)b * NR + i];
    sync();
    const int ne = W.rec[0], total = W.rec[1], ovf = W.rec[2];
    const int* ent = W.rec + 4;
#pragma unroll
    for (int it = 0; it < (ME * NF + NT - 1) / NT; ++it) {
      if (NT * it >= ne * NF) break;  // uniform
      const int idx = min(t + NT * it, ne * NF - 1);
      const int e = idx / NF, o = idx % NF;
      const int sl = ent[4 * e + 2] >> kBatchOffsetBits, N = sl >> 1;
      if ((sl & 1) == 0) continue;  // the upper cell of the face: no points to write
      const int ia = o / (D == 3 ? K : 1), ib = D == 3 ? o % K : 0;
      int sN, off;
      if constexpr (D == 3) {
        sN = N == 0 ? 1 : (N == 1 ? K : K * K);
        off = N == 0 ? ia * K + ib * K * K : (N == 1 ? ia + ib * K * K : ia + ib * K);
      } else {
        sN = N == 0 ? 1 : K;
        off = N == 0 ? ia * K : ia;
      }
      const T* Eo = tab + ((sl & 1) ? TabOff::E1(K) : TabOff::E0(K));
      const T* En = tab + ((sl & 1) ? TabOff::E0(K) : TabOff::E1(K));
      const int64_t ro = (int64_t)ent[4 * e] * ND + off, rn = (int64_t)ent[4 * e + 3] * ND + off;
#pragma unroll
      for (int fld = 0; fld < 2; ++fld) {
        const T* src = fld ? u : w;
        T o0 = 0, o1 = 0, n0 = 0, n1 = 0;
#pragma unroll
        for (int nn = 0; nn < K; ++nn) {
          const T a0 = src[ro + nn * sN], b0 = src[rn + nn * sN];
          o0 += Eo[nn] * a0;
          o1 += Eo[K + nn] * a0;
          n0 += En[nn] * b0;
          n1 += En[K + nn] * b0;
        }
        W.TR[e][4 * fld][o] = o0;
        W.TR[e][4 * fld + 1][o] = o1;
        W.TR[e][4 * fld + 2][o] = n0;
        W.TR[e][4 * fld + 3][o] = n1;
      }
    }
    sync();
    for (int g = t; g < total; g += NT) {
      const int2 hd = g < kBatchLines ? *reinterpret_cast<const int2*>(desc + 2 * ((int64_t)b * kBatchLines + g))
                                      : batch_desc(desc, n_batches, ovf, g);
      const int info = hd.y & 0xffffff, e = hd.y >> 24;
      const int slot = ent[4 * e + 2] >> kBatchOffsetBits;
      if ((slot & 1) == 0) continue;  // the face's upper cell: its lower cell writes
      const int n = info & 0xffff, p0 = hd.x;
      const bool alongB = ((info >> 16) & 0xf) == 1;
      const int fk = alongB ? 1 : 0;
      const int64_t stride = a.n_fcut;
      T F[K], dF[K];
      if constexpr (D == 3) {
        lagrange1d<K>(Xn, ID, a.fcut_x[(1 - fk) * stride + p0], F, dF);
      } else {
#pragma unroll
        for (int i = 0; i < K; ++i) F[i] = 1;
      }
      T col[8][K];
#pragma unroll
      for (int lk = 0; lk < K; ++lk) {
#pragma unroll
        for (int k8 = 0; k8 < 8; ++k8) col[k8][lk] = 0;
#pragma unroll
        for (int f = 0; f < (D == 3 ? K : 1); ++f) {
          const int o = D == 3 ? (alongB ? lk + f * K : lk * K + f) : lk;
#pragma unroll
          for (int k8 = 0; k8 < 8; ++k8) col[k8][lk] += F[f] * W.TR[e][k8][o];
        }
      }
      for (int pi = 0; pi < n; ++pi) {
        const int64_t q = p0 + pi;
        T Z[K], dZ[K];
        lagrange1d<K>(Xn, ID, a.fcut_x[fk * stride + q], Z, dZ);
        T ev[8];
#pragma unroll
        for (int k8 = 0; k8 < 8; ++k8) {
          T sacc = 0;
#pragma unroll
          for (int ii = 0; ii < K; ++ii) sacc += Z[ii] * col[k8][ii];
          ev[k8] = sacc;
        }
        // the lower cell: jump = own - neighbour, average of the d_n
        const T Jw = ev[0] - ev[2], Aw = T(0.5) * (ev[1] + ev[3]);
        const T Ju = ev[4] - ev[6], Au = T(0.5) * (ev[5] + ev[7]);
        dk[a.seg[3] + q] = (a.terms & 2) ? a.hs * a.fcut_w[q] * (-Aw * Ju - Jw * Au + a.gamma * Jw * Ju) : T(0);
      }
    }
    sync();
  }
}

// ------------------------------------------------ mixed evaluation
// The cut cells' volume and interface terms as precomputed element matrices
// (the "mixed" option of Section 3.2, eq. additive_decomp: the unstructured
// cell integrals precomputed, the rest matrix-free).  One wave per cut cell
// and round of 64 rows; the matrix is column-major, so that the lanes' row
// entries of one column are contiguous; the cell's DoFs come from LDS.  The
// product is added to v (stage 4).  A streaming kernel: nd^2 values per
// cell against 2 nd flops each row, far below any ridge point.
template <int K, int D, typename T>
__global__ void __launch_bounds__(64) cut_matrix_kernel(DevArgs<T> a, const T* __restrict__ x, T* __restrict__ v) {
  constexpr int ND = ipow(K, D), NPL = (ND + 63) / 64;
  __shared__ T U[ND];
  const int t = threadIdx.x;
  for (int c = blockIdx.x; c < a.n_cut; c += gridDim.x) {
    const int64_t r = a.cut_rank[c];
    for (int i = t; i < ND; i += 64) U[i] = x[r * ND + i];
    sync();
    const T* M = a.cmat + (int64_t)c * ND * ND;
    T acc[NPL];
#pragma unroll
    for (int j = 0; j < NPL; ++j) acc[j] = 0;
    for (int col = 0; col < ND; ++col) {
      const T uc = U[col];
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        const int i = t + 64 * j;
        if (i < ND) acc[j] += M[(int64_t)col * ND + i] * uc;
      }
    }
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
      const int i = t + 64 * j;
      if (i < ND) v[r * ND + i] += acc[j];
    }
    sync();
  }
}

// resident workgroups of a kernel per compute unit (persistent grids)
template <typename Kern>
int blocks_per_cu(Kern kernel) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 64, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

// workgroups of a line kernel: one per batch (the hardware hands the next
// batch to whichever workgroup slot frees first), or the resident ones of
// the chip striding through the batches with the next batch's record in
// flight.  Measured on the MI355X: one per batch is faster for the volume
// lines from K = 4 on (-9 % in double at the 64^3 ball, -4 % / -14 % for
// the 20 balls, -3 to -26 % at K = 5..8) and for the cut-face lines at K = 4
// once there are more than three batches per resident workgroup (-18 % at
// the 104^3 ball, -26 % for the 20 balls, +4 % at the 64^3 ball with under
// two); the persistent grid is faster for the other cases (up to 11 %).
inline int64_t line_grid(int64_t n_batches, int64_t resident, bool one_per_batch) {
  return one_per_batch ? n_batches : std::min(n_batches, resident);
}

// workgroups of a launch: g, capped by DevArgs::max_blocks when that is set
template <typename T>
inline int grid_cap(const DevArgs<T>& a, int64_t g) {
  int64_t c = std::min<int64_t>(g, 1 << 20);
  if (a.max_blocks > 0) c = std::min<int64_t>(c, a.max_blocks);
  return (int)c;
}

template <int K, int D, typename T>
hipError_t launch_kd(const DevArgs<T>& a, const T* x, const T* y, T* v, T* dk, bool adj, hipStream_t s) {
  if (adj) {
    // A is symmetric: A^T w is the apply of w; dkappa from the evaluation
    // kernels
    DevArgs<T> b = a;
    b.parts = 15;
    hipError_t e = launch_kd<K, D, T>(b, x, nullptr, v, nullptr, false, s);
    if (e != hipSuccess || dk == nullptr) return e;
    {
      constexpr int CW = KronShape<K, D>::C, CF = FaceDkShape<K, D>::C;
      if (a.n_inside > 0)
        inside_dk_kernel<K, D, T><<<grid_cap(a, (a.n_inside + CW - 1) / CW), 64, 0, s>>>(a, x, y, dk);
      if (a.n_sfaces > 0)
        face_dk_kernel<K, D, T><<<grid_cap(a, (a.n_active + CF - 1) / CF), 64, 0, s>>>(a, x, y, dk);
      if (a.n_vbatch > 0)
        cut_dk_kernel<K, D, T><<<grid_cap(a, a.n_vbatch), 64, 0, s>>>(a, x, y, dk, a.vbrec, a.vdesc,
                                                                              a.n_vbatch);
      if (a.n_fbatch > 0)
        cut_face_dk_kernel<K, D, T><<<grid_cap(a, a.n_fbatch), 64, 0, s>>>(a, x, y, dk, a.fbrec, a.fdesc,
                                                                            a.n_fbatch);
    }
    return hipGetLastError();
  }
  const bool both = a.kappa == nullptr && (a.parts & 3) == 3;
  constexpr int CW = KronShape<K, D>::C;
  if (both) {
    // inside cells and the structured faces of the cut cells in one launch
    const int64_t n_all = a.n_inside + a.n_cut;
    constexpr int CK = KronShape<K, D>::CK;
    const int gk = grid_cap(a, (n_all + CK - 1) / CK);
    if (gk > 0) inside_kron_kernel<K, D, T><<<gk, KronShape<K, D>::NTK, 0, s>>>(a, x, v, a.kinfo_all, (int)n_all, 1);
  } else if (a.kappa == nullptr) {
    constexpr int CK = KronShape<K, D>::CK;
    const int gk = (a.parts & 1) ? grid_cap(a, (a.n_inside + CK - 1) / CK) : 0;
    if (gk > 0) inside_kron_kernel<K, D, T><<<gk, KronShape<K, D>::NTK, 0, s>>>(a, x, v, a.kinfo_inside, a.n_inside, 1);
  } else {
    const int gk = (a.parts & 1) ? grid_cap(a, (a.n_inside + CW - 1) / CW) : 0;
    if (gk > 0)
      kappa_struct_kernel<K, D, T><<<gk, KronShape<K, D>::NT, 0, s>>>(a, x, v, a.kinfo_inside, a.kface_inside,
                                                                      a.n_inside, 1);
  }
  {
    // structured faces and ghost penalty of the cut cells (overwrites
    // their rows: Kronecker kernel with kappa = 1, per-point face
    // quadrature with kappa), then the volume / interface lines and the
    // cut-face lines are added
    const int gs = (a.parts & 2) && !both ? grid_cap(a, (a.n_cut + CW - 1) / CW) : 0;
    if (gs > 0) {
      if (a.kappa == nullptr)
        inside_kron_kernel<K, D, T><<<grid_cap(a, (a.n_cut + KronShape<K, D>::CK - 1) / KronShape<K, D>::CK),
                                      KronShape<K, D>::NTK, 0, s>>>(a, x, v, a.kinfo_cut, a.n_cut, 0);
      else
        kappa_struct_kernel<K, D, T><<<gs, KronShape<K, D>::NT, 0, s>>>(a, x, v, a.kinfo_cut, a.kface_cut, a.n_cut,
                                                                        0);
    }
    if ((a.parts & 4) && a.cmat != nullptr && a.n_cut > 0) {
      cut_matrix_kernel<K, D, T><<<grid_cap(a, a.n_cut), 64, 0, s>>>(a, x, v);
    } else if ((a.parts & 4) && (a.terms & 5) && a.n_vbatch > 0) {
      static const int nb = blocks_per_cu(cut_batch_kernel<K, D, T>);
      const int g = grid_cap(a, line_grid(a.n_vbatch, nb * a.n_cu, K >= 4));
      cut_batch_kernel<K, D, T><<<g, 64, 0, s>>>(a, x, v, a.vbrec, a.vdesc, a.n_vbatch);
    }
    if ((a.parts & 8) && (a.terms & 2) && a.n_fbatch > 0) {
      static const int nb = blocks_per_cu(cut_face_kernel<K, D, T>);
      const int g = grid_cap(a, line_grid(a.n_fbatch, nb * a.n_cu, K == 4 && a.n_fbatch > 3 * nb * a.n_cu));
      cut_face_kernel<K, D, T><<<g, 64, 0, s>>>(a, x, v, a.fbrec, a.fdesc, a.n_fbatch);
    }
  }
  return hipGetLastError();
}

template <int D, typename T>
hipError_t launch_d(const DevArgs<T>& a, int degree, const T* x, const T* y, T* v, T* dk, bool adj, hipStream_t s) {
  switch (degree) {
    case 1: return launch_kd<2, D>(a, x, y, v, dk, adj, s);
    case 2: return launch_kd<3, D>(a, x, y, v, dk, adj, s);
    case 3: return launch_kd<4, D>(a, x, y, v, dk, adj, s);
    case 4: return launch_kd<5, D>(a, x, y, v, dk, adj, s);
    case 5: return launch_kd<6, D>(a, x, y, v, dk, adj, s);
    case 6: return launch_kd<7, D>(a, x, y, v, dk, adj, s);
    case 7: return launch_kd<8, D>(a, x, y, v, dk, adj, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace kern
}  // namespace ufem
