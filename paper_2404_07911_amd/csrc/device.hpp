// Device-side data of an operator and the launch interface of the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ufem {

// Slot s = 2 * axis + side of an active cell; side 1 is the upper face (the
// cell is the lower, "-", side of it), side 0 the lower face.
// flags word of an active cell: bit s -> ghost penalty on slot s,
// bit 8 + s -> structured SIPG, bit 16 + s -> cut SIPG.
constexpr int kFlagGP = 0, kFlagStr = 8, kFlagCut = 16;
// in the combined list of the Kronecker kernel: a cut cell (faces only)
constexpr int kFlagNoVolume = 24;

// Table layout (per precision), K = p + 1:
//   S [K*K]   S[q*K+i]  = L_i(g_q), GLL Lagrange basis at the Gauss points
//   DG[K*K]   DG[q*K+r] = l'_r(g_q), derivative of the Gauss Lagrange basis
//   W [K]     Gauss weights on [0, 1]
//   E0[K*K]   E0[j*K+l] = L_l^(j)(0)
//   E1[K*K]   E1[j*K+l] = L_l^(j)(1)
//   X [K]     GLL nodes
//   ID[K]     1 / prod_{j != i} (x_i - x_j)
//   GW[K]     ghost-penalty weights gamma_j, j = 0..p
//   M [K*K]   1D mass matrix of the GLL Lagrange basis (exact: Gauss rule)
//   KS[K*K]   1D stiffness matrix of the GLL Lagrange basis
//   DS[K*K]   DS[q*K+i] = L_i'(g_q), GLL basis derivative at the Gauss points
//   GP[4*K*K] face ghost penalty of a face on side s (0: lower, 1: upper) of
//             the own cell, GP[(2s+n)*K*K + l*K + m] = sum_j gamma_j E^j_l
//             F^j_m with E the own basis derivatives at the face and F = E
//             (n = 0) or the neighbour's (n = 1); with the volume ghost
//             penalty tau_v times the 1D mass of the own basis with the own
//             (n = 0) or the neighbour's (n = 1) basis over the two-cell patch
// (kernels that stage the table in LDS copy its first lds_size(K) entries)
// Line batches of the cut-cell kernels.  Batch b has a record of
// batch_record_ints(ME) ints at a fixed stride: (entries, lines, offset of
// its descriptors beyond the first kBatchLines in the overflow area, 0), then
// ME entries of 4 ints: (active rank of the cell, lines along axis 0 | lines
// along axis 1 << 16, offset of the entry's first line in the batch | slot <<
// 24, active rank of the neighbour across the slot or -1).  Line descriptors
// are int pairs (first point, count | axis << 16 | kind << 20 | entry << 24):
// the first kBatchLines of batch b at [b * kBatchLines, ...) (unused slots
// zero), the rest in the overflow area after n_batches * kBatchLines.  The
// lines of an entry are consecutive and ordered by axis: cell axes for
// volume / interface entries (slot 15), in-face axes for cut-face entries
// (one per cut face of a cut cell).  Entries of one cell are consecutive and
// in one batch.
// entries (one per cell, or per cut face of a cell) and cells of a batch (a
// cut cell has at least 2 k^(d-1) volume and interface lines, so a batch of
// 64 lines rarely holds more volume entries than these; at degree 1 a cut
// cell has about 4 cut faces with 10 face lines in all, so that 6 cells
// fill a round of face lines; a 3D cut cell at degree 4 has at least 50
// lines, so its batches hold one cell)
// Volume batches depend on the precision (f32): at K^d = 64 the float
// kernel takes two cells per batch, whose smaller LDS allows four waves per
// SIMD (float volume lines 38.9 -> 35.6 us at 64^3, p = 3; 178 -> 142 us for
// 20 balls at 128^3), while the double kernel, held at two waves by its
// registers, keeps four (fewer batches).
constexpr __host__ __device__ int batch_max_entries(int nd, bool face, bool f32 = false) {
  return face ? (nd <= 8 ? 24 : (nd <= 64 ? 12 : 6))
              : (nd <= 27 ? 8 : (nd <= 64 ? (f32 ? 2 : 4) : (nd < 125 ? 2 : 1)));
}
constexpr __host__ __device__ int batch_max_cells(int nd, bool face, bool f32 = false) {
  return face ? (nd <= 8 ? 6 : (nd <= 64 ? 4 : (nd <= 125 ? 2 : 1))) : batch_max_entries(nd, false, f32);
}
constexpr __host__ __device__ int batch_record_ints(int me) { return 4 + 4 * me; }
constexpr int kBatchLines = 64;        // lines per round (one per lane)

constexpr int kBatchOffsetBits = 24;   // bits of the in-batch line offset

struct TabOff {
  static __host__ __device__ constexpr int S(int) { return 0; }
  static __host__ __device__ constexpr int DG(int K) { return K * K; }
  static __host__ __device__ constexpr int W(int K) { return 2 * K * K; }
  static __host__ __device__ constexpr int E0(int K) { return 2 * K * K + K; }
  static __host__ __device__ constexpr int E1(int K) { return 3 * K * K + K; }
  static __host__ __device__ constexpr int X(int K) { return 4 * K * K + K; }
  static __host__ __device__ constexpr int ID(int K) { return 4 * K * K + 2 * K; }
  static __host__ __device__ constexpr int GW(int K) { return 4 * K * K + 3 * K; }
  static __host__ __device__ constexpr int M(int K) { return 4 * K * K + 4 * K; }
  static __host__ __device__ constexpr int KS(int K) { return 5 * K * K + 4 * K; }
  static __host__ __device__ constexpr int DS(int K) { return 6 * K * K + 4 * K; }
  static __host__ __device__ constexpr int GP(int K) { return 7 * K * K + 4 * K; }
  static __host__ __device__ constexpr int lds_size(int K) { return 7 * K * K + 4 * K; }
  static __host__ __device__ constexpr int size(int K) { return 11 * K * K + 4 * K; }
};

template <typename T>
struct DevArgs {
  int32_t n_active, n_inside, n_cut;
  const int32_t* inside;     // active ranks of inside cells
  // per position of the inside / cut list: (active rank, flags, neighbour
  // ranks of the 2d slots, -1 padding), 8 ints
  const int32_t* kinfo_inside;
  const int32_t* kinfo_cut;
  const int32_t* kinfo_all;  // both, in rank order (position = active rank), cut cells flagged kFlagNoVolume
  // per position and slot: kappa offset of the structured face's points
  const int64_t* kface_inside;
  const int64_t* kface_cut;
  // line batches (layout above): volume / interface lines of cut cells and
  // cut-face lines; records and line descriptors
  const int32_t* vbrec;
  const int32_t* vdesc;
  const int32_t* fbrec;
  const int32_t* fdesc;
  int32_t n_vbatch, n_fbatch;
  int32_t n_cu;  // compute units of the device (persistent grids)
  // structured SIPG faces (kappa order: by lower cell, then axis): index of
  // the first one whose lower cell is active cell r, per r
  const int32_t* sf_first;
  int32_t n_sfaces;
  const T* vol_x;            // SoA: vol_x[a * n_vol + q]
  const T* vol_w;
  const T* surf_x;           // SoA
  const T* surf_w;
  const T* surf_n;           // SoA
  const T* fcut_x;           // SoA over dim-1 in-face axes, index (qoff - seg3)
  const T* fcut_w;
  int64_t n_vol, n_surf, n_fcut;
  int64_t seg[6];
  const T* tab;
  // mixed evaluation: element matrices of the cut cells' volume and interface
  // terms (cut order, column-major nd x nd), nullptr: matrix-free
  const T* cmat;
  const int32_t* cut_rank;   // active rank of each cut cell (cut order)
  const T* kappa;            // nullptr: kappa = 1
  T hs;                      // h^(dim - 2)
  T tau, gamma;
  int32_t terms;             // term mask
  int32_t parts;             // stage bits: 1 inside cells, 2 structured faces and ghost
                             // penalty of the cut cells, 4 cut volume and interface
                             // lines, 8 cut-face lines
  int32_t gp_volume;         // the ghost penalty is the volume kind (GP tables
                             // hold tau_v times the patch mass matrices)
  int32_t max_blocks;        // > 0: cap on the workgroups of every launch (the
                             // grid-stride and persistent loops then take
                             // several cell groups / batches per workgroup)
};

// Launchers: the per-dimension operator kernels live in op_<prec>_<dim>d.hip,
// the dispatch and the BLAS-1 in blas.hip.
template <typename T, int D>
hipError_t launch_operator_dim(const DevArgs<T>& a, int degree, const T* x, const T* y, T* v, T* dkappa, bool adjoint,
                               hipStream_t s);

template <typename T>
hipError_t launch_operator(const DevArgs<T>& a, int dim, int degree, const T* u, T* v, const T* w_adj, T* dkappa,
                           bool adjoint, hipStream_t s);

hipError_t launch_cg_tail(int prec, int64_t n, void* x, void* r, void* p, const void* ap, double* scal,
                           hipStream_t s);

// Mixed evaluation set-up (blas.hip): x := e_j in the rows of the cut cells
// (0 elsewhere); column j of the element matrices from the stage-4 result v.
hipError_t launch_unit_rows(int prec, int64_t n_dofs, int nd, int n_cut, const int32_t* cut_rank, int j, void* x,
                            hipStream_t s);
hipError_t launch_matrix_column(int prec, int nd, int n_cut, const int32_t* cut_rank, int j, const void* v, void* mat,
                                hipStream_t s);
hipError_t launch_matrix_cast(int64_t n, const double* in, float* out, hipStream_t s);

// Continuous space (blas.hip): ucell = P u (the node values copied into the
// cell DoFs), v = P^T vcell (each node sums its cell DoFs in a fixed order).
hipError_t launch_gather(int prec, int64_t n_cell, const int32_t* cell_node, const void* u, void* ucell,
                         hipStream_t s);
hipError_t launch_scatter(int prec, int64_t n_nodes, const int64_t* node_ptr, const int32_t* node_src,
                          const void* vcell, void* v, hipStream_t s);
// Static workspace of ufem_cg_iterate_static (blas.hip): 64 MiB for A p after
// 256 bytes of CG scalars.  static_scratch_address gives the calling
// thread's current device's copy.
constexpr size_t kStaticCgScalarBytes = 256;
constexpr size_t kStaticScratchBytes = (size_t(64) << 20) + kStaticCgScalarBytes;
hipError_t static_scratch_address(void** out);
// scal[0..3] := (r.r, 0, 0, 0)
hipError_t launch_cg_static_begin(int prec, int64_t n, const void* r, double* scal, hipStream_t s);
// out[0] := scal[0] (r.r), out[1] := scal[3] (breakdown flag)
hipError_t launch_cg_static_end(const double* scal, double* out, hipStream_t s);

hipError_t launch_dot(int prec, int64_t n, const void* x, const void* y, double* out, hipStream_t s);
hipError_t launch_axpby(int prec, int64_t n, double a, const void* x, double b, void* y, hipStream_t s);
hipError_t launch_cast(int pin, int pout, int64_t n, const void* x, void* y, hipStream_t s);
hipError_t launch_zero(int prec, int64_t n, void* y, hipStream_t s);

}  // namespace ufem
