// Host plan of the unfitted DG operator: cell classes, face lists,
// dimension-reduction quadrature of the cut entities and the
// quadrature-point layout.  Pure C++; no GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "ufem.h"

namespace ufem {

enum CellClass : int8_t { kInside = 0, kCut = 1, kOutside = 2 };
enum FaceKind : int32_t { kFaceStructured = 0, kFaceCut = 1, kFaceNone = 2 };

struct Face {
  int32_t bm, bp;  // background indices of the lower and upper cell
  int32_t axis;
  int32_t kind;    // FaceKind of the SIPG term
  int32_t gp;      // ghost penalty on the full face
  int64_t qp_off;  // kappa offset of its SIPG points (-1: none)
  int32_t qp_n;
};

struct Plan {
  ufem_problem prob{};
  std::vector<double> centers, radii;
  bool plane = false;              // level set n . x - c (unit n) instead of balls
  double pn[3] = {0, 0, 0}, pc = 0.0;
  int dim = 3, n = 0, p = 1, k = 2, q = 2, max_depth = 4;
  double h = 0.0, lo = 0.0;
  double tau = 0.0, gamma = 0.0;
  int gp_kind = UFEM_GP_FACE;      // ghost-penalty kind (ufem.h)
  std::vector<double> gp_w;  // gamma_j for j = 0..p (0 below jmin)

  std::vector<int8_t> cls;      // per background cell
  std::vector<int32_t> active;  // background index per active rank
  std::vector<int32_t> rank;    // background -> active rank or -1
  std::vector<int32_t> inside;  // active ranks of inside cells
  std::vector<int32_t> cut;     // active ranks of cut cells
  std::vector<Face> faces;
  // per active cell, 2*dim slots (slot = 2 axis + side; side 1 = upper face):
  std::vector<int32_t> slot_face;  // face index or -1

  // cut-cell rules (reference coordinates, reference weights), cut order
  std::vector<int64_t> vol_off, surf_off;     // size n_cut + 1
  std::vector<double> vol_x, vol_w;           // dim per point
  std::vector<double> surf_x, surf_w, surf_n; // dim per point
  // cut-face rules, in cut-face order: in-face reference coords (dim-1)
  std::vector<int64_t> fcut_off;  // size n_faces_cut + 1
  std::vector<int32_t> fcut_face; // face index of each cut face
  std::vector<double> fcut_x, fcut_w;

  // point lines: runs of consecutive points that share every coordinate but
  // one (the line axis); cell lines hold the volume lines then the interface
  // points (one-point lines), face lines the points of each cut face
  std::vector<int64_t> cell_line_off;  // size n_cut + 1
  std::vector<int64_t> face_line_off;  // size n_faces_cut + 1
  // per line: first point (index into the vol/surf/fcut arrays), count,
  // axis (cell axis; for face lines the in-face axis index), kind 0 volume,
  // 1 interface, 2 cut face
  std::vector<int32_t> line_first, line_n, line_axis, line_kind;

  // kappa layout
  int64_t seg[6] = {0, 0, 0, 0, 0, 0};
  int64_t n_faces_str = 0, n_faces_cut = 0, n_faces_gp = 0;
  int64_t n_fallback = 0;
  int64_t max_qp_cut_cell = 0;

  // cell DoFs: the discontinuous layout every kernel works on
  int64_t n_dofs() const { return (int64_t)active.size() * nd(); }
  // continuous space (FE_Q): the Gauss-Lobatto nodes of the active cells on
  // the global node lattice, numbered in lattice order; cell_node maps cell
  // DoF r * nd + l to its node, node_ptr / node_src list every node's cell
  // DoFs in increasing order
  bool cg = false;
  int64_t n_nodes = 0;
  std::vector<int32_t> cell_node;
  std::vector<int64_t> node_ptr;
  std::vector<int64_t> node_src;
  // DoFs of the space: nodes (continuous) or cell DoFs (discontinuous)
  int64_t n_space_dofs() const { return cg ? n_nodes : n_dofs(); }
  int nd() const { int r = 1; for (int a = 0; a < dim; ++a) r *= k; return r; }
  int nf() const { int r = 1; for (int a = 0; a < dim - 1; ++a) r *= k; return r; }
  void cell_lo(int32_t b, double* x) const;
};

// Builds the plan; returns an error message (empty on success).
std::string build_plan(const ufem_problem& prob, Plan& plan, int* code);
// Replaces the cut rules by explicit ones (layout of ufem_plan_import_quadrature)
// and rebuilds the point lines and the kappa layout.
std::string import_rules(Plan& plan, const int64_t* vol_count, const int64_t* face_count, const int64_t* surf_count,
                         const double* ref, const double* w, const double* nrm, int* code);

// 1D rules and Lagrange data used by the plan and the device tables.
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);
void gauss_lobatto01(int n, std::vector<double>& x);
// derivatives of order 0..maxd of the Lagrange polynomials on `nodes` at t:
// out[d * n + i]
void lagrange_all(const std::vector<double>& nodes, double t, int maxd, std::vector<double>& out);

}  // namespace ufem
