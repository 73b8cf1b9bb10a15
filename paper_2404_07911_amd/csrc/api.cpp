// C ABI of the operator library: plan creation (host), upload (setup),
// apply / adjoint launches and the solver BLAS-1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "device.hpp"
#include "plan.hpp"
#include "ufem.h"

struct ufem_plan {
  ufem::Plan P;
};

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hipfail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return UFEM_EHIP;
}

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Device address of the static CG workspace, per device (set at the first
// ufem_setup on that device, with the device current).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

int init_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(UFEM_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return UFEM_OK;
  void* p = nullptr;
  hipError_t e = ufem::static_scratch_address(&p);
  if (e != hipSuccess) return hipfail(e, "hipGetSymbolAddress(scratch)");
  if (!p) return fail(UFEM_EHIP, "hipGetSymbolAddress(scratch) returned null");
  g_scratch[device] = p;
  return UFEM_OK;
}

void* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

void fill_info(const ufem::Plan& P, ufem_info* I) {
  std::memset(I, 0, sizeof(*I));
  I->n_background = (int64_t)P.cls.size();
  I->n_active = (int64_t)P.active.size();
  I->n_inside = (int64_t)P.inside.size();
  I->n_cut = (int64_t)P.cut.size();
  I->n_dofs = P.n_space_dofs();
  I->n_cell_dofs = P.n_dofs();
  I->n_faces = (int64_t)P.faces.size();
  I->n_faces_str = P.n_faces_str;
  I->n_faces_cut = P.n_faces_cut;
  I->n_faces_gp = P.n_faces_gp;
  I->n_qp = P.seg[5];
  for (int i = 0; i < 6; ++i) I->seg[i] = P.seg[i];
  I->max_qp_cut_cell = P.max_qp_cut_cell;
  I->n_fallback = P.n_fallback;
  I->h = P.h;
}

// 1D tables in the TabOff layout (double; converted per precision)
std::vector<double> make_tables(const ufem::Plan& P) {
  const int K = P.k;
  std::vector<double> t(ufem::TabOff::size(K), 0.0);
  std::vector<double> gx, gw, xl, tmp;
  ufem::gauss_legendre01(K, gx, gw);
  ufem::gauss_lobatto01(K, xl);
  for (int q = 0; q < K; ++q) {
    ufem::lagrange_all(xl, gx[q], 0, tmp);
    for (int i = 0; i < K; ++i) t[ufem::TabOff::S(K) + q * K + i] = tmp[i];
    ufem::lagrange_all(gx, gx[q], 1, tmp);
    for (int r = 0; r < K; ++r) t[ufem::TabOff::DG(K) + q * K + r] = tmp[K + r];
    t[ufem::TabOff::W(K) + q] = gw[q];
  }
  ufem::lagrange_all(xl, 0.0, K - 1, tmp);
  for (int j = 0; j < K; ++j)
    for (int l = 0; l < K; ++l) t[ufem::TabOff::E0(K) + j * K + l] = tmp[j * K + l];
  ufem::lagrange_all(xl, 1.0, K - 1, tmp);
  for (int j = 0; j < K; ++j)
    for (int l = 0; l < K; ++l) t[ufem::TabOff::E1(K) + j * K + l] = tmp[j * K + l];
  for (int i = 0; i < K; ++i) {
    t[ufem::TabOff::X(K) + i] = xl[i];
    double den = 1.0;
    for (int j = 0; j < K; ++j)
      if (j != i) den *= xl[i] - xl[j];
    t[ufem::TabOff::ID(K) + i] = 1.0 / den;
    t[ufem::TabOff::GW(K) + i] = i <= P.p ? P.gp_w[i] : 0.0;
  }
  // 1D mass and stiffness of the GLL basis, integrated exactly by the K-point
  // Gauss rule (degree 2p <= 2K - 1)
  std::vector<double> dl;
  for (int q = 0; q < K; ++q) {
    ufem::lagrange_all(xl, gx[q], 1, dl);
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) {
        t[ufem::TabOff::M(K) + i * K + j] += gw[q] * dl[i] * dl[j];
        t[ufem::TabOff::KS(K) + i * K + j] += gw[q] * dl[K + i] * dl[K + j];
      }
    for (int i = 0; i < K; ++i) t[ufem::TabOff::DS(K) + q * K + i] = dl[K + i];
  }
  if (P.gp_kind != UFEM_GP_FACE) {
    // volume ghost penalty: tau_v times the 1D mass matrices of the own basis
    // with itself and with the neighbour's basis over the two-cell patch
    // (neighbour at [1, 2] for side 1, at [-1, 0] for side 0, in the own
    // cell's coordinates), by the K-point Gauss rule on each half (exact)
    const double tv = P.prob.gp_gamma;
    std::vector<double> lo_, ln_;
    for (int s = 0; s < 2; ++s) {
      const double sh = s ? 1.0 : -1.0;  // neighbour coordinate = x - sh
      double* Go = &t[ufem::TabOff::GP(K) + (2 * s) * K * K];
      double* Gn = Go + K * K;
      for (int half = 0; half < 2; ++half) {
        const double off = half ? sh : 0.0;  // the own cell, then the neighbour's cell
        for (int q = 0; q < K; ++q) {
          const double x = off + gx[q];
          ufem::lagrange_all(xl, x, 0, lo_);
          ufem::lagrange_all(xl, x - sh, 0, ln_);
          for (int l = 0; l < K; ++l)
            for (int m = 0; m < K; ++m) {
              Go[l * K + m] += tv * gw[q] * lo_[l] * lo_[m];
              Gn[l * K + m] += tv * gw[q] * lo_[l] * ln_[m];
            }
        }
      }
    }
    return t;
  }
  // ghost penalty of a face, folded over the derivative orders j
  for (int s = 0; s < 2; ++s) {
    const double* Eo = &t[s ? ufem::TabOff::E1(K) : ufem::TabOff::E0(K)];
    const double* En = &t[s ? ufem::TabOff::E0(K) : ufem::TabOff::E1(K)];
    for (int l = 0; l < K; ++l)
      for (int m = 0; m < K; ++m) {
        double oo = 0, on = 0;
        for (int j = 0; j < K; ++j) {
          const double g = t[ufem::TabOff::GW(K) + j] * Eo[j * K + l];
          oo += g * Eo[j * K + m];
          on += g * En[j * K + m];
        }
        t[ufem::TabOff::GP(K) + (2 * s) * K * K + l * K + m] = oo;
        t[ufem::TabOff::GP(K) + (2 * s + 1) * K * K + l * K + m] = on;
      }
  }
  return t;
}

}  // namespace

struct ufem_op {
  ufem::Plan P;  // host copy (layout, counts)
  int device = 0;
  int32_t terms = UFEM_TERM_ALL;
  int32_t max_blocks = 0;
  std::vector<void*> allocs;
  int64_t bytes = 0;
  int64_t max_bytes = 0;
  // integer data
  int32_t* inside = nullptr;
  int64_t *kface_inside = nullptr, *kface_cut = nullptr;
  // volume batches per precision (index 0: double, 1: float; the same
  // arrays when both precisions take the same batch size)
  int32_t *vbrec[2] = {nullptr, nullptr}, *vdesc[2] = {nullptr, nullptr};
  int32_t *fbrec = nullptr, *fdesc = nullptr, *kinfo_inside = nullptr,
          *kinfo_cut = nullptr, *kinfo_all = nullptr, *sf_first = nullptr;
  int32_t n_vbatch[2] = {0, 0}, n_fbatch = 0, n_sfaces = 0, n_cu = 1;
  int32_t* cut_rank = nullptr;      // active ranks of the cut cells
  // continuous space: P (cell DoF -> node), P^T (node -> its cell DoFs) and
  // three cell-layout vectors (float64 size, shared by both precisions)
  int32_t* cell_node = nullptr;
  int64_t* node_ptr = nullptr;
  int32_t* node_src = nullptr;
  void* cvec[3] = {nullptr, nullptr, nullptr};
  void* cmat[2] = {nullptr, nullptr};  // mixed evaluation: element matrices per precision
  bool mixed = false;
  // per-precision data
  struct Prec {
    void *vol_x = nullptr, *vol_w = nullptr, *surf_x = nullptr, *surf_w = nullptr, *surf_n = nullptr,
         *fcut_x = nullptr, *fcut_w = nullptr, *tab = nullptr, *kappa = nullptr;
    bool has_kappa = false;
  } prec[2];

  ~ufem_op() {
    DeviceGuard g(device);
    for (void* p : allocs) (void)hipFree(p);
  }
  int alloc(void** p, size_t n) {
    if (n == 0) n = 8;
    if (max_bytes > 0 && bytes + (int64_t)n > max_bytes)
      return fail(UFEM_ENOMEM, "device memory cap exceeded (max_device_bytes)");
    hipError_t e = hipMalloc(p, n);
    if (e != hipSuccess) return hipfail(e, "hipMalloc");
    allocs.push_back(*p);
    bytes += (int64_t)n;
    return UFEM_OK;
  }
  template <class V>
  int upload(void** p, const V& host) {
    size_t n = host.size() * sizeof(typename V::value_type);
    int rc = alloc(p, n);
    if (rc) return rc;
    if (!host.empty()) {
      hipError_t e = hipMemcpy(*p, host.data(), n, hipMemcpyHostToDevice);
      if (e != hipSuccess) return hipfail(e, "hipMemcpy");
    }
    return UFEM_OK;
  }
  template <typename T>
  int upload_prec(Prec& d, const std::vector<double>& tab);
  template <typename T>
  ufem::DevArgs<T> args(const Prec& d) const;
};

template <typename T>
int ufem_op::upload_prec(Prec& d, const std::vector<double>& tab) {
  const ufem::Plan& Q = P;
  const int dim = Q.dim;
  auto soa = [&](const std::vector<double>& aos, int comps) {
    size_t n = comps ? aos.size() / comps : 0;
    std::vector<T> out(aos.size());
    for (size_t i = 0; i < n; ++i)
      for (int c = 0; c < comps; ++c) out[c * n + i] = (T)aos[i * comps + c];
    return out;
  };
  auto conv = [&](const std::vector<double>& v) {
    std::vector<T> out(v.size());
    for (size_t i = 0; i < v.size(); ++i) out[i] = (T)v[i];
    return out;
  };
  int rc;
  if ((rc = upload(&d.vol_x, soa(Q.vol_x, dim)))) return rc;
  if ((rc = upload(&d.vol_w, conv(Q.vol_w)))) return rc;
  if ((rc = upload(&d.surf_x, soa(Q.surf_x, dim)))) return rc;
  if ((rc = upload(&d.surf_w, conv(Q.surf_w)))) return rc;
  if ((rc = upload(&d.surf_n, soa(Q.surf_n, dim)))) return rc;
  if ((rc = upload(&d.fcut_x, soa(Q.fcut_x, dim - 1)))) return rc;
  if ((rc = upload(&d.fcut_w, conv(Q.fcut_w)))) return rc;
  if ((rc = upload(&d.tab, conv(tab)))) return rc;
  if ((rc = alloc(&d.kappa, sizeof(T) * (size_t)std::max<int64_t>(1, Q.seg[5])))) return rc;
  return UFEM_OK;
}

template <typename T>
ufem::DevArgs<T> ufem_op::args(const Prec& d) const {
  ufem::DevArgs<T> a{};
  a.n_active = (int32_t)P.active.size();
  a.n_inside = (int32_t)P.inside.size();
  a.n_cut = (int32_t)P.cut.size();
  a.inside = inside;
  a.kinfo_inside = kinfo_inside;
  a.kinfo_cut = kinfo_cut;
  a.kinfo_all = kinfo_all;
  a.kface_inside = kface_inside;
  a.kface_cut = kface_cut;
  const int vp = sizeof(T) == 4 ? 1 : 0;
  a.vbrec = vbrec[vp];
  a.vdesc = vdesc[vp];
  a.fbrec = fbrec;
  a.fdesc = fdesc;
  a.n_cu = n_cu;
  a.n_vbatch = n_vbatch[vp];
  a.n_fbatch = n_fbatch;
  a.sf_first = sf_first;
  a.n_sfaces = n_sfaces;
  a.vol_x = (const T*)d.vol_x;
  a.vol_w = (const T*)d.vol_w;
  a.surf_x = (const T*)d.surf_x;
  a.surf_w = (const T*)d.surf_w;
  a.surf_n = (const T*)d.surf_n;
  a.fcut_x = (const T*)d.fcut_x;
  a.fcut_w = (const T*)d.fcut_w;
  a.n_vol = (int64_t)P.vol_w.size();
  a.n_surf = (int64_t)P.surf_w.size();
  a.n_fcut = (int64_t)P.fcut_w.size();
  for (int i = 0; i < 6; ++i) a.seg[i] = P.seg[i];
  a.tab = (const T*)d.tab;
  a.kappa = d.has_kappa ? (const T*)d.kappa : nullptr;
  a.cut_rank = cut_rank;
  a.cmat = mixed ? (const T*)cmat[&d == &prec[0] ? 0 : 1] : nullptr;
  a.hs = (T)std::pow(P.h, P.dim - 2);
  a.tau = (T)P.tau;
  a.gamma = (T)P.gamma;
  a.terms = P.cg ? (terms & ~UFEM_TERM_SIPG) : terms;  // no SIPG term in the continuous space
  a.parts = 15;
  a.max_blocks = max_blocks;
  a.gp_volume = P.gp_kind != UFEM_GP_FACE ? 1 : 0;
  return a;
}

// One apply v = A u of the space on `st` (stages `part` of the cell-DoF
// operator; the continuous space takes the whole apply: P, the cell
// operator, P^T).  adjoint: v = A^T w with w in `u`, u in `y`, and dkappa.
template <typename T>
static hipError_t run_apply(ufem_op* op, int prec, int part, const void* u, void* v, const void* y, void* dk,
                            bool adjoint, hipStream_t st) {
  auto a = op->args<T>(op->prec[prec]);
  a.parts = part;
  const ufem::Plan& P = op->P;
  if (!P.cg)
    return ufem::launch_operator<T>(a, P.dim, P.p, (const T*)(adjoint ? y : u), (T*)v, (const T*)(adjoint ? u : nullptr),
                                    (T*)dk, adjoint, st);
  const int64_t nc = P.n_dofs();
  hipError_t e = ufem::launch_gather(prec, nc, op->cell_node, u, op->cvec[0], st);
  if (e == hipSuccess && adjoint) e = ufem::launch_gather(prec, nc, op->cell_node, y, op->cvec[2], st);
  if (e == hipSuccess)
    e = ufem::launch_operator<T>(a, P.dim, P.p, (const T*)(adjoint ? op->cvec[2] : op->cvec[0]), (T*)op->cvec[1],
                                 (const T*)(adjoint ? op->cvec[0] : nullptr), (T*)dk, adjoint, st);
  if (e == hipSuccess) e = ufem::launch_scatter(prec, P.n_nodes, op->node_ptr, op->node_src, op->cvec[1], v, st);
  return e;
}

static hipError_t run_apply_p(ufem_op* op, int prec, int part, const void* u, void* v, hipStream_t st) {
  return prec == UFEM_F64 ? run_apply<double>(op, prec, part, u, v, nullptr, nullptr, false, st)
                          : run_apply<float>(op, prec, part, u, v, nullptr, nullptr, false, st);
}

extern "C" {

const char* ufem_last_error(void) { return g_err.c_str(); }

int ufem_plan_create(const ufem_problem* prob, ufem_plan** out) {
  if (!prob || !out) return fail(UFEM_EINVAL, "ufem_plan_create: null argument");
  *out = nullptr;
  try {
    ufem_plan* p = new ufem_plan();
    int code = UFEM_OK;
    std::string msg = ufem::build_plan(*prob, p->P, &code);
    if (code != UFEM_OK) {
      delete p;
      return fail(code, "ufem_plan_create: " + msg);
    }
    *out = p;
    return UFEM_OK;
  } catch (const std::bad_alloc&) {
    return fail(UFEM_ENOMEM, "ufem_plan_create: host allocation failed");
  } catch (const std::exception& e) {
    return fail(UFEM_EINVAL, std::string("ufem_plan_create: ") + e.what());
  }
}

int ufem_plan_destroy(ufem_plan* plan) {
  delete plan;
  return UFEM_OK;
}

int ufem_plan_info(const ufem_plan* plan, ufem_info* info) {
  if (!plan || !info) return fail(UFEM_EINVAL, "ufem_plan_info: null argument");
  fill_info(plan->P, info);
  return UFEM_OK;
}

int ufem_plan_cells(const ufem_plan* plan, int8_t* cls) {
  if (!plan || !cls) return fail(UFEM_EINVAL, "ufem_plan_cells: null argument");
  std::memcpy(cls, plan->P.cls.data(), plan->P.cls.size());
  return UFEM_OK;
}

int ufem_plan_faces(const ufem_plan* plan, int32_t* faces) {
  if (!plan || !faces) return fail(UFEM_EINVAL, "ufem_plan_faces: null argument");
  size_t i = 0;
  for (const ufem::Face& f : plan->P.faces) {
    faces[i++] = f.bm;
    faces[i++] = f.bp;
    faces[i++] = f.axis;
    faces[i++] = f.kind;
    faces[i++] = f.gp;
  }
  return UFEM_OK;
}

int ufem_plan_qp(const ufem_plan* plan, double* xyz, double* ref, double* w, double* nrm) {
  if (!plan) return fail(UFEM_EINVAL, "ufem_plan_qp: null plan");
  try {
  const ufem::Plan& P = plan->P;
  const int dim = P.dim, K = P.k;
  std::vector<double> gx, gw;
  ufem::gauss_legendre01(K, gx, gw);
  auto put = [&](int64_t q, const double* lo, const double* r, double wt, const double* n) {
    for (int a = 0; a < dim; ++a) {
      if (xyz) xyz[q * dim + a] = lo[a] + P.h * r[a];
      if (ref) ref[q * dim + a] = r[a];
      if (nrm) nrm[q * dim + a] = n ? n[a] : 0.0;
    }
    if (w) w[q] = wt;
  };
  const int nd = P.nd(), nf = P.nf();
  int64_t q = 0;
  double lo[3], r[3];
  for (int32_t ar : P.inside) {
    P.cell_lo(P.active[ar], lo);
    for (int l = 0; l < nd; ++l, ++q) {
      int rem = l;
      double wt = 1.0;
      for (int a = 0; a < dim; ++a) {
        int g = rem % K;
        rem /= K;
        r[a] = gx[g];
        wt *= gw[g];
      }
      put(q, lo, r, wt, nullptr);
    }
  }
  for (size_t i = 0; i < P.cut.size(); ++i) {
    P.cell_lo(P.active[P.cut[i]], lo);
    for (int64_t j = P.vol_off[i]; j < P.vol_off[i + 1]; ++j, ++q) put(q, lo, &P.vol_x[j * dim], P.vol_w[j], nullptr);
  }
  for (const ufem::Face& f : P.faces) {
    if (f.kind != ufem::kFaceStructured) continue;
    P.cell_lo(f.bm, lo);
    for (int l = 0; l < nf; ++l, ++q) {
      int rem = l;
      double wt = 1.0;
      for (int a = 0; a < dim; ++a) {
        if (a == f.axis) { r[a] = 1.0; continue; }
        int g = rem % K;
        rem /= K;
        r[a] = gx[g];
        wt *= gw[g];
      }
      put(q, lo, r, wt, nullptr);
    }
  }
  for (size_t i = 0; i + 1 < P.fcut_off.size(); ++i) {
    const ufem::Face& f = P.faces[P.fcut_face[i]];
    P.cell_lo(f.bm, lo);
    for (int64_t j = P.fcut_off[i]; j < P.fcut_off[i + 1]; ++j, ++q) {
      int c = 0;
      for (int a = 0; a < dim; ++a) r[a] = a == f.axis ? 1.0 : P.fcut_x[j * (dim - 1) + c++];
      put(q, lo, r, P.fcut_w[j], nullptr);
    }
  }
  for (size_t i = 0; i < P.cut.size(); ++i) {
    P.cell_lo(P.active[P.cut[i]], lo);
    for (int64_t j = P.surf_off[i]; j < P.surf_off[i + 1]; ++j, ++q)
      put(q, lo, &P.surf_x[j * dim], P.surf_w[j], &P.surf_n[j * dim]);
  }
  return UFEM_OK;
  } catch (const std::bad_alloc&) {
    return fail(UFEM_ENOMEM, "ufem_plan_qp: host allocation failed");
  } catch (const std::exception& e) {
    return fail(UFEM_EINVAL, std::string("ufem_plan_qp: ") + e.what());
  }
}

int ufem_plan_import_quadrature(ufem_plan* plan, const int64_t* vol_count, const int64_t* face_count,
                                const int64_t* surf_count, const double* ref, const double* w, const double* nrm) {
  if (!plan) return fail(UFEM_EINVAL, "ufem_plan_import_quadrature: null plan");
  try {
    ufem::Plan Q = plan->P;  // the plan is left unchanged on failure
    int code = UFEM_OK;
    std::string msg = ufem::import_rules(Q, vol_count, face_count, surf_count, ref, w, nrm, &code);
    if (code != UFEM_OK) return fail(code, "ufem_plan_import_quadrature: " + msg);
    plan->P = std::move(Q);
    return UFEM_OK;
  } catch (const std::bad_alloc&) {
    return fail(UFEM_ENOMEM, "ufem_plan_import_quadrature: host allocation failed");
  } catch (const std::exception& e) {
    return fail(UFEM_EINVAL, std::string("ufem_plan_import_quadrature: ") + e.what());
  }
}

int ufem_setup(const ufem_plan* plan, int device, void* stream, int64_t max_device_bytes, ufem_op** out) {
  (void)stream;
  if (!plan || !out) return fail(UFEM_EINVAL, "ufem_setup: null argument");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hipfail(e, "ufem_setup: hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(UFEM_EINVAL, "ufem_setup: no such device");
  DeviceGuard guard(device);
  if (!guard.ok) return fail(UFEM_EHIP, "ufem_setup: hipSetDevice failed");
  {
    const int rc = init_static_scratch(device);
    if (rc != UFEM_OK) return rc;
  }
  ufem_op* op = nullptr;
  try {
    op = new ufem_op();
    op->P = plan->P;
    op->device = device;
    op->max_bytes = max_device_bytes;
    if (hipDeviceGetAttribute(&op->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        op->n_cu < 1)
      op->n_cu = 1;
    const ufem::Plan& P = op->P;
    const int dim = P.dim, S = 2 * dim;
    const size_t na = P.active.size();
    // neighbour ranks and flags per active cell and slot
    std::vector<int32_t> nb(na * S, -1), flags(na, 0);
    for (size_t r = 0; r < na; ++r) {
      for (int s = 0; s < S; ++s) {
        int32_t fi = P.slot_face[r * S + s];
        if (fi < 0) continue;
        const ufem::Face& f = P.faces[fi];
        nb[r * S + s] = P.rank[(s & 1) ? f.bp : f.bm];
        if (f.gp) flags[r] |= 1 << (ufem::kFlagGP + s);
        if (f.kind == ufem::kFaceStructured) flags[r] |= 1 << (ufem::kFlagStr + s);
        if (f.kind == ufem::kFaceCut) flags[r] |= 1 << (ufem::kFlagCut + s);
      }
    }
    // point lines
    std::vector<int32_t> flb(P.faces.size(), 0), fle(P.faces.size(), 0), linfo(P.line_first.size());
    for (size_t i = 0; i + 1 < P.face_line_off.size(); ++i) {
      flb[P.fcut_face[i]] = (int32_t)P.face_line_off[i];
      fle[P.fcut_face[i]] = (int32_t)P.face_line_off[i + 1];
    }
    for (size_t l = 0; l < P.line_first.size(); ++l)
      linfo[l] = P.line_n[l] | (P.line_axis[l] << 16) | (P.line_kind[l] << 20);
    // cut cells processed in decreasing order of quadrature work
    std::vector<int32_t> order(P.cut.size());
    std::iota(order.begin(), order.end(), 0);
    std::vector<int64_t> cost(P.cut.size());
    for (size_t i = 0; i < P.cut.size(); ++i) {
      int64_t c = (P.vol_off[i + 1] - P.vol_off[i]) + (P.surf_off[i + 1] - P.surf_off[i]);
      for (int s = 0; s < S; ++s) {
        int32_t fi = P.slot_face[(size_t)P.cut[i] * S + s];
        if (fi >= 0) c += P.nf() + P.faces[fi].qp_n;
      }
      cost[i] = c;
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
    // line batches for the cut-cell kernels: cells (most work first) packed
    // into waves of at most 64 lines; a cell with more lines gets a wave of
    // its own.  Fixed-size batch records and line descriptors (layout in
    // device.hpp), the lines of each entry ordered by axis.
    bool batch_overflow = false;
    auto make_batches = [&](bool face, bool f32, std::vector<int32_t>& brec, std::vector<int32_t>& desc,
                            int32_t& n_batches) {
      const int me = ufem::batch_max_entries((int)P.nd(), face, f32);
      const int mc = ufem::batch_max_cells((int)P.nd(), face, f32);
      const int nr = ufem::batch_record_ints(me);
      std::vector<int32_t> rec, lines, ovf;  // current batch; overflow area
      int cur_n = 0, cur_cells = 0;
      std::vector<int32_t> slots;            // first-round descriptors of all batches
      auto close = [&]() {
        if (cur_n == 0) return;
        const int total = (int)lines.size() / 2;
        rec[0] = cur_n;
        rec[1] = total;
        rec[2] = (int32_t)(ovf.size() / 2);
        rec[3] = 0;
        brec.insert(brec.end(), rec.begin(), rec.end());
        for (int g = 0; g < ufem::kBatchLines; ++g) {
          slots.push_back(g < total ? lines[2 * g] : 0);
          slots.push_back(g < total ? lines[2 * g + 1] : 0);
        }
        if (total > ufem::kBatchLines) ovf.insert(ovf.end(), lines.begin() + 2 * ufem::kBatchLines, lines.end());
        cur_n = 0;
        cur_cells = 0;
        lines.clear();
      };
      for (int32_t ci : order) {
        const int32_t r = P.cut[ci];
        std::vector<int32_t> ce;  // (first line, end line, slot, neighbour)
        if (!face) {
          const int32_t lb = (int32_t)P.cell_line_off[ci], le = (int32_t)P.cell_line_off[ci + 1];
          if (le > lb) ce.insert(ce.end(), {lb, le, 15, -1});
        } else {
          for (int sl = 0; sl < S; ++sl) {
            int32_t fi = P.slot_face[(size_t)r * S + sl];
            if (fi < 0 || P.faces[fi].kind != ufem::kFaceCut || fle[fi] <= flb[fi]) continue;
            ce.insert(ce.end(), {flb[fi], fle[fi], sl, nb[(size_t)r * S + sl]});
          }
        }
        if (ce.empty()) continue;
        int nl = 0, n_e = (int)ce.size() / 4;
        for (int e = 0; e < n_e; ++e) {
          nl += ce[4 * e + 1] - ce[4 * e];
          if (face && ce[4 * e + 3] < 0) batch_overflow = true;  // a cut face always has a neighbour
        }
        const int cur_lines = (int)lines.size() / 2;
        if (cur_n > 0 && (cur_lines + nl > ufem::kBatchLines || cur_n + n_e > me || cur_cells + 1 > mc)) close();
        if (batch_overflow || n_e > me || nl >= (1 << ufem::kBatchOffsetBits)) {
          batch_overflow = true;
          return;
        }
        if (cur_n == 0) rec.assign(nr, 0);
        for (int e = 0; e < n_e; ++e) {
          const int32_t lb = ce[4 * e], le = ce[4 * e + 1], sl = ce[4 * e + 2];
          // volume lines by cell axis, face lines by in-face axis (the same
          // order, the in-face axes being the other cell axes ascending)
          int cnt[3] = {0, 0, 0};
          const int first = (int)lines.size() / 2;
          for (int ax = 0; ax < P.dim; ++ax)
            for (int32_t l = lb; l < le; ++l) {
              if (P.line_axis[l] != ax) continue;
              lines.push_back((int32_t)P.line_first[l]);
              lines.push_back(linfo[l] | ((cur_n + e) << 24));
              ++cnt[ax];
            }
          if (cnt[0] > 0xffff || cnt[1] > 0xffff) {
            batch_overflow = true;
            return;
          }
          int32_t* en = &rec[4 + 4 * (cur_n + e)];
          en[0] = r;
          en[1] = cnt[0] | (cnt[1] << 16);
          en[2] = first | (sl << ufem::kBatchOffsetBits);
          en[3] = ce[4 * e + 3];
        }
        cur_n += n_e;
        ++cur_cells;
        if ((int)lines.size() / 2 >= ufem::kBatchLines) close();
      }
      close();
      n_batches = (int32_t)(brec.size() / nr);
      desc = std::move(slots);
      desc.insert(desc.end(), ovf.begin(), ovf.end());
    };
    // structured faces in kappa order (by lower cell, then axis): the index
    // of each active cell's first one
    std::vector<int32_t> sff(na, 0);
    int32_t n_sf = 0;
    {
      std::vector<int32_t> cnt(na, 0);
      for (const ufem::Face& f : P.faces)
        if (f.kind == ufem::kFaceStructured) ++cnt[P.rank[f.bm]];
      for (size_t r = 0; r < na; ++r) {
        sff[r] = n_sf;
        n_sf += cnt[r];
      }
    }
    op->n_sfaces = n_sf;
    // per-position cell info of the Kronecker kernel's lists
    auto make_kinfo = [&](const std::vector<int32_t>& list) {
      std::vector<int32_t> ki(list.size() * 8, -1);
      for (size_t i = 0; i < list.size(); ++i) {
        const int32_t r = list[i];
        ki[8 * i] = r;
        ki[8 * i + 1] = flags[r];
        for (int sl = 0; sl < S; ++sl) ki[8 * i + 2 + sl] = nb[(size_t)r * S + sl];
      }
      return ki;
    };
    const std::vector<int32_t> kin = make_kinfo(P.inside), kcu = make_kinfo(P.cut);
    auto make_kface = [&](const std::vector<int32_t>& list) {
      std::vector<int64_t> kf(list.size() * S, 0);
      for (size_t i = 0; i < list.size(); ++i)
        for (int sl = 0; sl < S; ++sl) {
          const int32_t fi = P.slot_face[(size_t)list[i] * S + sl];
          if (fi >= 0) kf[i * S + sl] = P.faces[fi].qp_off;
        }
      return kf;
    };
    const std::vector<int64_t> kfin = make_kface(P.inside), kfcu = make_kface(P.cut);
    // both lists merged in rank (background) order, so that every XCD's
    // contiguous range gets its share of the cheaper cut cells and neighbours
    // stay close
    std::vector<int32_t> kall;
    kall.reserve(kin.size() + kcu.size());
    for (size_t i = 0, j = 0; i < P.inside.size() || j < P.cut.size();) {
      const bool take_cut = i == P.inside.size() || (j < P.cut.size() && P.cut[j] < P.inside[i]);
      if (take_cut) {
        kall.insert(kall.end(), kcu.begin() + 8 * j, kcu.begin() + 8 * (j + 1));
        kall[kall.size() - 7] |= 1 << ufem::kFlagNoVolume;
        ++j;
      } else {
        kall.insert(kall.end(), kin.begin() + 8 * i, kin.begin() + 8 * (i + 1));
        ++i;
      }
    }
    std::vector<int32_t> vb, vl, vb32, vl32, fb, fl;
    make_batches(false, false, vb, vl, op->n_vbatch[0]);
    const bool own32 = ufem::batch_max_entries((int)P.nd(), false, true) != ufem::batch_max_entries((int)P.nd(), false);
    if (own32) make_batches(false, true, vb32, vl32, op->n_vbatch[1]);
    make_batches(true, false, fb, fl, op->n_fbatch);

    if (batch_overflow) {
      delete op;
      return fail(UFEM_EUNSUPPORTED, "ufem_setup: a cut cell has more lines or cut faces than one line batch holds");
    }
    int rc;
    if ((rc = op->upload((void**)&op->inside, P.inside)) || (rc = op->upload((void**)&op->cut_rank, P.cut)) ||
        (rc = op->upload((void**)&op->kinfo_inside, kin)) || (rc = op->upload((void**)&op->kinfo_cut, kcu)) ||
        (rc = op->upload((void**)&op->kinfo_all, kall)) || (rc = op->upload((void**)&op->kface_inside, kfin)) ||
        (rc = op->upload((void**)&op->kface_cut, kfcu)) ||
        (rc = op->upload((void**)&op->vbrec[0], vb)) || (rc = op->upload((void**)&op->vdesc[0], vl)) ||
        (own32 && ((rc = op->upload((void**)&op->vbrec[1], vb32)) || (rc = op->upload((void**)&op->vdesc[1], vl32)))) ||
        (rc = op->upload((void**)&op->fbrec, fb)) || (rc = op->upload((void**)&op->fdesc, fl)) ||
        (rc = op->upload((void**)&op->sf_first, sff))) {
      delete op;
      return rc;
    }
    if (!own32) {
      op->vbrec[1] = op->vbrec[0];
      op->vdesc[1] = op->vdesc[0];
      op->n_vbatch[1] = op->n_vbatch[0];
    }
    if (P.cg) {
      std::vector<int32_t> src(P.node_src.begin(), P.node_src.end());
      if ((rc = op->upload((void**)&op->cell_node, P.cell_node)) || (rc = op->upload((void**)&op->node_ptr, P.node_ptr)) ||
          (rc = op->upload((void**)&op->node_src, src))) {
        delete op;
        return rc;
      }
      for (int i = 0; i < 3; ++i)
        if ((rc = op->alloc(&op->cvec[i], (size_t)P.n_dofs() * sizeof(double)))) {
          delete op;
          return rc;
        }
    }
    std::vector<double> tab = make_tables(P);
    if ((rc = op->upload_prec<double>(op->prec[0], tab)) || (rc = op->upload_prec<float>(op->prec[1], tab))) {
      delete op;
      return rc;
    }
    *out = op;
    return UFEM_OK;
  } catch (const std::bad_alloc&) {
    delete op;
    return fail(UFEM_ENOMEM, "ufem_setup: host allocation failed");
  } catch (const std::exception& ex) {
    delete op;
    return fail(UFEM_EINVAL, std::string("ufem_setup: ") + ex.what());
  } catch (...) {
    delete op;
    return fail(UFEM_EINVAL, "ufem_setup: unexpected host error");
  }
}

int ufem_destroy(ufem_op* op) {
  delete op;
  return UFEM_OK;
}

int ufem_info_op(const ufem_op* op, ufem_info* info) {
  if (!op || !info) return fail(UFEM_EINVAL, "ufem_info_op: null argument");
  fill_info(op->P, info);
  return UFEM_OK;
}

// (Re)build the element matrices of the mixed evaluation: column j of every
// cut cell's matrix is the stage-4 (volume and interface lines) result of the
// unit vector e_j in every cut cell, with the current kappa and term mask;
// float64 matrices, rounded once to float32 for the float32 operator.
static int build_mixed(ufem_op* op, hipStream_t st) {
  const ufem::Plan& P = op->P;
  const int nd = P.nd();
  const int ncut = (int)P.cut.size();
  const int64_t n = P.n_dofs();
  const int64_t nm = (int64_t)ncut * nd * nd;
  if (ncut == 0) return UFEM_OK;
  int rc;
  if (!op->cmat[0]) {
    if ((rc = op->alloc(&op->cmat[0], (size_t)nm * sizeof(double)))) return rc;
    if ((rc = op->alloc(&op->cmat[1], (size_t)nm * sizeof(float)))) return rc;
  }
  void *x = nullptr, *v = nullptr;
  hipError_t e = hipMalloc(&x, (size_t)n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&v, (size_t)n * sizeof(double));
  if (e != hipSuccess) {
    (void)hipFree(x);
    return hipfail(e, "ufem_set_mixed: hipMalloc");
  }
  const bool was = op->mixed;
  op->mixed = false;  // the columns come from the matrix-free line kernels
  auto a = op->args<double>(op->prec[0]);
  op->mixed = was;
  a.parts = 4;
  for (int j = 0; j < nd && e == hipSuccess; ++j) {
    e = ufem::launch_unit_rows(0, n, nd, ncut, op->cut_rank, j, x, st);
    if (e == hipSuccess) e = ufem::launch_zero(0, n, v, st);
    if (e == hipSuccess)
      e = ufem::launch_operator<double>(a, P.dim, P.p, (const double*)x, (double*)v, nullptr, nullptr, false, st);
    if (e == hipSuccess) e = ufem::launch_matrix_column(0, nd, ncut, op->cut_rank, j, v, op->cmat[0], st);
  }
  if (e == hipSuccess) e = ufem::launch_matrix_cast(nm, (const double*)op->cmat[0], (float*)op->cmat[1], st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(x);
  (void)hipFree(v);
  if (e != hipSuccess) return hipfail(e, "ufem_set_mixed: element matrices");
  return UFEM_OK;
}

int ufem_set_mixed(ufem_op* op, int32_t enable, void* stream) {
  if (!op) return fail(UFEM_EINVAL, "ufem_set_mixed: null op");
  DeviceGuard g(op->device);
  if (!enable) {
    op->mixed = false;
    return UFEM_OK;
  }
  const int rc = build_mixed(op, (hipStream_t)stream);
  if (rc != UFEM_OK) return rc;
  op->mixed = true;
  return UFEM_OK;
}

int ufem_set_max_blocks(ufem_op* op, int32_t max_blocks) {
  if (!op) return fail(UFEM_EINVAL, "ufem_set_max_blocks: null op");
  if (max_blocks < 0) return fail(UFEM_EINVAL, "ufem_set_max_blocks: max_blocks < 0");
  op->max_blocks = max_blocks;
  return UFEM_OK;
}

int ufem_set_terms(ufem_op* op, int32_t mask) {
  if (!op) return fail(UFEM_EINVAL, "ufem_set_terms: null op");
  if (mask < 0 || mask > UFEM_TERM_ALL) return fail(UFEM_EINVAL, "ufem_set_terms: bad mask");
  op->terms = mask;
  if (op->mixed) {
    DeviceGuard g(op->device);
    return build_mixed(op, nullptr);
  }
  return UFEM_OK;
}

int ufem_set_kappa(ufem_op* op, int32_t precision, const void* kappa, void* stream) {
  if (!op) return fail(UFEM_EINVAL, "ufem_set_kappa: null op");
  if (precision != UFEM_F64 && precision != UFEM_F32) return fail(UFEM_EINVAL, "ufem_set_kappa: bad precision");
  DeviceGuard g(op->device);
  auto& d = op->prec[precision];
  if (!kappa) {
    d.has_kappa = false;
    if (op->mixed && precision == UFEM_F64) return build_mixed(op, (hipStream_t)stream);
    return UFEM_OK;
  }
  size_t bytes = (size_t)op->P.seg[5] * (precision == UFEM_F64 ? 8 : 4);
  hipError_t e = hipMemcpyAsync(d.kappa, kappa, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(e, "ufem_set_kappa");
  d.has_kappa = true;
  if (op->mixed && precision == UFEM_F64) return build_mixed(op, (hipStream_t)stream);
  return UFEM_OK;
}

static bool overlap2(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}
static bool overlap(const void* a, const void* b, size_t n) { return overlap2(a, n, b, n); }

int ufem_apply(ufem_op* op, int32_t precision, const void* u, void* v, void* stream) {
  return ufem_apply_part(op, precision, UFEM_PART_ALL, u, v, stream);
}

int ufem_apply_part(ufem_op* op, int32_t precision, int32_t part, const void* u, void* v, void* stream) {
  if (!op || !u || !v) return fail(UFEM_EINVAL, "ufem_apply: null argument");
  if (part < 1 || part > UFEM_PART_ALL) return fail(UFEM_EINVAL, "ufem_apply_part: part must be a non-empty mask of UFEM_PART_* bits");
  if (precision != UFEM_F64 && precision != UFEM_F32) return fail(UFEM_EINVAL, "ufem_apply: bad precision");
  if (op->P.cg && part != UFEM_PART_ALL)
    return fail(UFEM_EUNSUPPORTED, "ufem_apply_part: the continuous space applies all stages at once");
  const size_t bytes = (size_t)op->P.n_space_dofs() * (precision == UFEM_F64 ? 8 : 4);
  if (overlap(u, v, bytes)) return fail(UFEM_EINVAL, "ufem_apply: u and v overlap");
  DeviceGuard g(op->device);
  hipError_t e = run_apply_p(op, precision, part, u, v, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(e, "ufem_apply: launch");
  return UFEM_OK;
}

int ufem_apply_adjoint(ufem_op* op, int32_t precision, const void* w, const void* u, void* ATw, void* dkappa,
                       void* stream) {
  if (!op || !w || !u || !ATw) return fail(UFEM_EINVAL, "ufem_apply_adjoint: null argument");
  if (precision != UFEM_F64 && precision != UFEM_F32) return fail(UFEM_EINVAL, "ufem_apply_adjoint: bad precision");
  const size_t s = precision == UFEM_F64 ? 8 : 4;
  const size_t bytes = (size_t)op->P.n_space_dofs() * s;
  if (overlap(w, ATw, bytes) || overlap(u, ATw, bytes)) return fail(UFEM_EINVAL, "ufem_apply_adjoint: output overlaps input");
  if (dkappa) {
    const size_t kb = (size_t)op->P.seg[5] * s;
    if (overlap2(dkappa, kb, ATw, bytes) || overlap2(dkappa, kb, w, bytes) || overlap2(dkappa, kb, u, bytes))
      return fail(UFEM_EINVAL, "ufem_apply_adjoint: dkappa overlaps a vector");
  }
  DeviceGuard g(op->device);
  hipError_t e = precision == UFEM_F64
                     ? run_apply<double>(op, precision, 15, w, ATw, u, dkappa, true, (hipStream_t)stream)
                     : run_apply<float>(op, precision, 15, w, ATw, u, dkappa, true, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(e, "ufem_apply_adjoint: launch");
  return UFEM_OK;
}

int ufem_cg_iterate(ufem_op* op, int32_t precision, int32_t n_iter, void* x, void* r, void* p, void* ap, double* scal,
                    void* stream) {
  if (!op || !x || !r || !p || !ap || !scal) return fail(UFEM_EINVAL, "ufem_cg_iterate: null argument");
  if (n_iter < 0) return fail(UFEM_EINVAL, "ufem_cg_iterate: n_iter < 0");
  if (precision != UFEM_F64 && precision != UFEM_F32) return fail(UFEM_EINVAL, "ufem_cg_iterate: bad precision");
  const size_t bytes = (size_t)op->P.n_space_dofs() * (precision == UFEM_F64 ? 8 : 4);
  const void* vec[4] = {x, r, p, ap};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (overlap(vec[i], vec[j], bytes)) return fail(UFEM_EINVAL, "ufem_cg_iterate: vectors overlap");
  for (int i = 0; i < 4; ++i)
    if (overlap2(scal, 4 * sizeof(double), vec[i], bytes)) return fail(UFEM_EINVAL, "ufem_cg_iterate: scal overlaps a vector");
  DeviceGuard g(op->device);
  const int64_t n = op->P.n_space_dofs();
  for (int it = 0; it < n_iter; ++it) {
    hipError_t e = run_apply_p(op, precision, 15, p, ap, (hipStream_t)stream);
    if (e != hipSuccess) return hipfail(e, "ufem_cg_iterate: apply");
    e = ufem::launch_cg_tail(precision, n, x, r, p, ap, scal, (hipStream_t)stream);
    if (e != hipSuccess) return hipfail(e, "ufem_cg_iterate: vector update");
  }
  return UFEM_OK;
}

int ufem_cg_iterate_static(ufem_op* op, int32_t precision, int32_t n_iter, void* x, void* r, void* p,
                           double* result, void* stream) {
  if (!op || !x || !r || !p || !result) return fail(UFEM_EINVAL, "ufem_cg_iterate_static: null argument");
  if (n_iter < 0) return fail(UFEM_EINVAL, "ufem_cg_iterate_static: n_iter < 0");
  if (precision != UFEM_F64 && precision != UFEM_F32) return fail(UFEM_EINVAL, "ufem_cg_iterate_static: bad precision");
  const size_t s = precision == UFEM_F64 ? 8 : 4;
  const size_t bytes = (size_t)op->P.n_space_dofs() * s;
  if (bytes > ufem::kStaticScratchBytes - ufem::kStaticCgScalarBytes)
    return fail(UFEM_EINVAL, "ufem_cg_iterate_static: n_dofs exceeds the static workspace (" +
                                 std::to_string((ufem::kStaticScratchBytes - ufem::kStaticCgScalarBytes) / s) +
                                 " values of this precision)");
  const void* vec[3] = {x, r, p};
  for (int i = 0; i < 3; ++i) {
    for (int j = i + 1; j < 3; ++j)
      if (overlap(vec[i], vec[j], bytes)) return fail(UFEM_EINVAL, "ufem_cg_iterate_static: vectors overlap");
    if (overlap2(result, 2 * sizeof(double), vec[i], bytes))
      return fail(UFEM_EINVAL, "ufem_cg_iterate_static: result overlaps a vector");
  }
  char* ws = (char*)static_scratch(op->device);
  if (!ws) return fail(UFEM_ESTATE, "ufem_cg_iterate_static: no workspace address for the operator's device");
  double* scal = (double*)ws;
  void* ap = ws + ufem::kStaticCgScalarBytes;
  DeviceGuard g(op->device);
  const int64_t n = op->P.n_space_dofs();
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = ufem::launch_cg_static_begin(precision, n, r, scal, st);
  if (e != hipSuccess) return hipfail(e, "ufem_cg_iterate_static: r.r");
  for (int it = 0; it < n_iter; ++it) {
    e = run_apply_p(op, precision, 15, p, ap, st);
    if (e != hipSuccess) return hipfail(e, "ufem_cg_iterate_static: apply");
    e = ufem::launch_cg_tail(precision, n, x, r, p, ap, scal, st);
    if (e != hipSuccess) return hipfail(e, "ufem_cg_iterate_static: vector update");
  }
  e = ufem::launch_cg_static_end(scal, result, st);
  if (e != hipSuccess) return hipfail(e, "ufem_cg_iterate_static: result");
  return UFEM_OK;
}

int ufem_dot(int32_t precision, int64_t n, const void* x, const void* y, double* out, void* stream) {
  if (!x || !y || !out || n < 0) return fail(UFEM_EINVAL, "ufem_dot: bad argument");
  if (precision != UFEM_F64 && precision != UFEM_F32) return fail(UFEM_EINVAL, "ufem_dot: bad precision");
  hipError_t e = ufem::launch_dot(precision, n, x, y, out, (hipStream_t)stream);
  return e == hipSuccess ? UFEM_OK : hipfail(e, "ufem_dot");
}

int ufem_axpby(int32_t precision, int64_t n, double a, const void* x, double b, void* y, void* stream) {
  if (!x || !y || n < 0) return fail(UFEM_EINVAL, "ufem_axpby: bad argument");
  if (precision != UFEM_F64 && precision != UFEM_F32) return fail(UFEM_EINVAL, "ufem_axpby: bad precision");
  hipError_t e = ufem::launch_axpby(precision, n, a, x, b, y, (hipStream_t)stream);
  return e == hipSuccess ? UFEM_OK : hipfail(e, "ufem_axpby");
}

int ufem_cast(int32_t pin, int32_t pout, int64_t n, const void* x, void* y, void* stream) {
  if (!x || !y || n < 0) return fail(UFEM_EINVAL, "ufem_cast: bad argument");
  if ((pin != UFEM_F64 && pin != UFEM_F32) || (pout != UFEM_F64 && pout != UFEM_F32))
    return fail(UFEM_EINVAL, "ufem_cast: bad precision");
  const size_t si = pin == UFEM_F64 ? 8 : 4, so = pout == UFEM_F64 ? 8 : 4;
  if (n > 0 && overlap2(x, (size_t)n * si, y, (size_t)n * so)) return fail(UFEM_EINVAL, "ufem_cast: x and y overlap");
  hipError_t e = ufem::launch_cast(pin, pout, n, x, y, (hipStream_t)stream);
  return e == hipSuccess ? UFEM_OK : hipfail(e, "ufem_cast");
}

}  // extern "C"
