// Host plan: classification, faces, dimension-reduction quadrature (Saye
// 2015, cited in Sections 1 and 2.3 of the paper) and the quadrature-point
// layout.
//
// Quadrature reading (the paper gives no steps of its own):
//  TOP problem on a box (integrate over {phi < 0}): prune balls that stay
//  away from the box; a ball containing the box gives the tensor Gauss rule;
//  the height direction is the free axis, among those along which every
//  remaining ball is strictly monotone, with the largest sum of |d psi/dx_k|
//  at the box centre (lowest axis on ties); with none, bisect along every
//  free axis (up to max_depth, then the tensor rule filtered by phi < 0);
//  otherwise a rule of the lower face split at the zero sets of the balls
//  restricted to the two end values of the height axis (SPLIT problem), and
//  along each line Gauss rules on the pieces between the closed-form roots
//  whose midpoint has phi < 0, and interface points at the roots where the
//  root's ball is the active minimum.
//  SPLIT problem (integrate over the whole box): drop functions of one sign;
//  with none left or in 1D, Gauss rules on the pieces between roots;
//  otherwise the same recursion with every piece kept.
//  A plane psi = n . x - c (unit n, one function) takes the same steps: its
//  bounds on a box are its values at the extreme corners, it is strictly
//  monotone along every axis with n_k != 0, the height criterion is |n_k|,
//  the root along a line is (c - sum_{a != k} n_a x_a) / n_k, and an
//  interface point has weight w' / |n_k| and normal n.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

// Every product and sum is rounded on its own (no fused multiply-add), so
// that the decisions on signs (classes, pieces, active roots) follow the
// plain arithmetic of the method.
#pragma clang fp contract(off)

namespace ufem {

// ------------------------------------------------------------- 1D rules
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration on P_n from the Chebyshev guesses, mapped to [0, 1]
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = t; p0 = 1.0; }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    // recompute the derivative at the converged root
    double p0 = 1.0, p1 = t;
    for (int j = 2; j <= n; ++j) {
      double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = t; p0 = 1.0; }
    dp = n * (t * p1 - p0) / (t * t - 1.0);
    x[n - 1 - i] = 0.5 * (t + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);
  }
  // symmetrise
  for (int i = 0; i < n / 2; ++i) {
    double a = 0.5 * (x[i] + (1.0 - x[n - 1 - i]));
    x[i] = a;
    x[n - 1 - i] = 1.0 - a;
    double b = 0.5 * (w[i] + w[n - 1 - i]);
    w[i] = b;
    w[n - 1 - i] = b;
  }
  if (n % 2 == 1) x[n / 2] = 0.5;
}

void gauss_lobatto01(int n, std::vector<double>& x) {
  // Newton iteration for the roots of (1 - t^2) P'_{N}(t), N = n - 1, using
  // t P_N - P_{N-1} = 0 (Chebyshev-Gauss-Lobatto start)
  const int N = n - 1;
  std::vector<double> t(n);
  for (int i = 0; i < n; ++i) t[i] = -std::cos(M_PI * i / N);
  for (int i = 1; i < N; ++i) {
    double ti = t[i];
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = ti;
      for (int j = 2; j <= N; ++j) {
        double p2 = ((2.0 * j - 1.0) * ti * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (N == 1) { p1 = ti; p0 = 1.0; }
      // f = t P_N - P_{N-1}, f' = (N + 1) P_N
      double f = ti * p1 - p0;
      double fp = (N + 1) * p1;
      double dt = f / fp;
      ti -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    t[i] = ti;
  }
  x.assign(n, 0.0);
  for (int i = 0; i < n; ++i) x[i] = 0.5 * (t[i] + 1.0);
  x[0] = 0.0;
  x[n - 1] = 1.0;
  for (int i = 1; i < n / 2; ++i) {
    double a = 0.5 * (x[i] + (1.0 - x[n - 1 - i]));
    x[i] = a;
    x[n - 1 - i] = 1.0 - a;
  }
  if (n % 2 == 1) x[n / 2] = 0.5;
}

void lagrange_all(const std::vector<double>& nodes, double z, int maxd, std::vector<double>& out) {
  // Fornberg's recursion for the weights of the derivatives of the
  // interpolating polynomial at z: c[j][d] = L_j^(d)(z)
  const int n = (int)nodes.size();
  const int m = maxd;
  std::vector<double> c((size_t)n * (m + 1), 0.0);
  auto C = [&](int j, int d) -> double& { return c[(size_t)j * (m + 1) + d]; };
  double c1 = 1.0, c4 = nodes[0] - z;
  C(0, 0) = 1.0;
  for (int i = 1; i < n; ++i) {
    int mn = std::min(i, m);
    double c2 = 1.0, c5 = c4;
    c4 = nodes[i] - z;
    for (int j = 0; j < i; ++j) {
      double c3 = nodes[i] - nodes[j];
      c2 *= c3;
      if (j == i - 1) {
        for (int d = mn; d >= 1; --d) C(i, d) = c1 * (d * C(i - 1, d - 1) - c5 * C(i - 1, d)) / c2;
        C(i, 0) = -c1 * c5 * C(i - 1, 0) / c2;
      }
      for (int d = mn; d >= 1; --d) C(j, d) = (c4 * C(j, d) - d * C(j, d - 1)) / c3;
      C(j, 0) = c4 * C(j, 0) / c3;
    }
    c1 = c2;
  }
  out.assign((size_t)(m + 1) * n, 0.0);
  for (int d = 0; d <= m; ++d)
    for (int j = 0; j < n; ++j) out[(size_t)d * n + j] = C(j, d);
}

void Plan::cell_lo(int32_t b, double* x) const {
  int32_t r = b;
  for (int a = 0; a < dim; ++a) {
    x[a] = lo + (r % n) * h;
    r /= n;
  }
}

// ---------------------------------------------------------- quadrature
namespace {

struct Fn {
  int ball;
  double vals[3];  // coordinates of the axes that are not free
};

struct Rule {
  std::vector<double> vx, vw;          // volume points (3 doubles each), weights
  std::vector<double> sx, sw, sn;      // interface points, weights, normals
};

class Saye {
 public:
  Saye(const Plan& P)
      : dim_(P.dim), q_(P.q), maxd_(P.max_depth), c_(P.centers), r_(P.radii), plane_(P.plane), pc_(P.pc) {
    for (int a = 0; a < 3; ++a) pn_[a] = P.pn[a];
    gauss_legendre01(q_, gx_, gw_);
  }
  int64_t n_fallback = 0;

  // volume + interface rule of the box [lo, hi] (physical)
  void cell(const double* lo, const double* hi, Rule& out) {
    double L[3] = {0, 0, 0}, H[3] = {0, 0, 0}, base[3] = {0, 0, 0};
    for (int a = 0; a < dim_; ++a) { L[a] = lo[a]; H[a] = hi[a]; base[a] = lo[a]; }
    std::vector<Fn> fs;
    for (int i = 0; i < nfun(); ++i) {
      Fn f;
      f.ball = i;
      for (int a = 0; a < 3; ++a) f.vals[a] = base[a];
      fs.push_back(f);
    }
    top(fs, L, H, (1 << dim_) - 1, base, 0, true, out);
  }
  // rule of the face x_axis = value of the box [lo, hi]
  void face(const double* lo, const double* hi, int axis, double value, Rule& out) {
    double L[3] = {0, 0, 0}, H[3] = {0, 0, 0}, base[3] = {0, 0, 0};
    for (int a = 0; a < dim_; ++a) { L[a] = lo[a]; H[a] = hi[a]; base[a] = lo[a]; }
    base[axis] = value;
    L[axis] = value;
    H[axis] = value;
    std::vector<Fn> fs;
    for (int i = 0; i < nfun(); ++i) {
      Fn f;
      f.ball = i;
      for (int a = 0; a < 3; ++a) f.vals[a] = base[a];
      fs.push_back(f);
    }
    int free = ((1 << dim_) - 1) & ~(1 << axis);
    top(fs, L, H, free, base, 0, false, out);
  }

 private:
  int dim_, q_, maxd_;
  const std::vector<double>& c_;
  const std::vector<double>& r_;
  bool plane_;
  double pn_[3], pc_;
  std::vector<double> gx_, gw_;

  int nfun() const { return plane_ ? 1 : (int)r_.size(); }
  const double* cen(int i) const { return &c_[(size_t)i * dim_]; }
  static bool isfree(int free, int a) { return (free >> a) & 1; }

  void bounds(const Fn& f, const double* lo, const double* hi, int free, double& mn, double& mx) const {
    if (plane_) {
      double s0 = 0.0, s1 = 0.0;
      for (int a = 0; a < dim_; ++a) {
        if (isfree(free, a)) {
          s0 += pn_[a] > 0 ? pn_[a] * lo[a] : pn_[a] * hi[a];
          s1 += pn_[a] > 0 ? pn_[a] * hi[a] : pn_[a] * lo[a];
        } else {
          s0 += pn_[a] * f.vals[a];
          s1 += pn_[a] * f.vals[a];
        }
      }
      mn = s0 - pc_;
      mx = s1 - pc_;
      return;
    }
    const double* c = cen(f.ball);
    double near2 = 0.0, far2 = 0.0;
    for (int a = 0; a < dim_; ++a) {
      double nz, fz;
      if (isfree(free, a)) {
        nz = std::min(std::max(c[a], lo[a]), hi[a]) - c[a];
        fz = std::max(std::fabs(lo[a] - c[a]), std::fabs(hi[a] - c[a]));
      } else {
        nz = f.vals[a] - c[a];
        fz = std::fabs(f.vals[a] - c[a]);
      }
      near2 += nz * nz;
      far2 += fz * fz;
    }
    mn = std::sqrt(near2) - r_[f.ball];
    mx = std::sqrt(far2) - r_[f.ball];
  }
  double coord(const Fn& f, const double* x, int free, int a) const { return isfree(free, a) ? x[a] : f.vals[a]; }
  double psi(const Fn& f, const double* x, int free) const {
    if (plane_) {
      double s = 0.0;
      for (int a = 0; a < dim_; ++a) s += pn_[a] * coord(f, x, free, a);
      return s - pc_;
    }
    const double* c = cen(f.ball);
    double s = 0.0;
    for (int a = 0; a < dim_; ++a) {
      double z = coord(f, x, free, a) - c[a];
      s += z * z;
    }
    return std::sqrt(s) - r_[f.ball];
  }
  bool monotone(const Fn& f, int k, const double* lo, const double* hi) const {
    if (plane_) return pn_[k] != 0.0;
    double ck = cen(f.ball)[k];
    return ck < lo[k] || ck > hi[k];
  }
  int height(const std::vector<Fn>& fs, const double* lo, const double* hi, int free) const {
    int best = -1;
    double bestval = -1.0;
    for (int k = 0; k < dim_; ++k) {
      if (!isfree(free, k)) continue;
      bool ok = true;
      for (const Fn& f : fs)
        if (!monotone(f, k, lo, hi)) { ok = false; break; }
      if (!ok) continue;
      double val = 0.0;
      for (const Fn& f : fs) {
        if (plane_) {
          val += std::fabs(pn_[k]);
          continue;
        }
        const double* c = cen(f.ball);
        double s = 0.0;
        for (int a = 0; a < dim_; ++a) {
          double xa = isfree(free, a) ? 0.5 * (lo[a] + hi[a]) : f.vals[a];
          s += (xa - c[a]) * (xa - c[a]);
        }
        double r = std::sqrt(s);
        if (r > 0.0) val += std::fabs((0.5 * (lo[k] + hi[k]) - c[k]) / r);
      }
      if (val > bestval) { best = k; bestval = val; }
    }
    return best;
  }
  struct Root { double t; int fi; };
  void roots(const std::vector<Fn>& fs, const double* x, int free, int k, double a, double b,
             std::vector<Root>& out) const {
    out.clear();
    for (int fi = 0; fi < (int)fs.size(); ++fi) {
      const Fn& f = fs[fi];
      if (plane_) {
        if (pn_[k] == 0.0) continue;
        double s = 0.0;
        for (int ax = 0; ax < dim_; ++ax)
          if (ax != k) s += pn_[ax] * coord(f, x, free, ax);
        const double t = (pc_ - s) / pn_[k];
        if (a < t && t < b) out.push_back({t, fi});
        continue;
      }
      const double* c = cen(f.ball);
      double s = 0.0;
      for (int ax = 0; ax < dim_; ++ax) {
        if (ax == k) continue;
        double z = coord(f, x, free, ax) - c[ax];
        s += z * z;
      }
      double D = r_[f.ball] * r_[f.ball] - s;
      if (D < 0.0) continue;
      double sq = std::sqrt(D);
      double t0 = c[k] - sq, t1 = c[k] + sq;
      if (a < t0 && t0 < b) out.push_back({t0, fi});
      if (a < t1 && t1 < b) out.push_back({t1, fi});
    }
    std::stable_sort(out.begin(), out.end(), [](const Root& u, const Root& v) { return u.t < v.t; });
  }
  void tensor(const double* lo, const double* hi, int free, const double* base,
              std::vector<double>& px, std::vector<double>& pw) const {
    int fr[3], m = 0;
    for (int a = 0; a < dim_; ++a)
      if (isfree(free, a)) fr[m++] = a;
    int total = 1;
    for (int j = 0; j < m; ++j) total *= q_;
    for (int idx = 0; idx < total; ++idx) {
      double x[3] = {base[0], base[1], base[2]};
      double w = 1.0;
      int rem = idx;
      for (int j = 0; j < m; ++j) {
        int a = fr[j];
        int g = rem % q_;
        rem /= q_;
        double L = hi[a] - lo[a];
        x[a] = lo[a] + L * gx_[g];
        w *= L * gw_[g];
      }
      px.insert(px.end(), x, x + 3);
      pw.push_back(w);
    }
  }
  template <class F>
  void children(const double* lo, const double* hi, int free, F&& fn) const {
    int fr[3], m = 0;
    for (int a = 0; a < dim_; ++a)
      if (isfree(free, a)) fr[m++] = a;
    for (int cidx = 0; cidx < (1 << m); ++cidx) {
      double clo[3] = {lo[0], lo[1], lo[2]}, chi[3] = {hi[0], hi[1], hi[2]};
      for (int j = 0; j < m; ++j) {
        int a = fr[j];
        double mid = 0.5 * (lo[a] + hi[a]);
        if ((cidx >> j) & 1) clo[a] = mid; else chi[a] = mid;
      }
      fn(clo, chi);
    }
  }
  static int popc(int v) { int c = 0; while (v) { c += v & 1; v >>= 1; } return c; }
  static int lowest(int v) { int a = 0; while (!((v >> a) & 1)) ++a; return a; }

  void split(const std::vector<Fn>& fs, const double* lo, const double* hi, int free, const double* base, int depth,
             std::vector<double>& px, std::vector<double>& pw) {
    std::vector<Fn> keep;
    for (const Fn& f : fs) {
      double mn, mx;
      bounds(f, lo, hi, free, mn, mx);
      if (mn < 0.0 && 0.0 < mx) keep.push_back(f);
    }
    if (keep.empty()) { tensor(lo, hi, free, base, px, pw); return; }
    std::vector<Root> rts;
    if (popc(free) == 1) {
      int k = lowest(free);
      double x[3] = {base[0], base[1], base[2]};
      roots(keep, x, free, k, lo[k], hi[k], rts);
      double e0 = lo[k];
      for (size_t r = 0; r <= rts.size(); ++r) {
        double e1 = r < rts.size() ? rts[r].t : hi[k];
        if (e1 > e0) {
          double L = e1 - e0;
          for (int g = 0; g < q_; ++g) {
            double y[3] = {x[0], x[1], x[2]};
            y[k] = e0 + L * gx_[g];
            px.insert(px.end(), y, y + 3);
            pw.push_back(L * gw_[g]);
          }
        }
        e0 = e1;
      }
      return;
    }
    int k = height(keep, lo, hi, free);
    if (k < 0) {
      if (depth < maxd_) {
        children(lo, hi, free, [&](const double* clo, const double* chi) {
          split(keep, clo, chi, free, base, depth + 1, px, pw);
        });
        return;
      }
      ++n_fallback;
      tensor(lo, hi, free, base, px, pw);
      return;
    }
    std::vector<Fn> fs2;
    for (const Fn& f : keep) {
      Fn flo = f, fhi = f;
      flo.vals[k] = lo[k];
      fhi.vals[k] = hi[k];
      fs2.push_back(flo);
      fs2.push_back(fhi);
    }
    std::vector<double> bx, bw;
    split(fs2, lo, hi, free & ~(1 << k), base, 0, bx, bw);
    for (size_t bi = 0; bi < bw.size(); ++bi) {
      const double* x = &bx[bi * 3];
      roots(keep, x, free, k, lo[k], hi[k], rts);
      double e0 = lo[k];
      for (size_t r = 0; r <= rts.size(); ++r) {
        double e1 = r < rts.size() ? rts[r].t : hi[k];
        if (e1 > e0) {
          double L = e1 - e0;
          for (int g = 0; g < q_; ++g) {
            double y[3] = {x[0], x[1], x[2]};
            y[k] = e0 + L * gx_[g];
            px.insert(px.end(), y, y + 3);
            pw.push_back(bw[bi] * (L * gw_[g]));
          }
        }
        e0 = e1;
      }
    }
  }

  void line(const std::vector<Fn>& rel, const double* x, double w, int free, int k, double a, double b, bool surf,
            Rule& out) {
    std::vector<Root> rts;
    roots(rel, x, free, k, a, b, rts);
    double e0 = a;
    for (size_t r = 0; r <= rts.size(); ++r) {
      double e1 = r < rts.size() ? rts[r].t : b;
      if (e1 > e0) {
        double y[3] = {x[0], x[1], x[2]};
        y[k] = 0.5 * (e0 + e1);
        double mn = 1e300;
        for (const Fn& f : rel) mn = std::min(mn, psi(f, y, free));
        if (mn < 0.0) {
          double L = e1 - e0;
          for (int g = 0; g < q_; ++g) {
            double z[3] = {x[0], x[1], x[2]};
            z[k] = e0 + L * gx_[g];
            out.vx.insert(out.vx.end(), z, z + 3);
            out.vw.push_back(w * (L * gw_[g]));
          }
        }
      }
      e0 = e1;
    }
    if (!surf) return;
    for (const Root& rt : rts) {
      double y[3] = {x[0], x[1], x[2]};
      y[k] = rt.t;
      bool active = true;
      for (int gi = 0; gi < (int)rel.size(); ++gi)
        if (gi != rt.fi && psi(rel[gi], y, free) < 0.0) { active = false; break; }
      if (!active) continue;
      if (plane_) {
        out.sx.insert(out.sx.end(), y, y + 3);
        out.sw.push_back(w / std::fabs(pn_[k]));
        for (int ax = 0; ax < 3; ++ax) out.sn.push_back(ax < dim_ ? pn_[ax] : 0.0);
        continue;
      }
      const Fn& f = rel[rt.fi];
      const double* c = cen(f.ball);
      double d[3] = {0, 0, 0}, s = 0.0;
      for (int ax = 0; ax < dim_; ++ax) {
        d[ax] = coord(f, y, free, ax) - c[ax];
        s += d[ax] * d[ax];
      }
      double r = std::sqrt(s);
      out.sx.insert(out.sx.end(), y, y + 3);
      out.sw.push_back(w * (r / std::fabs(rt.t - c[k])));
      for (int ax = 0; ax < 3; ++ax) out.sn.push_back(ax < dim_ ? d[ax] / r : 0.0);
    }
  }

  void top(const std::vector<Fn>& fs, const double* lo, const double* hi, int free, const double* base, int depth,
           bool surf, Rule& out) {
    std::vector<Fn> rel;
    for (const Fn& f : fs) {
      double mn, mx;
      bounds(f, lo, hi, free, mn, mx);
      if (mx < 0.0) { tensor(lo, hi, free, base, out.vx, out.vw); return; }
      if (mn < 0.0) rel.push_back(f);
    }
    if (rel.empty()) return;
    if (popc(free) == 1) {
      int k = lowest(free);
      line(rel, base, 1.0, free, k, lo[k], hi[k], surf, out);
      return;
    }
    int k = height(rel, lo, hi, free);
    if (k < 0) {
      if (depth < maxd_) {
        children(lo, hi, free, [&](const double* clo, const double* chi) {
          top(rel, clo, chi, free, base, depth + 1, surf, out);
        });
        return;
      }
      ++n_fallback;
      std::vector<double> px, pw;
      tensor(lo, hi, free, base, px, pw);
      for (size_t i = 0; i < pw.size(); ++i) {
        double mn = 1e300;
        for (const Fn& f : rel) mn = std::min(mn, psi(f, &px[i * 3], free));
        if (mn < 0.0) {
          out.vx.insert(out.vx.end(), &px[i * 3], &px[i * 3] + 3);
          out.vw.push_back(pw[i]);
        }
      }
      return;
    }
    std::vector<Fn> fs2;
    for (const Fn& f : rel) {
      Fn flo = f, fhi = f;
      flo.vals[k] = lo[k];
      fhi.vals[k] = hi[k];
      fs2.push_back(flo);
      fs2.push_back(fhi);
    }
    std::vector<double> bx, bw;
    split(fs2, lo, hi, free & ~(1 << k), base, 0, bx, bw);
    for (size_t bi = 0; bi < bw.size(); ++bi) line(rel, &bx[bi * 3], bw[bi], free, k, lo[k], hi[k], surf, out);
  }
};

int box_class(const Plan& P, const double* lo, const double* hi) {
  if (P.plane) {
    double mn = 0.0, mx = 0.0;
    for (int a = 0; a < P.dim; ++a) {
      mn += P.pn[a] > 0 ? P.pn[a] * lo[a] : P.pn[a] * hi[a];
      mx += P.pn[a] > 0 ? P.pn[a] * hi[a] : P.pn[a] * lo[a];
    }
    mn -= P.pc;
    mx -= P.pc;
    return mx < 0.0 ? kInside : (mn < 0.0 ? kCut : kOutside);
  }
  bool touch = false;
  for (size_t i = 0; i < P.radii.size(); ++i) {
    const double* c = &P.centers[i * P.dim];
    double near2 = 0.0, far2 = 0.0;
    for (int a = 0; a < P.dim; ++a) {
      double nz = std::min(std::max(c[a], lo[a]), hi[a]) - c[a];
      double fz = std::max(std::fabs(lo[a] - c[a]), std::fabs(hi[a] - c[a]));
      near2 += nz * nz;
      far2 += fz * fz;
    }
    if (std::sqrt(far2) < P.radii[i]) return kInside;
    if (std::sqrt(near2) < P.radii[i]) touch = true;
  }
  return touch ? kCut : kOutside;
}

template <class F>
void parallel_for(int64_t n, F&& fn) {
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (n < 64 || nt == 1) {
    fn(0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([&, a, b, t] { fn(a, b, (int)t); });
  }
  for (auto& t : th) t.join();
}


// Runs of consecutive points [begin, end) (stride `nc` coordinates) in which
// every point differs from the first one in the same single coordinate.
void group_lines(const std::vector<double>& x, int nc, int64_t begin, int64_t end, int kind, int default_axis,
                 Plan& P) {
  int64_t i = begin;
  while (i < end) {
    int64_t j = i + 1;
    int axis = -1;
    while (j < end && j - i < 4096) {
      int ndiff = 0, dax = -1;
      for (int a = 0; a < nc; ++a)
        if (x[j * nc + a] != x[i * nc + a]) { ++ndiff; dax = a; }
      if (ndiff != 1) break;
      if (axis < 0) axis = dax;
      else if (dax != axis) break;
      ++j;
    }
    P.line_first.push_back((int32_t)i);
    P.line_n.push_back((int32_t)(j - i));
    P.line_axis.push_back(axis < 0 ? default_axis : axis);
    P.line_kind.push_back(kind);
    i = j;
  }
}

}  // namespace

// Point lines and the kappa layout from the cut rules in P (vol / surf /
// fcut arrays with their offsets); shared by build_plan and the import of
// explicit rules.
std::string finish_rules(Plan& P, int* code) {
  const int dim = P.dim;
  const size_t ncut = P.cut.size();
  const std::vector<int32_t>& cutfaces = P.fcut_face;
  P.max_qp_cut_cell = 0;
  for (size_t i = 0; i < ncut; ++i) P.max_qp_cut_cell = std::max<int64_t>(P.max_qp_cut_cell, P.vol_off[i + 1] - P.vol_off[i]);
  // -- point lines
  if (P.vol_w.size() > 0x7fffffffu || P.surf_w.size() > 0x7fffffffu || P.fcut_w.size() > 0x7fffffffu) {
    *code = UFEM_EUNSUPPORTED;
    return "too many cut quadrature points for 32-bit point indices";
  }
  P.line_first.clear(); P.line_n.clear(); P.line_axis.clear(); P.line_kind.clear();
  P.cell_line_off.assign(ncut + 1, 0);
  for (size_t i = 0; i < ncut; ++i) {
    const size_t l0 = P.line_first.size();
    group_lines(P.vol_x, dim, P.vol_off[i], P.vol_off[i + 1], 0, dim - 1, P);
    // interface points: one-point lines along the cell's most frequent axis
    int cnt[3] = {0, 0, 0};
    for (size_t l = l0; l < P.line_first.size(); ++l) cnt[P.line_axis[l]] += P.line_n[l];
    int dom = dim - 1;
    for (int a = 0; a < dim; ++a)
      if (cnt[a] > cnt[dom]) dom = a;
    for (int64_t q = P.surf_off[i]; q < P.surf_off[i + 1]; ++q) {
      P.line_first.push_back((int32_t)q);
      P.line_n.push_back(1);
      P.line_axis.push_back(dom);
      P.line_kind.push_back(1);
    }
    P.cell_line_off[i + 1] = (int64_t)P.line_first.size();
  }
  P.face_line_off.assign(cutfaces.size() + 1, P.cell_line_off[ncut]);
  for (size_t i = 0; i < cutfaces.size(); ++i) {
    group_lines(P.fcut_x, dim - 1, P.fcut_off[i], P.fcut_off[i + 1], 2, 0, P);
    P.face_line_off[i + 1] = (int64_t)P.line_first.size();
  }

  // -- volume ghost penalty with stable neighbours: the faces of the patches
  // (each cut cell with the face neighbour of largest volume fraction; a
  // later slot wins only by more than 1e-10)
  if (P.gp_kind == UFEM_GP_VOLUME) {
    std::vector<double> frac(P.active.size(), 1.0);
    for (size_t i = 0; i < ncut; ++i) {
      double s = 0.0;
      for (int64_t q = P.vol_off[i]; q < P.vol_off[i + 1]; ++q) s += P.vol_w[q];
      frac[P.cut[i]] = s;
    }
    for (Face& f : P.faces) f.gp = 0;
    const int S = 2 * dim;
    for (size_t i = 0; i < ncut; ++i) {
      const int32_t r = P.cut[i];
      int32_t best_fi = -1;
      double best_f = 0.0;
      for (int sl = 0; sl < S; ++sl) {
        const int32_t fi = P.slot_face[(size_t)r * S + sl];
        if (fi < 0) continue;
        const Face& f = P.faces[fi];
        const int32_t nb = P.rank[(sl & 1) ? f.bp : f.bm];
        if (best_fi < 0 || frac[nb] > best_f + 1e-10) {
          best_fi = fi;
          best_f = frac[nb];
        }
      }
      if (best_fi >= 0) P.faces[best_fi].gp = 1;
    }
  }

  // -- kappa layout
  const int nd = P.nd(), nf = P.nf();
  P.seg[0] = 0;
  P.seg[1] = (int64_t)P.inside.size() * nd;
  P.seg[2] = P.seg[1] + P.vol_off[ncut];
  int64_t off = P.seg[2];
  P.n_faces_str = P.n_faces_cut = P.n_faces_gp = 0;
  for (Face& f : P.faces) {
    if (f.gp) ++P.n_faces_gp;
    if (f.kind == kFaceStructured) {
      f.qp_off = off;
      f.qp_n = nf;
      off += nf;
      ++P.n_faces_str;
    }
  }
  P.seg[3] = off;
  for (size_t i = 0; i < cutfaces.size(); ++i) {
    Face& f = P.faces[cutfaces[i]];
    f.qp_off = off + P.fcut_off[i];
    f.qp_n = (int32_t)(P.fcut_off[i + 1] - P.fcut_off[i]);
    ++P.n_faces_cut;
  }
  off += P.fcut_off[cutfaces.size()];
  P.seg[4] = off;
  P.seg[5] = off + P.surf_off[ncut];
  *code = UFEM_OK;
  return std::string();
}

std::string build_plan(const ufem_problem& pr, Plan& P, int* code) {
  *code = UFEM_EINVAL;
  if (pr.dim != 2 && pr.dim != 3) return "dim must be 2 or 3";
  if (pr.n < 2 || pr.n > 4096) return "n must be in [2, 4096]";
  if (!(pr.hi > pr.lo)) return "hi must exceed lo";
  if (pr.degree < 1 || pr.degree > 7) return "degree must be in [1, 7]";
  if (pr.levelset != UFEM_LEVELSET_BALLS && pr.levelset != UFEM_LEVELSET_PLANE) return "unknown level-set kind";
  if (pr.levelset == UFEM_LEVELSET_BALLS && (pr.n_balls < 1 || !pr.centers || !pr.radii))
    return "need at least one ball (centers, radii)";
  if (pr.q_cut < 0 || pr.q_cut > 16) return "q_cut must be in [0, 16]";
  if (pr.gp_jmin < 0 || pr.gp_jmin > pr.degree + 1) return "gp_jmin out of range";
  if (pr.gp_kind != UFEM_GP_FACE && pr.gp_kind != UFEM_GP_VOLUME && pr.gp_kind != UFEM_GP_VOLUME_ALL)
    return "unknown ghost-penalty kind";
  if (pr.space != UFEM_SPACE_DG && pr.space != UFEM_SPACE_CG) return "unknown space";
  double cells = std::pow((double)pr.n, pr.dim);
  if (cells > 2.2e9) return "background mesh too large";
  P.prob = pr;
  P.dim = pr.dim;
  P.n = pr.n;
  P.p = pr.degree;
  P.k = pr.degree + 1;
  P.q = pr.q_cut > 0 ? pr.q_cut : P.k;
  P.max_depth = pr.max_depth < 0 ? 4 : pr.max_depth;
  P.lo = pr.lo;
  P.h = (pr.hi - pr.lo) / pr.n;
  P.plane = pr.levelset == UFEM_LEVELSET_PLANE;
  P.centers.clear();
  P.radii.clear();
  if (P.plane) {
    double s = 0.0;
    for (int a = 0; a < pr.dim; ++a) s += pr.plane_normal[a] * pr.plane_normal[a];
    const double L = std::sqrt(s);
    if (!(L > 0.0) || !std::isfinite(L) || !std::isfinite(pr.plane_offset)) return "plane normal must be nonzero and finite";
    for (int a = 0; a < 3; ++a) P.pn[a] = a < pr.dim ? pr.plane_normal[a] / L : 0.0;
    P.pc = pr.plane_offset / L;
    P.prob.n_balls = 0;
  } else {
    P.centers.assign(pr.centers, pr.centers + (size_t)pr.n_balls * pr.dim);
    P.radii.assign(pr.radii, pr.radii + pr.n_balls);
    for (double r : P.radii)
      if (!(r > 0.0)) return "radii must be positive";
  }
  P.prob.centers = nullptr;
  P.prob.radii = nullptr;
  P.gp_kind = pr.gp_kind;
  P.tau = pr.nitsche_factor * P.p * P.p;
  P.gamma = pr.sipg_factor * P.p * P.p;
  P.gp_w.assign(P.p + 1, 0.0);
  double fact = 1.0;
  for (int j = 0; j <= P.p; ++j) {
    if (j > 0) fact *= j;
    if (j >= pr.gp_jmin) P.gp_w[j] = pr.gp_flat ? pr.gp_gamma : pr.gp_gamma / (fact * fact);
  }

  const int dim = P.dim, n = P.n;
  const int64_t nbg = (int64_t)std::llround(cells);
  // -- classification
  P.cls.assign(nbg, kOutside);
  parallel_for(nbg, [&](int64_t a, int64_t b, int) {
    for (int64_t c = a; c < b; ++c) {
      double lo[3], hi[3];
      P.cell_lo((int32_t)c, lo);
      for (int x = 0; x < dim; ++x) hi[x] = lo[x] + P.h;
      P.cls[c] = (int8_t)box_class(P, lo, hi);
    }
  });
  P.rank.assign(nbg, -1);
  P.active.clear();
  for (int64_t c = 0; c < nbg; ++c)
    if (P.cls[c] != kOutside) {
      P.rank[c] = (int32_t)P.active.size();
      P.active.push_back((int32_t)c);
    }
  if (P.active.empty()) { *code = UFEM_EINVAL; return "the level set leaves no active cell"; }
  if ((int64_t)P.active.size() * P.nd() > (int64_t)2000000000) { *code = UFEM_EUNSUPPORTED; return "too many DoFs"; }
  P.inside.clear();
  P.cut.clear();
  for (size_t r = 0; r < P.active.size(); ++r) (P.cls[P.active[r]] == kInside ? P.inside : P.cut).push_back((int32_t)r);

  // -- continuous space: the node lattice of (n p + 1)^dim Gauss-Lobatto
  // nodes, the nodes of active cells numbered in lattice order
  P.cg = pr.space == UFEM_SPACE_CG;
  P.n_nodes = 0;
  P.cell_node.clear();
  P.node_ptr.clear();
  P.node_src.clear();
  if (P.cg) {
    const int64_t L1 = (int64_t)n * P.p + 1;
    int64_t lat = 1;
    for (int a = 0; a < dim; ++a) lat *= L1;
    if (lat > (int64_t)2000000000) { *code = UFEM_EUNSUPPORTED; return "node lattice too large"; }
    std::vector<int32_t> lat2node((size_t)lat, -1);
    const int nd = P.nd(), K = P.k;
    auto lattice = [&](int32_t b, int l) {
      int64_t g = 0, stride = 1;
      int32_t rem = b;
      int rl = l;
      for (int a = 0; a < dim; ++a) {
        const int64_t I = (int64_t)(rem % n) * P.p + (rl % K);
        rem /= n;
        rl /= K;
        g += I * stride;
        stride *= L1;
      }
      return g;
    };
    for (int32_t b : P.active)
      for (int l = 0; l < nd; ++l) lat2node[(size_t)lattice(b, l)] = 0;
    for (int64_t g = 0; g < lat; ++g)
      if (lat2node[(size_t)g] == 0) lat2node[(size_t)g] = (int32_t)(P.n_nodes++) + 1;
    P.cell_node.resize((size_t)P.n_dofs());
    std::vector<int64_t> cnt((size_t)P.n_nodes + 1, 0);
    for (size_t r = 0; r < P.active.size(); ++r)
      for (int l = 0; l < nd; ++l) {
        const int32_t node = lat2node[(size_t)lattice(P.active[r], l)] - 1;
        P.cell_node[r * nd + l] = node;
        ++cnt[(size_t)node + 1];
      }
    P.node_ptr.assign((size_t)P.n_nodes + 1, 0);
    for (int64_t i = 0; i < P.n_nodes; ++i) P.node_ptr[i + 1] = P.node_ptr[i] + cnt[(size_t)i + 1];
    P.node_src.assign((size_t)P.n_dofs(), 0);
    std::vector<int64_t> fill(P.node_ptr.begin(), P.node_ptr.end() - 1);
    for (int64_t i = 0; i < P.n_dofs(); ++i) P.node_src[(size_t)fill[(size_t)P.cell_node[i]]++] = i;
  }

  // -- faces
  int64_t stride[3] = {1, n, (int64_t)n * n};
  P.faces.clear();
  P.slot_face.assign(P.active.size() * 2 * dim, -1);
  for (size_t r = 0; r < P.active.size(); ++r) {
    int32_t b = P.active[r];
    int ijk[3] = {0, 0, 0};
    int32_t rem = b;
    for (int a = 0; a < dim; ++a) { ijk[a] = rem % n; rem /= n; }
    for (int a = 0; a < dim; ++a) {
      if (ijk[a] + 1 >= n) continue;
      int32_t bp = (int32_t)(b + stride[a]);
      if (P.cls[bp] == kOutside) continue;
      double lo[3], hi[3];
      P.cell_lo(b, lo);
      for (int x = 0; x < dim; ++x) hi[x] = lo[x] + P.h;
      double flo[3] = {lo[0], lo[1], lo[2]};
      flo[a] = hi[a];
      int fc = box_class(P, flo, hi);
      Face f;
      f.bm = b;
      f.bp = bp;
      f.axis = a;
      f.kind = fc == kInside ? kFaceStructured : (fc == kCut ? kFaceCut : kFaceNone);
      f.gp = (P.cls[b] == kCut || P.cls[bp] == kCut) ? 1 : 0;
      f.qp_off = -1;
      f.qp_n = 0;
      int32_t fi = (int32_t)P.faces.size();
      P.faces.push_back(f);
      P.slot_face[r * 2 * dim + 2 * a + 1] = fi;
      P.slot_face[(size_t)P.rank[bp] * 2 * dim + 2 * a + 0] = fi;
    }
  }

  // -- cut-cell rules (parallel over cut cells, concatenated in cut order)
  const size_t ncut = P.cut.size();
  std::vector<Rule> rules(ncut);
  std::vector<int64_t> fallbacks(64, 0);
  parallel_for((int64_t)ncut, [&](int64_t a, int64_t b, int t) {
    Saye S(P);
    for (int64_t i = a; i < b; ++i) {
      int32_t bg = P.active[P.cut[i]];
      double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      P.cell_lo(bg, lo);
      for (int x = 0; x < dim; ++x) hi[x] = lo[x] + P.h;
      S.cell(lo, hi, rules[i]);
    }
    fallbacks[t] += S.n_fallback;
  });
  // cut faces
  std::vector<int32_t> cutfaces;
  for (size_t fi = 0; fi < P.faces.size(); ++fi)
    if (P.faces[fi].kind == kFaceCut) cutfaces.push_back((int32_t)fi);
  std::vector<Rule> frules(cutfaces.size());
  parallel_for((int64_t)cutfaces.size(), [&](int64_t a, int64_t b, int t) {
    Saye S(P);
    for (int64_t i = a; i < b; ++i) {
      const Face& f = P.faces[cutfaces[i]];
      double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      P.cell_lo(f.bm, lo);
      for (int x = 0; x < dim; ++x) hi[x] = lo[x] + P.h;
      S.face(lo, hi, f.axis, hi[f.axis], frules[i]);
    }
    fallbacks[32 + t] += S.n_fallback;
  });
  P.n_fallback = 0;
  for (int64_t v : fallbacks) P.n_fallback += v;

  // -- convert to reference coordinates and concatenate
  const double hd = std::pow(P.h, dim), hd1 = std::pow(P.h, dim - 1);
  P.vol_off.assign(ncut + 1, 0);
  P.surf_off.assign(ncut + 1, 0);
  P.vol_x.clear(); P.vol_w.clear(); P.surf_x.clear(); P.surf_w.clear(); P.surf_n.clear();
  P.max_qp_cut_cell = 0;
  for (size_t i = 0; i < ncut; ++i) {
    double lo[3] = {0, 0, 0};
    P.cell_lo(P.active[P.cut[i]], lo);
    const Rule& R = rules[i];
    for (size_t j = 0; j < R.vw.size(); ++j) {
      for (int a = 0; a < dim; ++a) P.vol_x.push_back((R.vx[j * 3 + a] - lo[a]) / P.h);
      P.vol_w.push_back(R.vw[j] / hd);
    }
    for (size_t j = 0; j < R.sw.size(); ++j) {
      for (int a = 0; a < dim; ++a) P.surf_x.push_back((R.sx[j * 3 + a] - lo[a]) / P.h);
      P.surf_w.push_back(R.sw[j] / hd1);
      for (int a = 0; a < dim; ++a) P.surf_n.push_back(R.sn[j * 3 + a]);
    }
    P.vol_off[i + 1] = P.vol_off[i] + (int64_t)R.vw.size();
    P.surf_off[i + 1] = P.surf_off[i] + (int64_t)R.sw.size();
    P.max_qp_cut_cell = std::max<int64_t>(P.max_qp_cut_cell, (int64_t)R.vw.size());
  }
  P.fcut_off.assign(cutfaces.size() + 1, 0);
  P.fcut_face = cutfaces;
  P.fcut_x.clear(); P.fcut_w.clear();
  for (size_t i = 0; i < cutfaces.size(); ++i) {
    const Face& f = P.faces[cutfaces[i]];
    double lo[3] = {0, 0, 0};
    P.cell_lo(f.bm, lo);
    const Rule& R = frules[i];
    for (size_t j = 0; j < R.vw.size(); ++j) {
      for (int a = 0; a < dim; ++a)
        if (a != f.axis) P.fcut_x.push_back((R.vx[j * 3 + a] - lo[a]) / P.h);
      P.fcut_w.push_back(R.vw[j] / hd1);
    }
    P.fcut_off[i + 1] = P.fcut_off[i] + (int64_t)R.vw.size();
  }

  return finish_rules(P, code);
}

std::string import_rules(Plan& P, const int64_t* vc, const int64_t* fc, const int64_t* sc, const double* ref,
                         const double* w, const double* nrm, int* code) {
  *code = UFEM_EINVAL;
  const int dim = P.dim;
  const size_t ncut = P.cut.size(), nfc = P.fcut_face.size();
  if ((ncut && (!vc || !sc)) || (nfc && !fc)) return "point counts missing";
  int64_t nv = 0, nf = 0, ns = 0;
  for (size_t i = 0; i < ncut; ++i) {
    if (vc[i] < 0 || sc[i] < 0) return "negative point count";
    nv += vc[i];
    ns += sc[i];
  }
  for (size_t i = 0; i < nfc; ++i) {
    if (fc[i] < 0) return "negative point count";
    nf += fc[i];
  }
  const int64_t total = nv + nf + ns;
  if (nv > 0x7fffffff || nf > 0x7fffffff || ns > 0x7fffffff) {
    *code = UFEM_EUNSUPPORTED;
    return "too many cut quadrature points for 32-bit point indices";
  }
  if (total > 0 && (!ref || !w || (ns > 0 && !nrm))) return "null point arrays";
  const double tol = 1e-12;
  for (int64_t q = 0; q < total; ++q) {
    if (!std::isfinite(w[q]) || w[q] < 0.0) return "weights must be finite and non-negative";
    for (int a = 0; a < dim; ++a) {
      const double x = ref[q * dim + a];
      if (!std::isfinite(x) || x < -tol || x > 1.0 + tol) return "reference coordinates must lie in [0, 1]";
    }
  }
  for (int64_t q = nv + nf; q < total; ++q)
    for (int a = 0; a < dim; ++a)
      if (!std::isfinite(nrm[q * dim + a])) return "normals must be finite";
  P.vol_off.assign(ncut + 1, 0);
  P.surf_off.assign(ncut + 1, 0);
  P.fcut_off.assign(nfc + 1, 0);
  for (size_t i = 0; i < ncut; ++i) {
    P.vol_off[i + 1] = P.vol_off[i] + vc[i];
    P.surf_off[i + 1] = P.surf_off[i] + sc[i];
  }
  for (size_t i = 0; i < nfc; ++i) P.fcut_off[i + 1] = P.fcut_off[i] + fc[i];
  P.vol_x.assign(ref, ref + nv * dim);
  P.vol_w.assign(w, w + nv);
  P.fcut_x.clear();
  P.fcut_x.reserve((size_t)nf * (dim - 1));
  for (size_t i = 0; i < nfc; ++i) {
    const int axis = P.faces[P.fcut_face[i]].axis;
    for (int64_t q = nv + P.fcut_off[i]; q < nv + P.fcut_off[i + 1]; ++q)
      for (int a = 0; a < dim; ++a)
        if (a != axis) P.fcut_x.push_back(ref[q * dim + a]);
  }
  P.fcut_w.assign(w + nv, w + nv + nf);
  P.surf_x.assign(ref + (nv + nf) * dim, ref + total * dim);
  P.surf_w.assign(w + nv + nf, w + total);
  P.surf_n.assign(nrm + (nv + nf) * dim, nrm + total * dim);
  return finish_rules(P, code);
}

}  // namespace ufem
