// Host set-up on periodic tetrahedral meshes (d = 3; the method is posed for d = 2, 3,
// Sec. 2): quadrature, the orthonormal Dubiner basis of the tetrahedron, face matching with
// the six face-vertex permutations, element geometry, the element condensation of eq. (FE3)
// and the facet matrix S as a 7-slot BSR (a face couples to itself and to the other three
// faces of each of its two elements).  FP64, once per context.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "dfdg_setup.h"

namespace dfdg {

const int kFacePerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

int face_perm_id(const int p[3]) {
  for (int i = 0; i < 6; ++i)
    if (kFacePerm[i][0] == p[0] && kFacePerm[i][1] == p[1] && kFacePerm[i][2] == p[2]) return i;
  return -1;
}

int face_perm_inverse(int id) {
  int q[3];
  for (int i = 0; i < 3; ++i) q[kFacePerm[id][i]] = i;
  return face_perm_id(q);
}

// Local face f of a tetrahedron: the vertices other than f, in increasing order; its face
// parameter (s, t) is x = a0 + s (a1 - a0) + t (a2 - a0).
static const int kFaceV[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
static const double kRefV3[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

static void ref_face_point(int f, double s, double t, double* xh) {
  const double* a = kRefV3[kFaceV[f][0]];
  const double* b = kRefV3[kFaceV[f][1]];
  const double* c = kRefV3[kFaceV[f][2]];
  for (int d = 0; d < 3; ++d) xh[d] = a[d] + s * (b[d] - a[d]) + t * (c[d] - a[d]);
}

// ---------------------------------------------------------------------------------------
// Quadrature
// ---------------------------------------------------------------------------------------

// n-point Gauss-Jacobi rule for the weight (1 - x)^alpha on [-1, 1] (beta = 0): the roots of
// P_n^{(alpha,0)} by Newton's method with deflation from Chebyshev guesses, and the weights
// 2^{alpha+1} / ((1 - x^2) P_n'(x)^2).
static void gauss_jacobi(int n, double alpha, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.141592653589793238462643383279502884;
  for (int k = 0; k < n; ++k) {
    double r = -std::cos((2.0 * k + 1.0) * pi / (2.0 * n));
    if (k > 0) r = 0.5 * (r + x[k - 1]);
    for (int it = 0; it < 200; ++it) {
      double p, dp;
      jacobi_poly(n, alpha, 0.0, r, &p, &dp);
      double s = 0;
      for (int i = 0; i < k; ++i) s += 1.0 / (r - x[i]);
      const double delta = -p / (dp - s * p);
      r += delta;
      if (std::fabs(delta) < 1e-16) break;
    }
    x[k] = r;
  }
  std::sort(x.begin(), x.end());
  for (int k = 0; k < n; ++k) {
    double p, dp;
    jacobi_poly(n, alpha, 0.0, x[k], &p, &dp);
    w[k] = std::pow(2.0, alpha + 1.0) / ((1.0 - x[k] * x[k]) * dp * dp);
  }
}

// Collapsed tetrahedron rule exact for total degree p: Gauss-Legendre in a, Gauss-Jacobi
// (1, 0) in b and (2, 0) in c, n = (p + 2) / 2 points each; xi = (1+a)(1-b)(1-c)/8,
// eta = (1+b)(1-c)/4, zeta = (1+c)/2, the Jacobian (1-b)(1-c)^2/64 in the Jacobi weights.
void tet_rule(int p, std::vector<double>& pts, std::vector<double>& w) {
  const int n = (p + 2) / 2;
  std::vector<double> a, wa, b, wb, c, wc;
  gauss_jacobi(n, 0.0, a, wa);
  gauss_jacobi(n, 1.0, b, wb);
  gauss_jacobi(n, 2.0, c, wc);
  pts.clear();
  w.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        pts.push_back(0.125 * (1 + a[i]) * (1 - b[j]) * (1 - c[k]));
        pts.push_back(0.25 * (1 + b[j]) * (1 - c[k]));
        pts.push_back(0.5 * (1 + c[k]));
        w.push_back(wa[i] * wb[j] * wc[k] / 64.0);
      }
}

// Fully symmetric positive rules on the reference triangle (Dunavant's degree-4 rule, 6
// points, and degree-6 rule, 12 points): orbits (a, a, 1-2a) and (a, b, 1-a-b) in
// barycentric coordinates.  Starting from the published parameters (about 12 digits), the
// moment equations sum_q w_q xi^i eta^j = i! j! / (i + j + 2)! (i + j <= degree) are solved
// by Gauss-Newton in long double.  The point set is invariant under the vertex
// permutations, so both sides of a face evaluate at the same points.
namespace {
// kind 0: the orbit (a, a, 1-2a), 3 points; kind 1: (a, b, 1-a-b), 6 points
void orbit_points(int kind, const long double* par, std::vector<long double>& xy) {
  if (kind == 0) {
    const long double a = par[0], b = 1 - 2 * a;
    const long double p[3][2] = {{a, a}, {a, b}, {b, a}};
    for (auto& q : p) { xy.push_back(q[0]); xy.push_back(q[1]); }
  } else {
    const long double a = par[0], b = par[1], c = 1 - a - b;
    const long double p[6][2] = {{a, b}, {b, a}, {a, c}, {c, a}, {b, c}, {c, b}};
    for (auto& q : p) { xy.push_back(q[0]); xy.push_back(q[1]); }
  }
}
long double fact(int n) { long double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }
}  // namespace

void sym_face_rule(int degree, std::vector<double>& pts, std::vector<double>& w) {
  std::vector<int> kinds;
  std::vector<long double> x;  // per orbit: parameters then the weight (relative to area 1)
  if (degree <= 4) {
    kinds = {0, 0};
    x = {0.445948490915965L, 0.223381589678011L, 0.091576213509771L, 0.109951743655322L};
  } else {
    kinds = {0, 0, 1};
    x = {0.249286745170910L, 0.116786275726379L, 0.063089014491502L, 0.050844906370207L,
         0.053145049844817L, 0.310352451033784L, 0.082851075618374L};
    degree = 6;
  }
  std::vector<std::pair<int, int>> ex;
  for (int i = 0; i <= degree; ++i)
    for (int j = 0; i + j <= degree; ++j) ex.push_back({i, j});
  const int ne = (int)ex.size(), nx = (int)x.size();
  auto build = [&](const std::vector<long double>& v, std::vector<long double>& xy, std::vector<long double>& ww) {
    xy.clear();
    ww.clear();
    size_t o = 0;
    for (int kind : kinds) {
      const int npar = kind == 0 ? 1 : 2;
      const size_t before = xy.size();
      orbit_points(kind, &v[o], xy);
      for (size_t q = before; q < xy.size(); q += 2) ww.push_back(0.5L * v[o + npar]);
      o += npar + 1;
    }
  };
  auto resid = [&](const std::vector<long double>& v, std::vector<long double>& r) {
    std::vector<long double> xy, ww;
    build(v, xy, ww);
    r.assign(ne, 0);
    for (int e = 0; e < ne; ++e) {
      long double s = 0;
      for (size_t q = 0; q < ww.size(); ++q) s += ww[q] * std::pow(xy[2 * q], ex[e].first) * std::pow(xy[2 * q + 1], ex[e].second);
      const long double exact = fact(ex[e].first) * fact(ex[e].second) / fact(ex[e].first + ex[e].second + 2);
      r[e] = s / exact - 1;
    }
  };
  std::vector<long double> r, r2, J((size_t)ne * nx);
  for (int it = 0; it < 30; ++it) {
    resid(x, r);
    for (int j = 0; j < nx; ++j) {  // forward-difference Jacobian in long double
      std::vector<long double> y = x;
      const long double h = 1e-9L * std::max(1.0L, std::fabs(x[j]));
      y[j] += h;
      resid(y, r2);
      for (int e = 0; e < ne; ++e) J[(size_t)e * nx + j] = (r2[e] - r[e]) / h;
    }
    // normal equations (J^T J) dx = -J^T r, Gaussian elimination with partial pivoting
    std::vector<long double> A((size_t)nx * (nx + 1), 0);
    for (int i = 0; i < nx; ++i) {
      for (int j = 0; j < nx; ++j) {
        long double s = 0;
        for (int e = 0; e < ne; ++e) s += J[(size_t)e * nx + i] * J[(size_t)e * nx + j];
        A[(size_t)i * (nx + 1) + j] = s;
      }
      long double s = 0;
      for (int e = 0; e < ne; ++e) s -= J[(size_t)e * nx + i] * r[e];
      A[(size_t)i * (nx + 1) + nx] = s;
    }
    for (int c = 0; c < nx; ++c) {
      int piv = c;
      for (int i = c + 1; i < nx; ++i)
        if (std::fabs(A[(size_t)i * (nx + 1) + c]) > std::fabs(A[(size_t)piv * (nx + 1) + c])) piv = i;
      for (int j = 0; j <= nx; ++j) std::swap(A[(size_t)c * (nx + 1) + j], A[(size_t)piv * (nx + 1) + j]);
      for (int i = c + 1; i < nx; ++i) {
        const long double f = A[(size_t)i * (nx + 1) + c] / A[(size_t)c * (nx + 1) + c];
        for (int j = c; j <= nx; ++j) A[(size_t)i * (nx + 1) + j] -= f * A[(size_t)c * (nx + 1) + j];
      }
    }
    std::vector<long double> dx(nx);
    for (int i = nx - 1; i >= 0; --i) {
      long double s = A[(size_t)i * (nx + 1) + nx];
      for (int j = i + 1; j < nx; ++j) s -= A[(size_t)i * (nx + 1) + j] * dx[j];
      dx[i] = s / A[(size_t)i * (nx + 1) + i];
    }
    long double step = 0;
    for (int i = 0; i < nx; ++i) {
      x[i] += dx[i];
      step = std::max(step, std::fabs(dx[i]));
    }
    if (step < 1e-18L) break;
  }
  std::vector<long double> xy, ww;
  build(x, xy, ww);
  pts.assign(xy.begin(), xy.end());
  w.assign(ww.begin(), ww.end());
}

// ---------------------------------------------------------------------------------------
// Orthonormal Dubiner basis of P^K on the reference tetrahedron
// ---------------------------------------------------------------------------------------
// psi_pqr = F_p(x1, y1) G_q(x2, y2) H_r(zeta) with the collapsed-coordinate factors written
// as polynomials: y1 = 1 - eta - zeta, x1 = 2 xi - y1, F_p = y1^p Legendre_p(x1 / y1);
// y2 = 1 - zeta, x2 = 2 eta - y2, G_q = y2^q Jacobi_q^{(2p+1,0)}(x2 / y2); H_r =
// Jacobi_r^{(2p+2q+2,0)}(2 zeta - 1).  The homogeneous recurrences are carried out in exact
// polynomial arithmetic on monomial coefficients (degree <= 3), and each function is scaled
// to unit L2 norm with the exact moments int xi^a eta^b zeta^c = a! b! c! / (a+b+c+3)!.
// Ordered by total degree d = p + q + r, then q + r, then r: the first dim P^j span P^j.
namespace {
constexpr int kD = kMaxK + 1;  // coefficient array extent per variable
struct Poly {
  std::array<double, kD * kD * kD> c{};
  double& at(int a, int b, int g) { return c[(a * kD + b) * kD + g]; }
  double at(int a, int b, int g) const { return c[(a * kD + b) * kD + g]; }
};
Poly pconst(double v) { Poly p; p.at(0, 0, 0) = v; return p; }
Poly plin(double c0, double cx, double cy, double cz) {
  Poly p;
  p.at(0, 0, 0) = c0; p.at(1, 0, 0) = cx; p.at(0, 1, 0) = cy; p.at(0, 0, 1) = cz;
  return p;
}
Poly padd(const Poly& a, double sa, const Poly& b, double sb) {
  Poly r;
  for (size_t i = 0; i < r.c.size(); ++i) r.c[i] = sa * a.c[i] + sb * b.c[i];
  return r;
}
Poly pmul(const Poly& a, const Poly& b) {
  Poly r;
  for (int a1 = 0; a1 < kD; ++a1)
    for (int b1 = 0; b1 < kD; ++b1)
      for (int g1 = 0; g1 < kD; ++g1) {
        const double x = a.at(a1, b1, g1);
        if (x == 0) continue;
        for (int a2 = 0; a2 + a1 < kD; ++a2)
          for (int b2 = 0; b2 + b1 < kD; ++b2)
            for (int g2 = 0; g2 + g1 < kD; ++g2) r.at(a1 + a2, b1 + b2, g1 + g2) += x * b.at(a2, b2, g2);
      }
  return r;
}
// y^n P_n^{(al,0)}(x / y) for n = 0..nmax (x, y polynomials), by the Jacobi recurrence
std::vector<Poly> hom_jacobi(int nmax, double al, const Poly& x, const Poly& y) {
  std::vector<Poly> H;
  H.push_back(pconst(1.0));
  if (nmax >= 1) H.push_back(padd(x, 0.5 * (al + 2.0), y, 0.5 * al));
  const Poly y2 = pmul(y, y);
  for (int n = 2; n <= nmax; ++n) {
    const double s = 2.0 * n + al;
    const double a1 = 2.0 * n * (n + al) * (s - 2.0);
    const double cx = (s - 1.0) * s * (s - 2.0), cy = (s - 1.0) * al * al;
    const double e = 2.0 * (n + al - 1.0) * (n - 1.0) * s;
    const Poly t1 = pmul(padd(x, cx, y, cy), H[n - 1]);
    const Poly t2 = pmul(y2, H[n - 2]);
    H.push_back(padd(t1, 1.0 / a1, t2, -e / a1));
  }
  return H;
}
long double factl(int n) { long double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }
struct Basis3 {
  int K = -1;
  std::vector<Poly> psi;
};
const Basis3& basis3(int K) {
  static Basis3 cache[kMaxK + 1];
  Basis3& B = cache[K];
  if (B.K == K) return B;
  std::vector<Poly> out;
  const Poly y1 = plin(1, 0, -1, -1), x1 = plin(-1, 2, 1, 1);  // x1 = 2 xi - y1
  const Poly y2 = plin(1, 0, 0, -1), x2 = plin(-1, 0, 2, 1);   // x2 = 2 eta - y2
  const Poly one = pconst(1.0), zl = plin(-1, 0, 0, 2);         // 2 zeta - 1
  const std::vector<Poly> F = hom_jacobi(K, 0.0, x1, y1);
  for (int d = 0; d <= K; ++d)
    for (int qr = 0; qr <= d; ++qr)
      for (int r = 0; r <= qr; ++r) {
        const int p = d - qr, q = qr - r;
        const std::vector<Poly> G = hom_jacobi(q, 2.0 * p + 1.0, x2, y2);
        const std::vector<Poly> H = hom_jacobi(r, 2.0 * p + 2.0 * q + 2.0, zl, one);
        Poly f = pmul(pmul(F[p], G[q]), H[r]);
        // exact squared L2 norm on the reference tetrahedron, from the monomial moments of
        // the products of f's terms (f^2 has degree up to 2K, beyond the coefficient array)
        const Poly& f2 = f;
        long double nrm = 0;
        for (int a1 = 0; a1 < kD; ++a1)
          for (int b1 = 0; b1 < kD; ++b1)
            for (int g1 = 0; g1 < kD; ++g1) {
              const long double u = f2.at(a1, b1, g1);
              if (u == 0) continue;
              for (int a2 = 0; a2 < kD; ++a2)
                for (int b2 = 0; b2 < kD; ++b2)
                  for (int g2 = 0; g2 < kD; ++g2) {
                    const long double v = f2.at(a2, b2, g2);
                    if (v == 0) continue;
                    nrm += u * v * factl(a1 + a2) * factl(b1 + b2) * factl(g1 + g2) /
                           factl(a1 + a2 + b1 + b2 + g1 + g2 + 3);
                  }
            }
        const double sc = (double)(1.0L / std::sqrt(nrm));
        for (double& v : f.c) v *= sc;
        out.push_back(f);
      }
  B.psi = out;
  B.K = K;
  return B;
}
}  // namespace

void dubiner3(int K, double xi, double eta, double zeta, double* vals, double* grads) {
  const Basis3& B = basis3(K);
  const int P = nP3(K);
  double px[kD], py[kD], pz[kD];
  px[0] = py[0] = pz[0] = 1;
  for (int i = 1; i < kD; ++i) {
    px[i] = px[i - 1] * xi;
    py[i] = py[i - 1] * eta;
    pz[i] = pz[i - 1] * zeta;
  }
  for (int i = 0; i < P; ++i) {
    const Poly& f = B.psi[i];
    double v = 0, g0 = 0, g1 = 0, g2 = 0;
    for (int a = 0; a < kD; ++a)
      for (int b = 0; b < kD; ++b)
        for (int c = 0; c < kD; ++c) {
          const double u = f.at(a, b, c);
          if (u == 0) continue;
          v += u * px[a] * py[b] * pz[c];
          if (a > 0) g0 += u * a * px[a - 1] * py[b] * pz[c];
          if (b > 0) g1 += u * b * px[a] * py[b - 1] * pz[c];
          if (c > 0) g2 += u * c * px[a] * py[b] * pz[c - 1];
        }
    vals[i] = v;
    if (grads) {
      grads[0 * P + i] = g0;
      grads[1 * P + i] = g1;
      grads[2 * P + i] = g2;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Reference tables
// ---------------------------------------------------------------------------------------
void build_ref_tables3(int K, RefTables& t) {
  t.dim = 3;
  t.K = K;
  t.P = nP3(K);
  t.NP = nPp3(K);
  t.NF = nF3(K);
  const int P = t.P, NF = t.NF;
  tet_rule(3 * K - 1, t.vq, t.vw);
  std::vector<double> fpts;
  sym_face_rule(K == 1 ? 4 : 6, fpts, t.fw);
  t.fs = fpts;  // [nqf][2] face parameters (s, t)
  for (double& w : t.fw) w *= 2.0;  // weights summing to 1 (times the face area)
  tet_rule(2 * K + 2, t.pq, t.pw);
  t.nqv = (int)t.vw.size();
  t.nqf = (int)t.fw.size();
  t.nqp = (int)t.pw.size();
  std::vector<double> v(P), g(3 * P);
  t.Vv.assign((size_t)t.nqv * P, 0);
  t.Gv.assign((size_t)t.nqv * 3 * P, 0);
  for (int q = 0; q < t.nqv; ++q) {
    dubiner3(K, t.vq[3 * q], t.vq[3 * q + 1], t.vq[3 * q + 2], v.data(), g.data());
    for (int i = 0; i < P; ++i) {
      t.Vv[(size_t)q * P + i] = v[i];
      for (int a = 0; a < 3; ++a) t.Gv[((size_t)q * 3 + a) * P + i] = g[a * P + i];
    }
  }
  t.Vf.assign((size_t)4 * t.nqf * P, 0);
  t.Gf.assign((size_t)4 * t.nqf * 3 * P, 0);
  for (int f = 0; f < 4; ++f)
    for (int r = 0; r < t.nqf; ++r) {
      double xh[3];
      ref_face_point(f, fpts[2 * r], fpts[2 * r + 1], xh);
      dubiner3(K, xh[0], xh[1], xh[2], v.data(), g.data());
      for (int i = 0; i < P; ++i) {
        t.Vf[((size_t)f * t.nqf + r) * P + i] = v[i];
        for (int a = 0; a < 3; ++a) t.Gf[(((size_t)f * t.nqf + r) * 3 + a) * P + i] = g[a * P + i];
      }
    }
  t.Vp.assign((size_t)t.nqp * P, 0);
  for (int q = 0; q < t.nqp; ++q) {
    dubiner3(K, t.pq[3 * q], t.pq[3 * q + 1], t.pq[3 * q + 2], v.data(), nullptr);
    for (int i = 0; i < P; ++i) t.Vp[(size_t)q * P + i] = v[i];
  }
  // Dh[a][j][i] = int_That dpsi_i/dxi_a psi_j (degree 2K - 1: the volume rule is exact)
  t.Dh.assign((size_t)3 * t.NP * P, 0);
  for (int q = 0; q < t.nqv; ++q)
    for (int a = 0; a < 3; ++a)
      for (int j = 0; j < t.NP; ++j)
        for (int i = 0; i < P; ++i)
          t.Dh[((size_t)a * t.NP + j) * P + i] += t.vw[q] * t.Gv[((size_t)q * 3 + a) * P + i] * t.Vv[(size_t)q * P + j];
  // Ch[f][m][i] = int_Fhat mu_m(s, t) psi_i(xhat_f(s, t)) dA over the reference triangle of
  // area 1/2, mu_m the orthonormal Dubiner basis of the triangle (degree 2K rule)
  std::vector<double> cs, cw, mu(NF);
  triangle_rule(2 * K, cs, cw);
  t.Ch.assign((size_t)4 * NF * P, 0);
  for (int f = 0; f < 4; ++f)
    for (size_t r = 0; r < cw.size(); ++r) {
      double xh[3];
      ref_face_point(f, cs[2 * r], cs[2 * r + 1], xh);
      dubiner3(K, xh[0], xh[1], xh[2], v.data(), nullptr);
      dubiner(K, cs[2 * r], cs[2 * r + 1], mu.data(), nullptr);
      for (int m = 0; m < NF; ++m)
        for (int i = 0; i < P; ++i) t.Ch[((size_t)f * NF + m) * P + i] += cw[r] * mu[m] * v[i];
    }
  // face point and face basis permutations.  A face point with barycentric coordinates
  // (l0, l1, l2) on the face's vertices a0, a1, a2 (face parameter (s, t) = (l1, l2)) is, for
  // a face whose vertex a_i is the other face's vertex b_{perm[i]}, the point with
  // barycentric coordinate l_i on b_{perm[i]}.
  auto map_point = [](int pid, double s, double tt, double& s2, double& t2) {
    const double l[3] = {1.0 - s - tt, s, tt};
    double l2[3];
    for (int i = 0; i < 3; ++i) l2[kFacePerm[pid][i]] = l[i];
    s2 = l2[1];
    t2 = l2[2];
  };
  t.fpidx.assign((size_t)6 * t.nqf, -1);
  for (int pid = 0; pid < 6; ++pid)
    for (int r = 0; r < t.nqf; ++r) {
      double s2, t2;
      map_point(pid, fpts[2 * r], fpts[2 * r + 1], s2, t2);
      for (int r2 = 0; r2 < t.nqf; ++r2)
        if (std::fabs(fpts[2 * r2] - s2) < 1e-12 && std::fabs(fpts[2 * r2 + 1] - t2) < 1e-12) t.fpidx[(size_t)pid * t.nqf + r] = r2;
    }
  t.Qf.assign((size_t)6 * NF * NF, 0);
  std::vector<double> mu2(NF);
  for (int pid = 0; pid < 6; ++pid)
    for (size_t r = 0; r < cw.size(); ++r) {
      double s2, t2;
      map_point(pid, cs[2 * r], cs[2 * r + 1], s2, t2);
      dubiner(K, cs[2 * r], cs[2 * r + 1], mu.data(), nullptr);  // own face parameter
      dubiner(K, s2, t2, mu2.data(), nullptr);                    // the other face's
      for (int m = 0; m < NF; ++m)
        for (int n = 0; n < NF; ++n) t.Qf[((size_t)pid * NF + m) * NF + n] += cw[r] * mu2[m] * mu[n];
    }
}

// ---------------------------------------------------------------------------------------
// Mesh: periodic face matching
// ---------------------------------------------------------------------------------------
// a == b modulo the period (per[d] = 0: no period in direction d; then relative to ext[d])
static bool same_mod3(const double* a, const double* b, const double* per, const double* ext, double tol) {
  for (int d = 0; d < 3; ++d) {
    double x = (a[d] - b[d]) / (per[d] > 0 ? per[d] : ext[d]);
    if (per[d] > 0) x -= std::nearbyint(x);
    if (std::fabs(x) > tol) return false;
  }
  return true;
}

int build_mesh3(int T, const double* xyz, const double* period, MeshHost& m, std::string& err) {
  m.dim = 3;
  m.T = T;
  m.xyz.assign(xyz, xyz + 12 * (size_t)T);
  for (int d = 0; d < 3; ++d) m.period[d] = period[d];
  double scale = std::max(period[0], std::max(period[1], period[2]));
  for (double v : m.xyz) scale = std::max(scale, std::fabs(v));
  // directions without a period (walls): coordinates relative to an extent that covers the
  // mesh, so that (x + ext) / (2 ext) lies in (0, 1)
  const bool walls = period[0] == 0 || period[1] == 0 || period[2] == 0;
  double ext[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = 1.0;
    for (int t = 0; t < T; ++t)
      for (int j = 0; j < 4; ++j) ext[d] = std::max(ext[d], 2.0 * std::fabs(m.xyz[12 * (size_t)t + 3 * j + d]));
  }
  auto unit = [&](double x, int d) {  // position in [0, 1): modulo the period, else in the extent
    if (period[d] > 0) {
      x /= period[d];
      return x - std::floor(x);
    }
    return (x + ext[d]) / (2.0 * ext[d]);
  };
  for (int t = 0; t < T; ++t) {
    const double* v = &m.xyz[12 * (size_t)t];
    double J[3][3];
    for (int i = 0; i < 3; ++i)
      for (int r = 0; r < 3; ++r) J[i][r] = v[3 * (r + 1) + i] - v[i];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 1e-14 * scale * scale * scale)) {
      err = "element " + std::to_string(t) + " is inverted or degenerate (det J = " + std::to_string(det) +
            "); vertices must be positively oriented";
      return -2;
    }
  }
  m.efacet.assign(4 * (size_t)T, -1);
  m.fL.clear(); m.fLloc.clear(); m.fR.clear(); m.fRloc.clear(); m.frev.clear();
  std::unordered_map<uint64_t, int> first;
  first.reserve(4 * (size_t)T);
  const double Q = 2097152.0;  // 2^21 per coordinate
  auto vert = [&](int t, int f, int j) { return &m.xyz[12 * (size_t)t + 3 * kFaceV[f][j]]; };
  for (int t = 0; t < T; ++t)
    for (int f = 0; f < 4; ++f) {
      uint64_t key = 0;
      for (int d = 0; d < 3; ++d) {
        const double mid = unit((vert(t, f, 0)[d] + vert(t, f, 1)[d] + vert(t, f, 2)[d]) / 3.0, d);
        const long long q = std::llround(mid * Q) % (long long)Q;
        key = (key << 21) | (uint64_t)q;
      }
      auto it = first.find(key);
      if (it == first.end()) {
        const int F = (int)m.fL.size();
        first.emplace(key, F);
        m.fL.push_back(t); m.fLloc.push_back(f);
        m.fR.push_back(-1); m.fRloc.push_back(-1); m.frev.push_back(0);
        m.efacet[4 * (size_t)t + f] = F;
      } else {
        const int F = it->second;
        const int L = m.fL[F], fl = m.fLloc[F];
        if (L == t) {
          err = "element " + std::to_string(t) + " is adjacent to itself across the periodic boundary";
          return -2;
        }
        int p[3] = {-1, -1, -1};
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            if (same_mod3(vert(L, fl, i), vert(t, f, j), period, ext, 1e-9)) p[i] = j;
        const int pid = face_perm_id(p);
        if (pid < 0) {
          err = "face vertices of elements " + std::to_string(L) + " and " + std::to_string(t) +
                " do not match modulo the period";
          return -2;
        }
        m.fR[F] = t; m.fRloc[F] = f; m.frev[F] = (uint8_t)pid;
        m.efacet[4 * (size_t)t + f] = F;
        first.erase(it);
      }
    }
  if (!first.empty() && !walls) {  // faces left without a partner are boundary faces with walls
    err = std::to_string(first.size()) + " faces have no periodic partner";
    return -2;
  }
  m.E = (int)m.fL.size();
  // number the faces along a Morton curve of their barycentres (modulo the period)
  {
    const int E = m.E;
    std::vector<uint64_t> key(E);
    for (int F = 0; F < E; ++F) {
      const int t = m.fL[F], f = m.fLloc[F];
      uint32_t q[3];
      for (int d = 0; d < 3; ++d) {
        const double mid = unit((vert(t, f, 0)[d] + vert(t, f, 1)[d] + vert(t, f, 2)[d]) / 3.0, d);
        q[d] = (uint32_t)std::min(65535.0, std::floor(mid * 65536.0));
      }
      uint64_t k = 0;
      for (int bit = 15; bit >= 0; --bit)
        k = (k << 3) | (((q[2] >> bit) & 1u) << 2) | (((q[1] >> bit) & 1u) << 1) | ((q[0] >> bit) & 1u);
      key[F] = k;
    }
    std::vector<int> order(E);
    for (int F = 0; F < E; ++F) order[F] = F;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key[x] < key[y]; });
    std::vector<int> newid(E);
    for (int i = 0; i < E; ++i) newid[order[i]] = i;
    auto perm = [&](auto& v) {
      auto w = v;
      for (int i = 0; i < E; ++i) w[i] = v[order[i]];
      v.swap(w);
    };
    perm(m.fL); perm(m.fLloc); perm(m.fR); perm(m.fRloc); perm(m.frev);
    for (int& F : m.efacet) F = newid[F];
  }
  return 0;
}

// ---------------------------------------------------------------------------------------
// Geometry, condensation and the facet matrix
// ---------------------------------------------------------------------------------------
int build_setup3(const MeshHost& m, int K, double alpha, HostSetup& h, std::string& err) {
  build_ref_tables3(K, h.tabs);
  const RefTables& tb = h.tabs;
  for (int v : tb.fpidx)
    if (v < 0 || v >= tb.nqf) {  // the face rule must be invariant under the vertex permutations
      err = "face rule is not symmetric under the face-vertex permutations";
      return -2;
    }
  const int T = m.T, E = m.E, P = tb.P, NP = tb.NP, NF = tb.NF, NU = 3 * P, NS = kSlots3;
  h.dim = 3;
  h.T = T;
  h.E = E;
  h.K = K;
  const size_t T4 = 4 * (size_t)T;
  h.Jinv.assign(9 * (size_t)T, 0);
  h.detJ.assign(T, 0);
  h.isq.assign(T, 0);
  h.nbr.assign(T4, 0);
  h.code.assign(T4, 0);
  h.efacet.assign(T4, 0);
  h.nx.assign(T4, 0);
  h.ny.assign(T4, 0);
  h.nz.assign(T4, 0);
  h.flen.assign(T4, 0);
  h.sig.assign(T4, 0);
  h.sF.assign(T4, 0);
  h.G.assign((size_t)nGpk3(K) * T, 0);
  h.qL.assign(E, 0);
  h.qR.assign(E, 0);
  h.zdef.assign(E, 0);
  h.cols.assign((size_t)NS * E, 0);
  h.vals.assign((size_t)NS * NF * NF * E, 0);
  h.dinv.assign((size_t)E * NF, 0);
  h.binv.assign((size_t)E * NF * NF, 0);

  std::vector<double> hT(T);
  for (int t = 0; t < T; ++t) {
    const double* v = &m.xyz[12 * (size_t)t];
    double J[3][3];
    for (int i = 0; i < 3; ++i)
      for (int r = 0; r < 3; ++r) J[i][r] = v[3 * (r + 1) + i] - v[i];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2],
                 c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    // inverse: Jinv[r][j] = dxi_r/dx_j = cofactor(j, r) / det
    const double inv[3][3] = {{c00 / det, (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det, (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det},
                              {c01 / det, (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det, (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det},
                              {c02 / det, (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det, (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det}};
    for (int r = 0; r < 3; ++r)
      for (int j = 0; j < 3; ++j) h.Jinv[(size_t)(3 * r + j) * T + t] = inv[r][j];
    h.detJ[t] = det;
    h.isq[t] = 1.0 / std::sqrt(det);
    hT[t] = std::cbrt(det);  // (d! |T|)^(1/d) with |T| = det / 6
  }
  for (int t = 0; t < T; ++t) {
    const double* v = &m.xyz[12 * (size_t)t];
    for (int f = 0; f < 4; ++f) {
      const int F = m.efacet[4 * (size_t)t + f];
      const bool isR = (m.fR[F] == t && m.fRloc[F] == f);
      const bool wall = m.fR[F] < 0;  // boundary face: one side, nbr = -1
      const bool open = wall && !m.fopen.empty() && m.fopen[F];  // outflow boundary
      const int nb = isR ? m.fL[F] : m.fR[F];
      const int nbf = wall ? 0 : (isR ? m.fLloc[F] : m.fRloc[F]);
      // permutation carrying this element's face vertices to the neighbour's
      const int pid = wall ? 0 : (isR ? face_perm_inverse(m.frev[F]) : (int)m.frev[F]);
      const double* a = v + 3 * kFaceV[f][0];
      const double* b = v + 3 * kFaceV[f][1];
      const double* c = v + 3 * kFaceV[f][2];
      const double* o = v + 3 * f;  // the vertex opposite the face
      const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
      double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
      const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      double sgn = (n[0] * (a[0] - o[0]) + n[1] * (a[1] - o[1]) + n[2] * (a[2] - o[2])) > 0 ? 1.0 : -1.0;
      const size_t idx = (size_t)f * T + t;
      h.nbr[idx] = nb;
      h.code[idx] = nbf | (pid << 2) | ((isR ? 1 : 0) << 5) | ((open ? 1 : 0) << 6);
      h.efacet[idx] = F;
      h.nx[idx] = sgn * n[0] / nn;
      h.ny[idx] = sgn * n[1] / nn;
      h.nz[idx] = sgn * n[2] / nn;
      h.flen[idx] = 0.5 * nn;
      h.sig[idx] = alpha * K * K / (wall ? hT[t] : std::min(hT[t], hT[nb]));
      // sqrt(|F| / |Fhat| / det J), |Fhat| = 1/2; no face rows of C_T on an outflow face
      h.sF[idx] = open ? 0.0 : std::sqrt(nn / h.detJ[t]);
    }
  }
  double zz = 0;
  for (int F = 0; F < E; ++F) {
    h.qL[F] = m.fLloc[F] * NF * T + m.fL[F];
    // -1: closed boundary face, -2: outflow face (the matrix-free product tells them apart)
    h.qR[F] = m.fR[F] < 0 ? ((!m.fopen.empty() && m.fopen[F]) ? -2 : -1) : m.fRloc[F] * NF * T + m.fR[F];
    const double area = h.flen[(size_t)m.fLloc[F] * T + m.fL[F]];
    h.zdef[F] = std::sqrt(area);  // the constant multiplier on mode 0 of the orthonormal face basis
    zz += area;
  }
  for (int F = 0; F < E; ++F) h.zdef[F] /= std::sqrt(zz);
  h.nearnull = h.zdef;
  h.singular = true;
  for (int F = 0; F < E; ++F)
    if (!m.fopen.empty() && m.fopen[F]) h.singular = false;
  if (!h.singular) std::fill(h.zdef.begin(), h.zdef.end(), 0.0);  // S is definite: no kernel

  // Element condensation (eq. (FE3)): D_T = sum_a Jinv[a][c] Dh[a]; the rows of face f are
  // sqrt(2|F|/det J) n_c Ch[f], mapped to the L side's face basis (Qf) on the R side
  struct Tet : CondenseElement {
    const HostSetup& h;
    int T, NP, P, NF, NU;
    Tet(const HostSetup& hh, int t, int np, int p, int nf) : h(hh), T(t), NP(np), P(p), NF(nf), NU(3 * p) {}
    bool isR(int t, int f) const override { return (h.code[(size_t)f * T + t] >> 5) & 1; }
    void build(int t, double* D, double* C) const override {
      const RefTables& tb = h.tabs;
      double Ji[3][3];
      for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) Ji[r][j] = h.Jinv[(size_t)(3 * r + j) * T + t];
      for (int j = 0; j < NP; ++j)
        for (int c = 0; c < 3; ++c)
          for (int i = 0; i < P; ++i) {
            double s = 0;
            for (int a = 0; a < 3; ++a) s += Ji[a][c] * tb.Dh[((size_t)a * NP + j) * P + i];
            D[(size_t)j * NU + c * P + i] = s;
          }
      std::vector<double> Cl((size_t)NF * NU);
      for (int f = 0; f < 4; ++f) {
        const size_t idx = (size_t)f * T + t;
        const double n[3] = {h.nx[idx], h.ny[idx], h.nz[idx]};
        for (int mm = 0; mm < NF; ++mm)
          for (int c = 0; c < 3; ++c)
            for (int i = 0; i < P; ++i)
              Cl[(size_t)mm * NU + c * P + i] = h.sF[idx] * n[c] * tb.Ch[((size_t)f * NF + mm) * P + i];
        const bool R = (h.code[idx] >> 5) & 1;
        const int pid = (h.code[idx] >> 2) & 7;
        for (int mm = 0; mm < NF; ++mm)
          for (int x = 0; x < NU; ++x) {
            double s = 0;
            if (R)
              for (int n2 = 0; n2 < NF; ++n2) s += tb.Qf[((size_t)pid * NF + mm) * NF + n2] * Cl[(size_t)n2 * NU + x];
            else
              s = Cl[(size_t)mm * NU + x];
            C[((size_t)f * NF + mm) * NU + x] = s;
          }
      }
    }
  } el(h, T, NP, P, NF);
  // boundary faces have no R side: its three blocks stay zero, with the row's own column
  for (int F = 0; F < E; ++F)
    if (m.fR[F] < 0)
      for (int s = 4; s < NS; ++s) h.cols[(size_t)s * E + F] = F;
  if (condense_elements(h, 4, NP, NU, NF, el, err)) return -2;
  // an outflow face's row and column of S vanish: an identity block fixes its multiplier to 0
  for (int F = 0; F < E; ++F)
    if (!m.fopen.empty() && m.fopen[F])
      for (int a = 0; a < NF; ++a) h.vals[(((size_t)0 * NF + a) * NF + a) * E + F] = 1.0;
  // merge repeated columns of a row (tiny periodic meshes) into their first slot
  for (int F = 0; F < E; ++F)
    for (int s = 1; s < NS; ++s)
      for (int s2 = 0; s2 < s; ++s2)
        if (h.cols[(size_t)s * E + F] == h.cols[(size_t)s2 * E + F]) {
          for (int a = 0; a < NF * NF; ++a) {
            h.vals[((size_t)s2 * NF * NF + a) * E + F] += h.vals[((size_t)s * NF * NF + a) * E + F];
            h.vals[((size_t)s * NF * NF + a) * E + F] = 0.0;
          }
          break;
        }
  std::vector<double> B((size_t)NF * NF);
  for (int F = 0; F < E; ++F) {
    for (int a = 0; a < NF; ++a) {
      const double d = h.vals[(((size_t)0 * NF + a) * NF + a) * E + F];
      if (!(d > 0)) {
        err = "facet matrix has a non-positive diagonal at face " + std::to_string(F);
        return -2;
      }
      h.dinv[(size_t)F * NF + a] = 1.0 / d;
      for (int b = 0; b < NF; ++b) B[(size_t)a * NF + b] = h.vals[(((size_t)0 * NF + a) * NF + b) * E + F];
    }
    if (!spd_inverse(NF, B.data())) {
      err = "facet diagonal block " + std::to_string(F) + " is not positive definite";
      return -2;
    }
    for (int a = 0; a < NF * NF; ++a) h.binv[(size_t)F * NF * NF + a] = B[a];
  }
  return 0;
}

}  // namespace dfdg
