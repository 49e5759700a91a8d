// Host part of the set-up: quadrature, the orthonormal Dubiner basis and its reference
// tabulations, periodic facet matching, element geometry, the element condensation
// data and the facet matrix S of the hybrid-mixed system (eq. (FE3) after static
// condensation).  Everything here runs once per context, in FP64, on the CPU.
#include "dfdg_setup.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <thread>
#include <unordered_map>

namespace dfdg {

// ---------------------------------------------------------------------------------------
// Quadrature
// ---------------------------------------------------------------------------------------

// Gauss-Legendre on [0,1] by Newton's method on P_n (long double), nodes mirrored so that
// x[n-1-i] == 1 - x[i] exactly: the facet integrals of two neighbours traverse the same
// points in opposite order.
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    long double z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int j = 2; j <= n; ++j) {
        long double p2 = ((2 * j - 1) * z * p1 - (j - 1) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    {
      long double p0 = 1, p1 = z;
      for (int j = 2; j <= n; ++j) {
        long double p2 = ((2 * j - 1) * z * p1 - (j - 1) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
    }
    long double wt = 2.0L / ((1 - z * z) * dp * dp);
    // z is the i-th largest root in (-1,1): map to [0,1]
    long double s_hi = 0.5L * (1 + z);
    x[n - 1 - i] = (double)s_hi;
    x[i] = (double)(1.0L - s_hi);
    w[i] = w[n - 1 - i] = (double)(0.5L * wt);
  }
  if (n % 2 == 1) x[n / 2] = 0.5;
}

// Collapsed rule on {xi, eta >= 0, xi + eta <= 1}: xi = u (1 - v), eta = v, with the
// Jacobian (1 - v) folded into the weights; Gauss-Legendre in u and v.  Exact for total
// degree p (the v-integrand has degree p + 1).
void triangle_rule(int p, std::vector<double>& pts, std::vector<double>& w) {
  std::vector<double> xu, wu, xv, wv;
  gauss_legendre01(triNu(p), xu, wu);
  gauss_legendre01(triNv(p), xv, wv);
  pts.clear();
  w.clear();
  for (size_t i = 0; i < xu.size(); ++i)
    for (size_t j = 0; j < xv.size(); ++j) {
      pts.push_back(xu[i] * (1.0 - xv[j]));
      pts.push_back(xv[j]);
      w.push_back(wu[i] * wv[j] * (1.0 - xv[j]));
    }
}

// Fully symmetric rules with fewer points than the collapsed ones, in barycentric orbits
// (weights relative to the area, scaled by 1/2 below):
//   degree 2: the three points (2/3, 1/6, 1/6) and permutations, weight 1/3 each;
//   degree 5 (Radon's seven-point rule): the centroid, weight 9/40, and the orbits
//     (1 - 2a, a, a) for a = (6 -+ sqrt 15)/21, weights (155 -+ sqrt 15)/1200.
void residual_volume_rule(int K, std::vector<double>& pts, std::vector<double>& w) {
  if (K > 2) {
    triangle_rule(3 * K - 1, pts, w);
    return;
  }
  pts.clear();
  w.clear();
  auto orbit3 = [&](double a, double wt) {
    const double b = 1.0 - 2.0 * a;
    const double xy[3][2] = {{a, a}, {b, a}, {a, b}};
    for (const auto& p : xy) {
      pts.push_back(p[0]);
      pts.push_back(p[1]);
      w.push_back(0.5 * wt);
    }
  };
  if (K == 1) {
    orbit3(1.0 / 6.0, 1.0 / 3.0);
    return;
  }
  const double r15 = std::sqrt(15.0);
  pts.push_back(1.0 / 3.0);
  pts.push_back(1.0 / 3.0);
  w.push_back(0.5 * 9.0 / 40.0);
  orbit3((6.0 - r15) / 21.0, (155.0 - r15) / 1200.0);
  orbit3((6.0 + r15) / 21.0, (155.0 + r15) / 1200.0);
}

// ---------------------------------------------------------------------------------------
// Orthonormal Dubiner basis of P^K on the reference triangle
// ---------------------------------------------------------------------------------------
// psi_pq = Q_p(s, t) R_q(eta) * sqrt((2p+1)(2p+2q+2)) with s = 2 xi - 1 + eta, t = 1 - eta,
// Q_p(s, t) = t^p Legendre_p(s / t) (a polynomial, computed by the homogenised Legendre
// recurrence so that the collapsed-coordinate singularity at eta = 1 never appears) and
// R_q(eta) = Jacobi_q^{(2p+1, 0)}(2 eta - 1).  Ordered by total degree d = p + q, then q:
// the first dim P^j functions span P^j.

void jacobi_poly(int n, double a, double b, double x, double* val, double* der) {
  // P_n^{(a,b)}(x) and its derivative by the three-term recurrence.
  auto eval = [](int n, double a, double b, double x) {
    if (n == 0) return 1.0;
    double p0 = 1.0, p1 = 0.5 * ((a + b + 2) * x + (a - b));
    for (int k = 2; k <= n; ++k) {
      double c = 2 * k + a + b;
      double a1 = 2 * k * (k + a + b) * (c - 2);
      double a2 = (c - 1) * (c * (c - 2) * x + a * a - b * b);
      double a3 = 2 * (k + a - 1) * (k + b - 1) * c;
      double p2 = (a2 * p1 - a3 * p0) / a1;
      p0 = p1;
      p1 = p2;
    }
    return p1;
  };
  *val = eval(n, a, b, x);
  if (der) *der = (n == 0) ? 0.0 : 0.5 * (n + a + b + 1) * eval(n - 1, a + 1, b + 1, x);
}

void dubiner(int K, double xi, double eta, double* vals, double* grads) {
  const int P = nP(K);
  const double s = 2 * xi - 1 + eta, t = 1 - eta;
  // Q_p and partial derivatives wrt s and t
  double Q[kMaxK + 2], Qs[kMaxK + 2], Qt[kMaxK + 2];
  Q[0] = 1; Qs[0] = 0; Qt[0] = 0;
  Q[1] = s; Qs[1] = 1; Qt[1] = 0;
  for (int p = 1; p < K; ++p) {
    Q[p + 1] = ((2 * p + 1) * s * Q[p] - p * t * t * Q[p - 1]) / (p + 1);
    Qs[p + 1] = ((2 * p + 1) * (Q[p] + s * Qs[p]) - p * t * t * Qs[p - 1]) / (p + 1);
    Qt[p + 1] = ((2 * p + 1) * s * Qt[p] - p * (2 * t * Q[p - 1] + t * t * Qt[p - 1])) / (p + 1);
  }
  int idx = 0;
  for (int d = 0; d <= K; ++d)
    for (int q = 0; q <= d; ++q, ++idx) {
      const int p = d - q;
      double R, Rd;
      jacobi_poly(q, 2 * p + 1, 0, 2 * eta - 1, &R, &Rd);
      const double c = std::sqrt((2.0 * p + 1) * (2.0 * p + 2.0 * q + 2));
      vals[idx] = c * Q[p] * R;
      if (grads) {
        // d/dxi = 2 dQ/ds R ;  d/deta = (dQ/ds - dQ/dt) R + Q * 2 R'
        grads[0 * P + idx] = c * 2 * Qs[p] * R;
        grads[1 * P + idx] = c * ((Qs[p] - Qt[p]) * R + Q[p] * 2 * Rd);
      }
    }
}

double legendre01_orthonormal(int m, double s) {
  double x = 2 * s - 1, p0 = 1, p1 = x;
  if (m == 0) return 1.0;
  for (int j = 2; j <= m; ++j) {
    double p2 = ((2 * j - 1) * x * p1 - (j - 1) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  return std::sqrt(2.0 * m + 1) * p1;
}

// Local facet f joins reference vertices (f+1)%3 -> (f+2)%3.
static const double kRefV[3][2] = {{0, 0}, {1, 0}, {0, 1}};
static void ref_facet_point(int f, double s, double* xh) {
  const double* a = kRefV[(f + 1) % 3];
  const double* b = kRefV[(f + 2) % 3];
  xh[0] = a[0] + s * (b[0] - a[0]);
  xh[1] = a[1] + s * (b[1] - a[1]);
}

void build_ref_tables(int K, RefTables& t) {
  t.K = K;
  t.P = nP(K);
  t.NP = nPp(K);
  t.NF = nF(K);
  const int P = t.P;
  residual_volume_rule(K, t.vq, t.vw);
  gauss_legendre01(nQF(K), t.fs, t.fw);
  triangle_rule(projDeg(K), t.pq, t.pw);
  t.nqv = (int)t.vw.size();
  t.nqf = (int)t.fw.size();
  t.nqp = (int)t.pw.size();
  std::vector<double> v(P), g(2 * P);
  t.Vv.assign(t.nqv * P, 0);
  t.Gv.assign(t.nqv * 2 * P, 0);
  for (int q = 0; q < t.nqv; ++q) {
    dubiner(K, t.vq[2 * q], t.vq[2 * q + 1], v.data(), g.data());
    for (int i = 0; i < P; ++i) {
      t.Vv[q * P + i] = v[i];
      t.Gv[(q * 2 + 0) * P + i] = g[i];
      t.Gv[(q * 2 + 1) * P + i] = g[P + i];
    }
  }
  t.Vf.assign(3 * t.nqf * P, 0);
  t.Gf.assign(3 * t.nqf * 2 * P, 0);
  for (int f = 0; f < 3; ++f)
    for (int r = 0; r < t.nqf; ++r) {
      double xh[2];
      ref_facet_point(f, t.fs[r], xh);
      dubiner(K, xh[0], xh[1], v.data(), g.data());
      for (int i = 0; i < P; ++i) {
        t.Vf[(f * t.nqf + r) * P + i] = v[i];
        t.Gf[((f * t.nqf + r) * 2 + 0) * P + i] = g[i];
        t.Gf[((f * t.nqf + r) * 2 + 1) * P + i] = g[P + i];
      }
    }
  t.Vp.assign(t.nqp * P, 0);
  for (int q = 0; q < t.nqp; ++q) {
    dubiner(K, t.pq[2 * q], t.pq[2 * q + 1], v.data(), nullptr);
    for (int i = 0; i < P; ++i) t.Vp[q * P + i] = v[i];
  }
  // Dh[a][j][i] = int_That dpsi_i/dxi_a psi_j  (degree 2K-1: the volume rule is exact)
  t.Dh.assign(2 * t.NP * P, 0);
  for (int q = 0; q < t.nqv; ++q)
    for (int a = 0; a < 2; ++a)
      for (int j = 0; j < t.NP; ++j)
        for (int i = 0; i < P; ++i)
          t.Dh[(a * t.NP + j) * P + i] += t.vw[q] * t.Gv[(q * 2 + a) * P + i] * t.Vv[q * P + j];
  // Ch[f][m][i] = int_0^1 l_m(s) psi_i(xhat_f(s)) ds  (degree 2K: K+1 Gauss points)
  std::vector<double> cs, cw;
  gauss_legendre01(K + 1, cs, cw);
  t.Ch.assign(3 * t.NF * P, 0);
  for (int f = 0; f < 3; ++f)
    for (size_t r = 0; r < cs.size(); ++r) {
      double xh[2];
      ref_facet_point(f, cs[r], xh);
      dubiner(K, xh[0], xh[1], v.data(), nullptr);
      for (int m = 0; m < t.NF; ++m) {
        const double l = legendre01_orthonormal(m, cs[r]);
        for (int i = 0; i < P; ++i) t.Ch[(f * t.NF + m) * P + i] += cw[r] * l * v[i];
      }
    }
  // Zh: the divergence-free [P^K]^2 of the reference element is spanned by the curls
  // (d psi/d eta, -d psi/d xi) of the non-constant modes psi of P^{K+1} (the local basis of
  // eq. (FE4) built from stream functions).  Coefficients on the orthonormal P^K modes by
  // exact quadrature (degree 2K), then orthonormalised by modified Gram-Schmidt, twice.
  {
    const int P1 = nP(K + 1), ND = nDF(K), NU = 2 * P;
    std::vector<double> zp, zw, v1(P1), g1(2 * P1);
    triangle_rule(2 * K, zp, zw);
    std::vector<double> Zc((size_t)(P1 - 1) * NU, 0.0);
    for (size_t q = 0; q < zw.size(); ++q) {
      dubiner(K, zp[2 * q], zp[2 * q + 1], v.data(), nullptr);
      dubiner(K + 1, zp[2 * q], zp[2 * q + 1], v1.data(), g1.data());
      for (int b = 1; b < P1; ++b)
        for (int i = 0; i < P; ++i) {
          Zc[(size_t)(b - 1) * NU + 0 * P + i] += zw[q] * g1[P1 + b] * v[i];
          Zc[(size_t)(b - 1) * NU + 1 * P + i] -= zw[q] * g1[b] * v[i];
        }
    }
    for (int r = 0; r < ND; ++r) {
      double* zr = &Zc[(size_t)r * NU];
      for (int pass = 0; pass < 2; ++pass)
        for (int l = 0; l < r; ++l) {
          const double* zl = &Zc[(size_t)l * NU];
          double d = 0;
          for (int x = 0; x < NU; ++x) d += zl[x] * zr[x];
          for (int x = 0; x < NU; ++x) zr[x] -= d * zl[x];
        }
      double n2 = 0;
      for (int x = 0; x < NU; ++x) n2 += zr[x] * zr[x];
      const double inv = 1.0 / std::sqrt(n2);  // n2 > 0: the curl is injective modulo constants
      for (int x = 0; x < NU; ++x) zr[x] *= inv;
    }
    t.Zh = Zc;  // [r][c][i] with r < ND = P1 - 1
  }
}

// ---------------------------------------------------------------------------------------
// Mesh: periodic facet matching
// ---------------------------------------------------------------------------------------

// a == b modulo the period (per[d] = 0: no period in direction d; then relative to ext[d])
static bool same_mod(const double* a, const double* b, const double* per, const double* ext, double tol) {
  for (int d = 0; d < 2; ++d) {
    double x;
    if (per[d] > 0) {
      x = (a[d] - b[d]) / per[d];
      x -= std::nearbyint(x);
    } else {
      x = (a[d] - b[d]) / ext[d];
    }
    if (std::fabs(x) > tol) return false;
  }
  return true;
}

int build_mesh(int T, const double* xyz, const double* period, MeshHost& m, std::string& err) {
  m.T = T;
  m.xyz.assign(xyz, xyz + 6 * (size_t)T);
  m.period[0] = period[0];
  m.period[1] = period[1];
  double scale = 0;
  for (size_t i = 0; i < m.xyz.size(); ++i) scale = std::max(scale, std::fabs(m.xyz[i]));
  scale = std::max(scale, std::max(period[0], period[1]));
  // a direction without period (period 0) has walls: facets there keep one side; keys and
  // the facet ordering use the coordinate relative to the mesh's extent instead
  double ext[2] = {period[0], period[1]};
  for (int d = 0; d < 2; ++d)
    if (!(period[d] > 0)) {
      double mx = 0;
      for (size_t i = d; i < m.xyz.size(); i += 2) mx = std::max(mx, std::fabs(m.xyz[i]));
      ext[d] = 2.0 * mx + 1.0;
    }
  const bool walls = !(period[0] > 0) || !(period[1] > 0);
  auto rel = [&](double x, int d) {  // position in [0, 1): modulo the period, or within the extent
    if (period[d] > 0) {
      const double r = x / period[d];
      return r - std::floor(r);
    }
    return x / ext[d] + 0.5;
  };
  for (int t = 0; t < T; ++t) {
    const double* v = &m.xyz[6 * (size_t)t];
    double det = (v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1]);
    if (!(det > 1e-14 * scale * scale)) {
      err = "element " + std::to_string(t) + " is inverted or degenerate (det J = " + std::to_string(det) +
            "); vertices must be counter-clockwise";
      return -2;
    }
  }
  m.efacet.assign(3 * (size_t)T, -1);
  m.fL.clear(); m.fLloc.clear(); m.fR.clear(); m.fRloc.clear(); m.frev.clear();
  std::unordered_map<uint64_t, int> first;
  first.reserve(3 * (size_t)T);
  const double Q = 1073741824.0;  // 2^30
  for (int t = 0; t < T; ++t)
    for (int f = 0; f < 3; ++f) {
      const double* a = &m.xyz[6 * (size_t)t + 2 * ((f + 1) % 3)];
      const double* b = &m.xyz[6 * (size_t)t + 2 * ((f + 2) % 3)];
      uint64_t key = 0;
      for (int d = 0; d < 2; ++d) {
        const double mid = rel(0.5 * (a[d] + b[d]), d);
        long long q = std::llround(mid * Q) % (long long)Q;
        key = (key << 32) | (uint64_t)q;
      }
      auto it = first.find(key);
      if (it == first.end()) {
        const int F = (int)m.fL.size();
        first.emplace(key, F);
        m.fL.push_back(t); m.fLloc.push_back(f);
        m.fR.push_back(-1); m.fRloc.push_back(-1); m.frev.push_back(0);
        m.efacet[3 * t + f] = F;
      } else {
        const int F = it->second;
        if (m.fR[F] >= 0) {
          err = "facet matched by more than two elements (element " + std::to_string(t) + ")";
          return -2;
        }
        const int L = m.fL[F], fl = m.fLloc[F];
        if (L == t) {
          err = "element " + std::to_string(t) + " is adjacent to itself across the periodic boundary";
          return -2;
        }
        const double* la = &m.xyz[6 * (size_t)L + 2 * ((fl + 1) % 3)];
        const double* lb = &m.xyz[6 * (size_t)L + 2 * ((fl + 2) % 3)];
        int rev;
        if (same_mod(a, lb, period, ext, 1e-9) && same_mod(b, la, period, ext, 1e-9)) rev = 1;
        else if (same_mod(a, la, period, ext, 1e-9) && same_mod(b, lb, period, ext, 1e-9)) rev = 0;
        else {
          err = "facet endpoints of elements " + std::to_string(L) + " and " + std::to_string(t) +
                " do not match modulo the period";
          return -2;
        }
        m.fR[F] = t; m.fRloc[F] = f; m.frev[F] = (uint8_t)rev;
        m.efacet[3 * t + f] = F;
        first.erase(it);
      }
    }
  if (!first.empty() && !walls) {
    err = std::to_string(first.size()) + " facets have no periodic partner (a boundary needs a period component 0)";
    return -2;
  }
  m.E = (int)m.fL.size();
  // Number the facets along a Morton curve of their midpoints (modulo the period), so that
  // the facet system and the multigrid hierarchy keep neighbours close in memory whatever
  // the element numbering of the caller.
  {
    const int E = m.E;
    std::vector<uint64_t> key(E);
    for (int F = 0; F < E; ++F) {
      const int t = m.fL[F], f = m.fLloc[F];
      const double* a = &m.xyz[6 * (size_t)t + 2 * ((f + 1) % 3)];
      const double* b = &m.xyz[6 * (size_t)t + 2 * ((f + 2) % 3)];
      uint32_t q[2];
      for (int d = 0; d < 2; ++d) {
        const double mid = rel(0.5 * (a[d] + b[d]), d);
        q[d] = (uint32_t)std::min(65535.0, std::max(0.0, std::floor(mid * 65536.0)));
      }
      uint64_t k = 0;
      for (int bit = 15; bit >= 0; --bit) k = (k << 2) | (((q[1] >> bit) & 1u) << 1) | ((q[0] >> bit) & 1u);
      key[F] = (k << 32) | (uint32_t)F;  // ties keep the first-occurrence order
    }
    std::vector<int> order(E);
    for (int F = 0; F < E; ++F) order[F] = F;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return key[x] < key[y]; });
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

// Cholesky inverse of a small SPD matrix (row-major n x n) in place; false if not SPD.
bool spd_inverse(int n, double* A) {
  std::vector<double> L(n * n, 0.0), Li(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
      if (i == j) {
        if (!(s > 0)) return false;
        L[i * n + i] = std::sqrt(s);
      } else {
        L[i * n + j] = s / L[j * n + j];
      }
    }
  for (int i = 0; i < n; ++i) {
    Li[i * n + i] = 1.0 / L[i * n + i];
    for (int j = 0; j < i; ++j) {
      double s = 0;
      for (int k = j; k < i; ++k) s -= L[i * n + k] * Li[k * n + j];
      Li[i * n + j] = s / L[i * n + i];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int k = std::max(i, j); k < n; ++k) s += Li[k * n + i] * Li[k * n + j];
      A[i * n + j] = s;
    }
  return true;
}

int build_setup(const MeshHost& m, int K, double alpha, HostSetup& h, std::string& err) {
  build_ref_tables(K, h.tabs);
  const RefTables& tb = h.tabs;
  const int T = m.T, E = m.E, P = tb.P, NP = tb.NP, NF = tb.NF, NU = 2 * P;
  h.T = T;
  h.E = E;
  h.K = K;
  h.Jinv.assign(4 * (size_t)T, 0);
  h.detJ.assign(T, 0);
  h.isq.assign(T, 0);
  h.nbr.assign(3 * (size_t)T, 0);
  h.code.assign(3 * (size_t)T, 0);
  h.efacet.assign(3 * (size_t)T, 0);
  h.nx.assign(3 * (size_t)T, 0);
  h.ny.assign(3 * (size_t)T, 0);
  h.flen.assign(3 * (size_t)T, 0);
  h.sig.assign(3 * (size_t)T, 0);
  h.sF.assign(3 * (size_t)T, 0);
  h.G.assign((size_t)nGpk(K) * T, 0);
  if (h.fe4) h.G4.assign((size_t)nG4pk(K) * T, 0);
  else h.G4.clear();
  h.qL.assign(E, 0);
  h.qR.assign(E, 0);
  h.zdef.assign(E, 0);
  h.cols.assign((size_t)kSlots * E, 0);
  h.vals.assign((size_t)kSlots * NF * NF * E, 0);
  h.dinv.assign((size_t)E * NF, 0);
  h.binv.assign((size_t)E * NF * NF, 0);

  std::vector<double> hT(T);
  for (int t = 0; t < T; ++t) {
    const double* v = &m.xyz[6 * (size_t)t];
    const double J00 = v[2] - v[0], J01 = v[4] - v[0], J10 = v[3] - v[1], J11 = v[5] - v[1];
    const double det = J00 * J11 - J01 * J10;
    h.detJ[t] = det;
    h.isq[t] = 1.0 / std::sqrt(det);
    h.Jinv[0 * (size_t)T + t] = J11 / det;   // dxi/dx
    h.Jinv[1 * (size_t)T + t] = -J01 / det;  // dxi/dy
    h.Jinv[2 * (size_t)T + t] = -J10 / det;  // deta/dx
    h.Jinv[3 * (size_t)T + t] = J00 / det;   // deta/dy
    hT[t] = std::sqrt(det);  // (d! |T|)^(1/d) with |T| = det/2
  }
  for (int t = 0; t < T; ++t) {
    const double* v = &m.xyz[6 * (size_t)t];
    for (int f = 0; f < 3; ++f) {
      const int F = m.efacet[3 * t + f];
      const bool isR = (m.fR[F] == t && m.fRloc[F] == f);
      const bool wall = m.fR[F] < 0;  // boundary facet: one side, nbr = -1
      const bool open = wall && !m.fopen.empty() && m.fopen[F];  // outflow boundary
      const int nb = isR ? m.fL[F] : m.fR[F];
      const int nbf = wall ? 0 : (isR ? m.fLloc[F] : m.fRloc[F]);
      const double* a = v + 2 * ((f + 1) % 3);
      const double* b = v + 2 * ((f + 2) % 3);
      const double tx = b[0] - a[0], ty = b[1] - a[1];
      const double len = std::sqrt(tx * tx + ty * ty);
      const size_t idx = (size_t)f * T + t;
      h.nbr[idx] = nb;
      h.code[idx] = nbf | (m.frev[F] << 2) | ((isR ? 1 : 0) << 3) | ((open ? 1 : 0) << 4);
      h.efacet[idx] = F;
      h.nx[idx] = ty / len;
      h.ny[idx] = -tx / len;
      h.flen[idx] = len;
      h.sig[idx] = alpha * K * K / (wall ? hT[t] : std::min(hT[t], hT[nb]));
      // the face rows of C_T: none on an outflow facet (no multiplier there, p = 0)
      h.sF[idx] = open ? 0.0 : std::sqrt(len / h.detJ[t]);
    }
  }
  double zz = 0;
  for (int F = 0; F < E; ++F) {
    h.qL[F] = m.fLloc[F] * NF * T + m.fL[F];
    h.qR[F] = m.fR[F] < 0 ? -1 : m.fRloc[F] * NF * T + m.fR[F];  // -1: boundary facet
    const double len = h.flen[(size_t)m.fLloc[F] * T + m.fL[F]];
    h.zdef[F] = std::sqrt(len);
    zz += len;
  }
  for (int F = 0; F < E; ++F) h.zdef[F] /= std::sqrt(zz);
  h.nearnull = h.zdef;
  h.singular = true;
  for (int F = 0; F < E; ++F)
    if (!m.fopen.empty() && m.fopen[F]) h.singular = false;
  if (!h.singular) std::fill(h.zdef.begin(), h.zdef.end(), 0.0);  // S is definite: no kernel

  // Element condensation (eq. (FE3)): D_T = sum_a Jinv[a][c] Dh[a], C_T rows of face f are
  // sqrt(|F|/det J) n_c Ch[f] (sign (-1)^m on the R side of a reversed facet: the L side's
  // Legendre parameter runs the other way)
  struct Tri : CondenseElement {
    const HostSetup& h;
    int T, NP, P, NF, NU;
    Tri(const HostSetup& hh, int t, int np, int p, int nf) : h(hh), T(t), NP(np), P(p), NF(nf), NU(2 * p) {}
    bool isR(int t, int f) const override { return (h.code[(size_t)f * T + t] >> 3) & 1; }
    void build(int t, double* D, double* C) const override {
      const RefTables& tb = h.tabs;
      const double Ji[2][2] = {{h.Jinv[0 * (size_t)T + t], h.Jinv[1 * (size_t)T + t]},
                               {h.Jinv[2 * (size_t)T + t], h.Jinv[3 * (size_t)T + t]}};
      for (int j = 0; j < NP; ++j)
        for (int c = 0; c < 2; ++c)
          for (int i = 0; i < P; ++i)
            D[j * NU + c * P + i] = Ji[0][c] * tb.Dh[(0 * NP + j) * P + i] + Ji[1][c] * tb.Dh[(1 * NP + j) * P + i];
      for (int f = 0; f < 3; ++f) {
        const size_t idx = (size_t)f * T + t;
        const bool flip = ((h.code[idx] >> 3) & 1) && ((h.code[idx] >> 2) & 1);
        const double n[2] = {h.nx[idx], h.ny[idx]};
        for (int mm = 0; mm < NF; ++mm) {
          const double sg = (flip && (mm & 1)) ? -1.0 : 1.0;
          for (int c = 0; c < 2; ++c)
            for (int i = 0; i < P; ++i)
              C[(f * NF + mm) * NU + c * P + i] = sg * h.sF[idx] * n[c] * tb.Ch[(f * NF + mm) * P + i];
        }
      }
    }
    // Z_T = (J (x) I_P) Zhat / sqrt(det J): the Piola image of the reference basis, which the
    // map keeps divergence-free; J = det J adj(Jinv)
    bool build_Z(int t, double* Z) const override {
      const RefTables& tb = h.tabs;
      const int ND = nDF(h.K);
      const double dt = h.detJ[t], is = h.isq[t];
      const double J[2][2] = {{dt * h.Jinv[3 * (size_t)T + t], -dt * h.Jinv[1 * (size_t)T + t]},
                              {-dt * h.Jinv[2 * (size_t)T + t], dt * h.Jinv[0 * (size_t)T + t]}};
      for (int c = 0; c < 2; ++c)
        for (int i = 0; i < P; ++i)
          for (int r = 0; r < ND; ++r)
            Z[(size_t)(c * P + i) * ND + r] =
                is * (J[c][0] * tb.Zh[((size_t)r * 2 + 0) * P + i] + J[c][1] * tb.Zh[((size_t)r * 2 + 1) * P + i]);
      return true;
    }
  } el(h, T, NP, P, NF);
  // boundary facets have no R side: its two blocks stay zero, with the row's own column
  for (int F = 0; F < E; ++F)
    if (m.fR[F] < 0)
      for (int s = 3; s < kSlots; ++s) h.cols[(size_t)s * E + F] = F;
  if (condense_elements(h, 3, NP, NU, NF, el, err)) return -2;
  // an outflow facet's row (and column) of S is zero: its multiplier is fixed to 0 by an
  // identity diagonal block and the zero right-hand side the element rows give it
  for (int F = 0; F < E; ++F)
    if (!m.fopen.empty() && m.fopen[F])
      for (int a = 0; a < NF; ++a) h.vals[(((size_t)0 * NF + a) * NF + a) * E + F] = 1.0;
  // merge repeated columns of a row (tiny periodic meshes) into their first slot
  for (int F = 0; F < E; ++F)
    for (int s = 1; s < kSlots; ++s)
      for (int s2 = 0; s2 < s; ++s2)
        if (h.cols[(size_t)s * E + F] == h.cols[(size_t)s2 * E + F]) {
          for (int a = 0; a < NF * NF; ++a) {
            h.vals[((size_t)s2 * NF * NF + a) * E + F] += h.vals[((size_t)s * NF * NF + a) * E + F];
            h.vals[((size_t)s * NF * NF + a) * E + F] = 0.0;
          }
          break;
        }
  std::vector<double> B(NF * NF);
  for (int F = 0; F < E; ++F) {
    for (int a = 0; a < NF; ++a) {
      const double d = h.vals[(((size_t)0 * NF + a) * NF + a) * E + F];
      if (!(d > 0)) {
        err = "facet matrix has a non-positive diagonal at facet " + std::to_string(F);
        return -2;
      }
      h.dinv[(size_t)F * NF + a] = 1.0 / d;
      for (int b = 0; b < NF; ++b) B[a * NF + b] = h.vals[(((size_t)0 * NF + a) * NF + b) * E + F];
    }
    if (!spd_inverse(NF, B.data())) {
      err = "facet diagonal block " + std::to_string(F) + " is not positive definite";
      return -2;
    }
    for (int a = 0; a < NF * NF; ++a) h.binv[(size_t)F * NF * NF + a] = B[a];
  }
  return 0;
}

// ---------------------------------------------------------------------------------------
// Element condensation on the host's cores
// ---------------------------------------------------------------------------------------
int condense_elements(HostSetup& h, int nfac, int NP, int NU, int NF, const CondenseElement& el, std::string& err) {
  const int T = h.T, E = h.E, NR = nfac * NF;
  // the R side's diagonal block of a face row is written here and added after the
  // parallel loop (the L side writes slot 0 itself), so no two threads write one value
  std::vector<double> diagR((size_t)E * NF * NF, 0.0);
  std::atomic<int> bad(-1);
  const int ND = h.fe4 ? NU - NP : 0;
  auto work = [&](int t0, int t1) {
    std::vector<double> D((size_t)NP * NU), DDt((size_t)NP * NP), C((size_t)NR * NU), CDt((size_t)NR * NP),
        X((size_t)NR * NP), ST((size_t)NR * NR), Z((size_t)NU * ND), ZZ((size_t)ND * ND), CZ((size_t)NR * ND),
        XZ((size_t)NR * ND);
    for (int t = t0; t < t1; ++t) {
      el.build(t, D.data(), C.data());
      for (int j = 0; j < NP; ++j)
        for (int l = 0; l < NP; ++l) {
          double s = 0;
          for (int x = 0; x < NU; ++x) s += D[(size_t)j * NU + x] * D[(size_t)l * NU + x];
          DDt[(size_t)j * NP + l] = s;
        }
      if (!spd_inverse(NP, DDt.data())) {
        int exp = -1;
        bad.compare_exchange_strong(exp, t);
        return;
      }
      for (int j = 0, p = 0; j < NP; ++j)
        for (int l = 0; l <= j; ++l, ++p) h.G[(size_t)p * T + t] = DDt[(size_t)j * NP + l];
      if (h.fe4) {  // eq. (FE4): S_T = (C Z)(Z^T Z)^{-1}(C Z)^T on the locally divergence-free basis
        if (!el.build_Z(t, Z.data())) {
          int exp = -1;
          bad.compare_exchange_strong(exp, t);
          return;
        }
        for (int a = 0; a < ND; ++a)
          for (int b = 0; b < ND; ++b) {
            double s = 0;
            for (int x = 0; x < NU; ++x) s += Z[(size_t)x * ND + a] * Z[(size_t)x * ND + b];
            ZZ[(size_t)a * ND + b] = s;
          }
        if (!spd_inverse(ND, ZZ.data())) {
          int exp = -1;
          bad.compare_exchange_strong(exp, t);
          return;
        }
        for (int j = 0, p = 0; j < ND; ++j)
          for (int l = 0; l <= j; ++l, ++p) h.G4[(size_t)p * T + t] = ZZ[(size_t)j * ND + l];
        for (int r = 0; r < NR; ++r)
          for (int a = 0; a < ND; ++a) {
            double s = 0;
            for (int x = 0; x < NU; ++x) s += C[(size_t)r * NU + x] * Z[(size_t)x * ND + a];
            CZ[(size_t)r * ND + a] = s;
          }
        for (int r = 0; r < NR; ++r)
          for (int a = 0; a < ND; ++a) {
            double s = 0;
            for (int b = 0; b < ND; ++b) s += CZ[(size_t)r * ND + b] * ZZ[(size_t)b * ND + a];
            XZ[(size_t)r * ND + a] = s;
          }
        for (int r = 0; r < NR; ++r)
          for (int c2 = 0; c2 <= r; ++c2) {
            double s = 0;
            for (int a = 0; a < ND; ++a) s += XZ[(size_t)r * ND + a] * CZ[(size_t)c2 * ND + a];
            ST[(size_t)r * NR + c2] = ST[(size_t)c2 * NR + r] = s;
          }
      }
      for (int r = 0; r < NR && !h.fe4; ++r)
        for (int j = 0; j < NP; ++j) {
          double s = 0;
          for (int x = 0; x < NU; ++x) s += C[(size_t)r * NU + x] * D[(size_t)j * NU + x];
          CDt[(size_t)r * NP + j] = s;
        }
      for (int r = 0; r < NR && !h.fe4; ++r)
        for (int j = 0; j < NP; ++j) {
          double s = 0;
          for (int l = 0; l < NP; ++l) s += CDt[(size_t)r * NP + l] * DDt[(size_t)l * NP + j];
          X[(size_t)r * NP + j] = s;
        }
      for (int r = 0; r < NR && !h.fe4; ++r)
        for (int c2 = 0; c2 <= r; ++c2) {
          double s = 0;
          for (int x = 0; x < NU; ++x) s += C[(size_t)r * NU + x] * C[(size_t)c2 * NU + x];
          for (int j = 0; j < NP; ++j) s -= X[(size_t)r * NP + j] * CDt[(size_t)c2 * NP + j];
          ST[(size_t)r * NR + c2] = ST[(size_t)c2 * NR + r] = s;
        }
      for (int f = 0; f < nfac; ++f) {
        const int F = h.efacet[(size_t)f * T + t];
        const bool isR = el.isR(t, f);
        for (int f2 = 0; f2 < nfac; ++f2) {
          const int F2 = h.efacet[(size_t)f2 * T + t];
          if (f2 == f) {
            double* dst = isR ? &diagR[(size_t)F * NF * NF] : nullptr;
            for (int a = 0; a < NF; ++a)
              for (int b = 0; b < NF; ++b) {
                const double v = ST[((size_t)f * NF + a) * NR + f2 * NF + b];
                if (isR) dst[a * NF + b] = v;
                else h.vals[(((size_t)0 * NF + a) * NF + b) * E + F] = v;
              }
            if (!isR) h.cols[F] = F;
            continue;
          }
          const int slot = (isR ? nfac : 1) + ((f2 - f + nfac) % nfac) - 1;
          h.cols[(size_t)slot * E + F] = F2;
          for (int a = 0; a < NF; ++a)
            for (int b = 0; b < NF; ++b)
              h.vals[(((size_t)slot * NF + a) * NF + b) * E + F] = ST[((size_t)f * NF + a) * NR + f2 * NF + b];
        }
      }
    }
  };
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if ((long)T < 4096L * nt) nt = std::max<long>(1, T / 4096) < nt ? (unsigned)std::max<long>(1, T / 4096) : nt;
  std::vector<std::thread> pool;
  const int chunk = (T + (int)nt - 1) / (int)nt;
  for (unsigned i = 0; i < nt; ++i) {
    const int t0 = (int)i * chunk, t1 = std::min(T, t0 + chunk);
    if (t0 < t1) pool.emplace_back(work, t0, t1);
  }
  for (auto& th : pool) th.join();
  if (bad.load() >= 0) {
    err = (h.fe4 ? "local divergence-free basis of element " : "divergence matrix of element ") +
          std::to_string(bad.load()) + " is rank deficient";
    return -2;
  }
  for (int F = 0; F < E; ++F)
    for (int a = 0; a < NF * NF; ++a) h.vals[(size_t)a * E + F] += diagR[(size_t)F * NF * NF + a];
  return 0;
}

}  // namespace dfdg
