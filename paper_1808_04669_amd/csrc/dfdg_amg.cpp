// Smoothed-aggregation AMG set-up for the facet matrix S (host, FP64, deterministic).
//
// S is the statically condensed hybrid-mixed operator (eq. (FE3)); on a periodic mesh its
// kernel is the constant multiplier, which is also the near-null space the coarse levels
// must represent.  Each level: a strength graph (|a_ij| >= theta sqrt(a_ii a_jj), on the
// mode-0 entries of the facet blocks for the finest level), greedy aggregation (roots whose
// neighbourhood is free, then attachment, then leftovers), a tentative prolongator carrying
// the near-null vector aggregate by aggregate, damped-Jacobi smoothing of the prolongator
// (weight 4/(3 rho(D^{-1}A)); a set number of steps on the finest level, one below), and
// the Galerkin product R A P with R = P^T.
// The coarsest operator is inverted densely after adding its (near-)kernel direction; the
// inverse is then projected onto the complement of that direction (a pseudo-inverse).
#include "dfdg_amg.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <thread>

namespace dfdg {

// fn(chunk, begin, end) over kChunks fixed row ranges of [0, n), on up to 16 host threads.
// The ranges do not depend on the thread count, so per-chunk partial results combined in
// chunk order give the same bits on every host.
static constexpr int kChunks = 64;
template <typename Fn>
static void parallel_chunks(int n, Fn fn) {
  const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto range = [&](int c, int& b, int& e) {
    b = (int)((long)n * c / kChunks);
    e = (int)((long)n * (c + 1) / kChunks);
  };
  if (nt == 1 || n < 2 * kChunks) {
    for (int c = 0; c < kChunks; ++c) {
      int b, e;
      range(c, b, e);
      fn(c, b, e);
    }
    return;
  }
  std::vector<std::thread> pool;
  for (int w = 0; w < nt; ++w)
    pool.emplace_back([&, w]() {
      for (int c = w; c < kChunks; c += nt) {
        int b, e;
        range(c, b, e);
        fn(c, b, e);
      }
    });
  for (auto& th : pool) th.join();
}

// distinct columns of facet row F, sorted (tiny periodic meshes repeat a column in two slots)
static int row_columns(int E, int NS, const std::vector<int>& cols, int F, int* cs) {
  int nu = 0;
  for (int s = 0; s < NS; ++s) {
    const int c = cols[(size_t)s * E + F];
    bool seen = false;
    for (int t = 0; t < nu; ++t) seen |= (cs[t] == c);
    if (!seen) cs[nu++] = c;
  }
  std::sort(cs, cs + nu);
  return nu;
}

static Csr bsr_to_csr(int E, int NF, int NS, const std::vector<int>& cols, const std::vector<double>& vals) {
  Csr A;
  A.n = A.m = E * NF;
  A.ptr.assign(A.n + 1, 0);
  std::vector<int> nus(E);
  parallel_chunks(E, [&](int, int b, int e) {
    std::vector<int> cs(NS);
    for (int F = b; F < e; ++F) nus[F] = row_columns(E, NS, cols, F, cs.data());
  });
  for (int F = 0; F < E; ++F)
    for (int a = 0; a < NF; ++a) A.ptr[F * NF + a + 1] = A.ptr[F * NF + a] + nus[F] * NF;
  A.col.resize(A.ptr[A.n]);
  A.val.resize(A.ptr[A.n]);
  parallel_chunks(E, [&](int, int b, int e) {
    std::vector<int> cs(NS);
    for (int F = b; F < e; ++F) {
      const int nu = row_columns(E, NS, cols, F, cs.data());
      for (int a = 0; a < NF; ++a) {
        int k = A.ptr[F * NF + a];
        for (int t = 0; t < nu; ++t)
          for (int bb = 0; bb < NF; ++bb, ++k) {
            double v = 0;
            for (int s = 0; s < NS; ++s)
              if (cols[(size_t)s * E + F] == cs[t]) v += vals[(((size_t)s * NF + a) * NF + bb) * E + F];
            A.col[k] = cs[t] * NF + bb;
            A.val[k] = v;
          }
      }
    }
  });
  return A;
}

static void spmv(const Csr& A, const std::vector<double>& x, std::vector<double>& y) {
  y.assign(A.n, 0.0);
  parallel_chunks(A.n, [&](int, int b, int e) {
    for (int i = b; i < e; ++i) {
      double s = 0;
      for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) s += A.val[k] * x[A.col[k]];
      y[i] = s;
    }
  });
}

static std::vector<double> diag_inv(const Csr& A) {
  std::vector<double> d(A.n, 0.0);
  parallel_chunks(A.n, [&](int, int b, int e) {
    for (int i = b; i < e; ++i)
      for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
        if (A.col[k] == i) d[i] = 1.0 / A.val[k];
  });
  return d;
}

// Spectral radius of D^{-1} A by power iteration from a fixed pseudo-random start.
static double rho_dinv_a(const Csr& A, const std::vector<double>& dinv, int iters = 40) {
  std::vector<double> x(A.n), y;
  uint64_t s = 0x9E3779B97F4A7C15ull;
  for (int i = 0; i < A.n; ++i) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    x[i] = (double)(s >> 11) / 9007199254740992.0 - 0.5;
  }
  double lam = 0;
  std::vector<double> pny(kChunks), pnx(kChunks);
  for (int it = 0; it < iters; ++it) {
    spmv(A, x, y);
    parallel_chunks(A.n, [&](int c, int b, int e) {
      double sy = 0, sx = 0;
      for (int i = b; i < e; ++i) {
        y[i] *= dinv[i];
        sy += y[i] * y[i];
        sx += x[i] * x[i];
      }
      pny[c] = sy;
      pnx[c] = sx;
    });
    double ny = 0, nx = 0;
    for (int c = 0; c < kChunks; ++c) {
      ny += pny[c];
      nx += pnx[c];
    }
    lam = std::sqrt(ny / nx);
    const double inv = 1.0 / std::sqrt(ny);
    for (int i = 0; i < A.n; ++i) x[i] = y[i] * inv;
  }
  return lam;
}

// T = A^T with the entries of each row of T in increasing column order (the serial
// scatter's order): each chunk of A's rows counts its columns, the chunks' offsets within
// every row of T follow in chunk order, and each chunk then scatters its own entries.
static Csr transpose(const Csr& A) {
  Csr T;
  T.n = A.m;
  T.m = A.n;
  T.ptr.assign(T.n + 1, 0);
  std::vector<std::vector<int>> cnt(kChunks);
  parallel_chunks(A.n, [&](int ch, int b, int e) {
    cnt[ch].assign(A.m, 0);
    for (int k = A.ptr[b]; k < A.ptr[e]; ++k) cnt[ch][A.col[k]]++;
  });
  for (int c = 0; c < A.m; ++c) {  // cnt becomes each chunk's start in row c of T
    int run = 0;
    for (int ch = 0; ch < kChunks; ++ch) {
      const int n = cnt[ch].empty() ? 0 : cnt[ch][c];
      if (!cnt[ch].empty()) cnt[ch][c] = run;
      run += n;
    }
    T.ptr[c + 1] = T.ptr[c] + run;
  }
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  parallel_chunks(A.n, [&](int ch, int b, int e) {
    std::vector<int>& pos = cnt[ch];
    for (int i = b; i < e; ++i)
      for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        const int c = A.col[k];
        const int p = T.ptr[c] + pos[c]++;
        T.col[p] = i;
        T.val[p] = A.val[k];
      }
  });
  return T;
}

// C = A B (Gustavson with a dense accumulator); columns of each row sorted.  Row ranges
// run on the host's threads, each into its own buffers, joined in row order.
static Csr matmul(const Csr& A, const Csr& B) {
  Csr C;
  C.n = A.n;
  C.m = B.m;
  C.ptr.assign(C.n + 1, 0);
  std::vector<std::vector<int>> pc(kChunks);
  std::vector<std::vector<double>> pv(kChunks);
  std::vector<int> rowlen(A.n);
  parallel_chunks(A.n, [&](int ch, int b, int e) {
    std::vector<double> acc(B.m, 0.0);
    std::vector<int> mark(B.m, -1), touched;
    auto& oc = pc[ch];
    auto& ov = pv[ch];
    for (int i = b; i < e; ++i) {
      touched.clear();
      for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        const int j = A.col[k];
        const double a = A.val[k];
        for (int l = B.ptr[j]; l < B.ptr[j + 1]; ++l) {
          const int c = B.col[l];
          if (mark[c] != i) {
            mark[c] = i;
            acc[c] = 0;
            touched.push_back(c);
          }
          acc[c] += a * B.val[l];
        }
      }
      std::sort(touched.begin(), touched.end());
      for (int c : touched) {
        oc.push_back(c);
        ov.push_back(acc[c]);
      }
      rowlen[i] = (int)touched.size();
    }
  });
  for (int i = 0; i < A.n; ++i) C.ptr[i + 1] = C.ptr[i] + rowlen[i];
  C.col.reserve(C.ptr[C.n]);
  C.val.reserve(C.ptr[C.n]);
  for (int ch = 0; ch < kChunks; ++ch) {
    C.col.insert(C.col.end(), pc[ch].begin(), pc[ch].end());
    C.val.insert(C.val.end(), pv[ch].begin(), pv[ch].end());
  }
  return C;
}

// One damped-Jacobi step on a prolongator: (I - omega D^{-1} A) P, rows merged in column
// order (both operands' rows are sorted), exact zeros dropped; row ranges on the host's threads.
static Csr smooth_prolongator(const Csr& A, const std::vector<double>& dinv, double omega, const Csr& Pin) {
  const Csr AP = matmul(A, Pin);
  Csr P;
  P.n = Pin.n;
  P.m = Pin.m;
  P.ptr.assign(P.n + 1, 0);
  std::vector<std::vector<int>> pc(kChunks);
  std::vector<std::vector<double>> pv(kChunks);
  std::vector<int> rowlen(P.n);
  parallel_chunks(P.n, [&](int ch, int b0, int e0) {
    for (int r = b0; r < e0; ++r) {
      int a = Pin.ptr[r], b = AP.ptr[r], len = 0;
      while (a < Pin.ptr[r + 1] || b < AP.ptr[r + 1]) {
        int c;
        double v = 0;
        if (b >= AP.ptr[r + 1] || (a < Pin.ptr[r + 1] && Pin.col[a] < AP.col[b])) {
          c = Pin.col[a];
          v = Pin.val[a++];
        } else if (a >= Pin.ptr[r + 1] || AP.col[b] < Pin.col[a]) {
          c = AP.col[b];
          v = -omega * dinv[r] * AP.val[b++];
        } else {
          c = Pin.col[a];
          v = Pin.val[a++] - omega * dinv[r] * AP.val[b++];
        }
        if (v != 0.0) {
          pc[ch].push_back(c);
          pv[ch].push_back(v);
          ++len;
        }
      }
      rowlen[r] = len;
    }
  });
  for (int r = 0; r < P.n; ++r) P.ptr[r + 1] = P.ptr[r] + rowlen[r];
  for (int ch = 0; ch < kChunks; ++ch) {
    P.col.insert(P.col.end(), pc[ch].begin(), pc[ch].end());
    P.val.insert(P.val.end(), pv[ch].begin(), pv[ch].end());
  }
  return P;
}

// Greedy aggregation of the nodes of a symmetric strength graph (adjacency lists).
static int aggregate(int n, const std::vector<int>& gptr, const std::vector<int>& gadj, std::vector<int>& agg) {
  agg.assign(n, -1);
  int na = 0;
  for (int i = 0; i < n; ++i) {  // 1: roots with a free neighbourhood
    if (agg[i] >= 0) continue;
    bool free = true;
    for (int k = gptr[i]; k < gptr[i + 1] && free; ++k) free = agg[gadj[k]] < 0;
    if (!free) continue;
    agg[i] = na;
    for (int k = gptr[i]; k < gptr[i + 1]; ++k) agg[gadj[k]] = na;
    ++na;
  }
  std::vector<int> pending(n, -1);
  for (int i = 0; i < n; ++i) {  // 2: attach to a neighbouring aggregate
    if (agg[i] >= 0) continue;
    for (int k = gptr[i]; k < gptr[i + 1]; ++k)
      if (agg[gadj[k]] >= 0) {
        pending[i] = agg[gadj[k]];
        break;
      }
  }
  for (int i = 0; i < n; ++i)
    if (pending[i] >= 0) agg[i] = pending[i];
  for (int i = 0; i < n; ++i) {  // 3: leftovers with their free neighbours
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int k = gptr[i]; k < gptr[i + 1]; ++k)
      if (agg[gadj[k]] < 0) agg[gadj[k]] = na;
    ++na;
  }
  return na;
}

// In-place inverse of a dense SPD matrix (row-major) by Cholesky; every inner loop runs
// along contiguous rows.
static bool dense_spd_inverse(int n, std::vector<double>& A) {
  const size_t N = (size_t)n;
  std::vector<double> L(N * N, 0.0);
  for (int i = 0; i < n; ++i) {
    const double* Li = &L[i * N];
    for (int j = 0; j <= i; ++j) {
      const double* Lj = &L[j * N];
      double s = A[i * N + j];
      for (int k = 0; k < j; ++k) s -= Li[k] * Lj[k];
      if (i == j) {
        if (!(s > 0)) return false;
        L[i * N + i] = std::sqrt(s);
      } else {
        L[i * N + j] = s / L[j * N + j];
      }
    }
  }
  // M = L^{-1}, row by row: row_i(M) = (e_i - sum_{k<i} L_ik row_k(M)) / L_ii
  std::vector<double> M(N * N, 0.0);
  for (int i = 0; i < n; ++i) {
    double* Mi = &M[i * N];
    Mi[i] = 1.0;
    for (int k = 0; k < i; ++k) {
      const double l = L[i * N + k];
      if (l == 0.0) continue;
      const double* Mk = &M[k * N];
      for (int j = 0; j <= k; ++j) Mi[j] -= l * Mk[j];
    }
    const double d = 1.0 / L[i * N + i];
    for (int j = 0; j <= i; ++j) Mi[j] *= d;
  }
  // A^{-1} = M^T M = sum_k row_k(M)^T row_k(M)
  std::fill(A.begin(), A.end(), 0.0);
  for (int k = 0; k < n; ++k) {
    const double* Mk = &M[k * N];
    for (int i = 0; i <= k; ++i) {
      const double a = Mk[i];
      if (a == 0.0) continue;
      double* Ai = &A[i * N];
      for (int j = 0; j <= i; ++j) Ai[j] += a * Mk[j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) A[j * N + i] = A[i * N + j];
  return true;
}

int build_amg(int E, int NF, int NS, const std::vector<int>& cols, const std::vector<double>& vals,
              const std::vector<double>& z, bool singular, double theta, int max_coarse, int fine_smooth,
              AmgHierarchy& H, std::string& err) {
  H.lv.clear();
  AmgLevel L0;
  L0.A = bsr_to_csr(E, NF, NS, cols, vals);
  std::vector<double> B = z;  // near-null vector on the current level
  int nf = NF;                // unknowns per node on the current level
  H.lv.push_back(std::move(L0));
  for (int level = 0; level < 20; ++level) {
    AmgLevel& L = H.lv.back();
    L.dinv = diag_inv(L.A);
    for (double d : L.dinv)
      if (!(d > 0) || !std::isfinite(d)) {
        err = "multigrid: non-positive diagonal on level " + std::to_string(level);
        return -1;
      }
    L.lmax = rho_dinv_a(L.A, L.dinv);
    const int n = L.A.n;
    if (n <= max_coarse) break;
    // strength graph on nodes
    const int nn = n / nf;
    std::vector<int> gptr(nn + 1, 0), gadj;
    std::vector<double> dd(nn);
    for (int i = 0; i < nn; ++i) dd[i] = std::fabs(1.0 / L.dinv[i * nf]);
    for (int i = 0; i < nn; ++i) {
      const int row = i * nf;  // mode-0 row of the node
      std::vector<int> nb;
      for (int k = L.A.ptr[row]; k < L.A.ptr[row + 1]; ++k) {
        const int c = L.A.col[k];
        if (c % nf != 0) continue;
        const int j = c / nf;
        if (j == i) continue;
        if (std::fabs(L.A.val[k]) >= theta * std::sqrt(dd[i] * dd[j])) nb.push_back(j);
      }
      std::sort(nb.begin(), nb.end());
      nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
      gadj.insert(gadj.end(), nb.begin(), nb.end());
      gptr[i + 1] = (int)gadj.size();
    }
    // symmetrise the graph (strength measure is symmetric for symmetric A; be safe)
    {
      std::vector<std::vector<int>> adj(nn);
      for (int i = 0; i < nn; ++i)
        for (int k = gptr[i]; k < gptr[i + 1]; ++k) {
          adj[i].push_back(gadj[k]);
          adj[gadj[k]].push_back(i);
        }
      gadj.clear();
      for (int i = 0; i < nn; ++i) {
        std::sort(adj[i].begin(), adj[i].end());
        adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
        gadj.insert(gadj.end(), adj[i].begin(), adj[i].end());
        gptr[i + 1] = (int)gadj.size();
      }
    }
    std::vector<int> agg;
    const int na = aggregate(nn, gptr, gadj, agg);
    if (na >= nn) break;                  // no coarsening possible
    if (2 * na > nn && n <= 4096) break;  // coarsening stalls: invert this level densely
    // tentative prolongator: the near-null vector, normalised per aggregate
    std::vector<double> nrm(na, 0.0);
    for (int r = 0; r < n; ++r) nrm[agg[r / nf]] += B[r] * B[r];
    for (double& v : nrm) v = std::sqrt(v);
    Csr Pt;
    Pt.n = n;
    Pt.m = na;
    Pt.ptr.assign(n + 1, 0);
    for (int r = 0; r < n; ++r) {
      const int a = agg[r / nf];
      if (B[r] != 0.0 && nrm[a] > 0) {
        Pt.col.push_back(a);
        Pt.val.push_back(B[r] / nrm[a]);
      }
      Pt.ptr[r + 1] = (int)Pt.col.size();
    }
    // smoothed prolongator P = (I - omega D^{-1} A)^m Pt: m = fine_smooth steps on the
    // finest level (a wider, better interpolation where the two-grid rate is set), one below
    const double omega = 4.0 / (3.0 * L.lmax);
    Csr P = std::move(Pt);
    const int steps = level == 0 ? fine_smooth : 1;
    for (int st = 0; st < steps; ++st) P = smooth_prolongator(L.A, L.dinv, omega, P);
    Csr R = transpose(P);
    Csr AP = matmul(L.A, P);
    Csr Ac = matmul(R, AP);
    if (level > 0) {  // for the fused transfer kernels of the coarse levels
      L.RA = transpose(AP);
      L.AP = std::move(AP);
    }
    L.P = std::move(P);
    L.R = std::move(R);
    AmgLevel next;
    next.A = std::move(Ac);
    H.lv.push_back(std::move(next));
    B = nrm;
    nf = 1;
  }
  // coarsest: dense inverse of A_c + s B B^T / (B.B) (adds the kernel direction)
  AmgLevel& C = H.lv.back();
  const int nc = C.A.n;
  if (nc > 4096) {
    err = "multigrid: coarsest level too large (" + std::to_string(nc) + ")";
    return -1;
  }
  std::vector<double> D((size_t)nc * nc, 0.0);
  double tr = 0;
  for (int i = 0; i < nc; ++i)
    for (int k = C.A.ptr[i]; k < C.A.ptr[i + 1]; ++k) {
      D[(size_t)i * nc + C.A.col[k]] = C.A.val[k];
      if (C.A.col[k] == i) tr += C.A.val[k];
    }
  double bb = 0;
  if (singular)
    for (int i = 0; i < nc; ++i) bb += B[i] * B[i];
  const double s = tr / nc;
  if (bb > 0)
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nc; ++j) D[(size_t)i * nc + j] += s * B[i] * B[j] / bb;
  if (!dense_spd_inverse(nc, D)) {
    err = "multigrid: coarsest operator is not positive definite";
    return -1;
  }
  // Pseudo-inverse of A_c: Q D Q with Q = I - B B^T / (B.B), so that the coarse solve
  // neither reads nor returns a kernel component.  The inverse of the shifted operator
  // alone returns the residual's kernel component (pure rounding) divided by s, the mean
  // coarse diagonal, which is small after several Galerkin products; near the attainable
  // accuracy that component dominates the search direction, (p, S p) loses its sign and
  // the PCG diverges.
  if (bb > 0) {
    std::vector<double> Db((size_t)nc, 0.0);
    double bDb = 0;
    for (int i = 0; i < nc; ++i) {
      double t = 0;
      for (int j = 0; j < nc; ++j) t += D[(size_t)i * nc + j] * B[j];
      Db[i] = t;
    }
    for (int i = 0; i < nc; ++i) bDb += B[i] * Db[i];
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nc; ++j)
        D[(size_t)i * nc + j] += (-Db[i] * B[j] - B[i] * Db[j] + B[i] * B[j] * bDb / bb) / bb;
  }
  H.coarse_inv = std::move(D);
  H.n_coarse = nc;
  return 0;
}

}  // namespace dfdg
