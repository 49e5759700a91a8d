// Internal declarations shared by the host setup, the C ABI and the HIP kernels.
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#if !defined(__HIPCC__) && !defined(__host__)
#define __host__
#define __device__
#endif

namespace dfdg {

// ---- compile-time sizes of the degree-K discretisation -----------------------------
__host__ __device__ constexpr int nP(int K) { return (K + 1) * (K + 2) / 2; }    // dim P^K(T)
__host__ __device__ constexpr int nPp(int K) { return K * (K + 1) / 2; }         // dim P^{K-1}(T)
__host__ __device__ constexpr int nF(int K) { return K + 1; }                    // dim P^K(F)
__host__ __device__ constexpr int nGpk(int K) { return nPp(K) * (nPp(K) + 1) / 2; }  // packed (D D^T)^{-1}
// Collapsed Gauss-Legendre triangle rule exact for degree p: nu x nv points.
__host__ __device__ constexpr int triNu(int p) { return (p + 2) / 2; }
__host__ __device__ constexpr int triNv(int p) { return (p + 3) / 2; }
__host__ __device__ constexpr int triN(int p) { return triNu(p) * triNv(p); }
// Residual rules: volume exact for degree 3K-1 ((u x u) : grad v), facet Gauss-Legendre
// exact for degree 3K (u.n u.v on the facet).  The volume rule is a fully symmetric one
// for K = 1 (3 points, degree 2) and K = 2 (7 points, degree 5), else the collapsed rule.
__host__ __device__ constexpr int nQV(int K) { return K == 1 ? 3 : K == 2 ? 7 : triN(3 * K - 1); }
__host__ __device__ constexpr int nQF(int K) { return (3 * K + 2) / 2; }
// Projection rule (initial data): exact for degree 2K+4.
__host__ __device__ constexpr int projDeg(int K) { return 2 * K + 4; }
__host__ __device__ constexpr int nQP(int K) { return triN(projDeg(K)); }
constexpr int kMaxK = 3;
constexpr int kSlots = 5;           // BSR blocks per facet row: itself + 2 + 2 neighbours
// 32-bit words of a facet row of S in FP16, two values per word
__host__ __device__ constexpr int nPairs(int NF) { return (kSlots * NF * NF + 1) / 2; }
constexpr int kMaxEvalPts = 1024;

// ---- reference tabulations (host, FP64) ---------------------------------------------
struct RefTables {
  int K = 0, P = 0, NP = 0, NF = 0, nqv = 0, nqf = 0, nqp = 0;
  std::vector<double> vq, vw;        // volume rule points [nqv][2], weights (sum 1/2)
  std::vector<double> fs, fw;        // facet rule on [0,1], symmetric
  std::vector<double> pq, pw;        // projection rule
  std::vector<double> Vv, Gv;        // psi_i at volume points [q][i], grads [q][a][i]
  std::vector<double> Vf, Gf;        // per local facet [f][r][i], [f][r][a][i]
  std::vector<double> Vp;            // projection points [q][i]
  std::vector<double> Dh;            // [a][j][i] = int dpsi_i/dxi_a psi_j, j < NP
  std::vector<double> Ch;            // [f][m][i] = int_0^1 l_m(s) psi_i(xhat_f(s)) ds
};
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);
void triangle_rule(int degree, std::vector<double>& pts, std::vector<double>& w);
// Volume rule of the residual for degree K (nQV(K) points, exact for degree 3K-1).
void residual_volume_rule(int K, std::vector<double>& pts, std::vector<double>& w);
void dubiner(int K, double xi, double eta, double* vals, double* grads /*[2][P] or null*/);
double legendre01_orthonormal(int m, double s);
void build_ref_tables(int K, RefTables& t);

// ---- device-side views --------------------------------------------------------------
struct DevGeo {
  int T, E;
  int fgrid;            // blocks of the facet-row kernels (grid-stride loops over the rows)
  const double* Jinv;   // [4][T], Jinv[r][j] = dxi_r/dx_j at (2r+j)*T + t
  const double* detJ;   // [T]  (> 0)
  const double* isq;    // [T]  1 / sqrt(detJ)
  const int* nbr;       // [3][T] neighbour across local facet f
  const int* code;      // [3][T] bits 0-1 neighbour's local facet, bit 2 reversed parameter,
                        //        bit 3 this element is the R side of the facet
  const int* efacet;    // [3][T] facet id
  const double* nx;     // [3][T] outward normal
  const double* ny;
  const double* flen;   // [3][T] |F|
  const double* sig;    // [3][T] alpha k^2 / h_F
  const double* sF;     // [3][T] sqrt(|F| / detJ)
  const double* G;      // [nGpk][T] packed lower triangle of (D_T D_T^T)^{-1}
  const int* qL;        // [E] f_L*NF*T + L : base of L's contribution in a [3][NF][T] array
  const int* qR;        // [E]
  const double* zdef;   // [E] normalised kernel vector of S (component m = 0)
};
struct DevTabs {
  const double* Vv; const double* Gv; const double* Wv;
  const double* Vf; const double* Gf; const double* Wf;
  const double* Vp; const double* Wp;
  const double* Dh; const double* Ch;
};
struct DevBsr {
  const int* cols;      // [5][E]
  const double* vals;   // [5][NF][NF][E]
  const double* dinv;   // [E][NF]       point Jacobi
  const double* binv;   // [E][NF][NF]   facet-block Jacobi
  const float* vals32;  // [5][NF][NF][E] (MIXED)
  const float* dinv32;  // [E][NF]
  const float* binv32;  // [E][NF][NF]
  // FP16 copy of S / scale16 for the finest V-cycle level, or null: [nPairs(NF)][E] words;
  // word j of row F holds values 2j (low half) and 2j+1 (high half) of the row's
  // [5][NF][NF] sequence (the last high half is zero when 5 NF^2 is odd)
  const uint32_t* vals16;
  float scale16;
};

// Scalars of one PCG run (device memory).  Written by block 0 of a kernel (or by a
// one-block finishing kernel) and read by later kernels and by the host.
struct PcgScalars {
  double rz, rr, gg, tol2, zg;
  double rr0;  // (r, r) at the start of the run (written with the first iteration)
  int iters, done, maxit, zero_rhs;
  int it;      // index of the next iteration (set to 1 at the start, advanced by the update kernel)
  int pad;
};
enum { PCG_RUNNING = 0, PCG_CONVERGED = 1, PCG_BREAKDOWN = 2, PCG_MAXIT = 3, PCG_NONFINITE = 4 };

}  // namespace dfdg
