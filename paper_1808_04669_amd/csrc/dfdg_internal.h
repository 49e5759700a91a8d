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
// dim of the locally divergence-free [P^K(T)]^2 (curls of P^{K+1} modulo constants), and its
// packed Gram inverse (the reduced local space of eq. (FE4))
__host__ __device__ constexpr int nDF(int K) { return 2 * nP(K) - nPp(K); }
__host__ __device__ constexpr int nG4pk(int K) { return nDF(K) * (nDF(K) + 1) / 2; }
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
// Tetrahedra (d = 3): P = dim P^K(T), NP = dim P^{K-1}(T), NF = dim P^K(F); seven BSR blocks
// per face row (itself + the 3 other faces of each neighbour).  K = 1, 2.
__host__ __device__ constexpr int nP3(int K) { return (K + 1) * (K + 2) * (K + 3) / 6; }
__host__ __device__ constexpr int nPp3(int K) { return K * (K + 1) * (K + 2) / 6; }
__host__ __device__ constexpr int nF3(int K) { return (K + 1) * (K + 2) / 2; }
__host__ __device__ constexpr int nGpk3(int K) { return nPp3(K) * (nPp3(K) + 1) / 2; }
// Gauss-Jacobi collapsed tetrahedron rule exact for degree p: n^3 points, n = (p+2)/2
__host__ __device__ constexpr int tetN(int p) { return ((p + 2) / 2) * ((p + 2) / 2) * ((p + 2) / 2); }
__host__ __device__ constexpr int nQV3(int K) { return tetN(3 * K - 1); }       // residual volume rule
__host__ __device__ constexpr int nQF3(int K) { return K == 1 ? 6 : 12; }      // symmetric face rule
__host__ __device__ constexpr int nQP3(int K) { return tetN(2 * K + 2); }      // projection rule
constexpr int kMaxK3 = 2;
constexpr int kSlots3 = 7;
// 32-bit words of a facet row of S in FP16, two values per word
__host__ __device__ constexpr int nPairs(int NF, int NS) { return (NS * NF * NF + 1) / 2; }
// Threads per facet row in the facet-system kernels: 2 for the 252-value rows of
// tetrahedral meshes at k = 2 (each thread takes half the row's outputs), else 1.
__host__ __device__ constexpr int facet_split(int NF, int NS) { return (NF % 2 == 0 && NS * NF * NF > 128) ? 2 : 1; }
constexpr int kMaxEvalPts = 1024;

// ---- reference tabulations (host, FP64) ---------------------------------------------
struct RefTables {
  int dim = 2;
  int K = 0, P = 0, NP = 0, NF = 0, nqv = 0, nqf = 0, nqp = 0;
  std::vector<double> vq, vw;        // volume rule points [nqv][2], weights (sum 1/2)
  std::vector<double> fs, fw;        // facet rule on [0,1], symmetric
  std::vector<double> pq, pw;        // projection rule
  std::vector<double> Vv, Gv;        // psi_i at volume points [q][i], grads [q][a][i]
  std::vector<double> Vf, Gf;        // per local facet [f][r][i], [f][r][a][i]
  std::vector<double> Vp;            // projection points [q][i]
  std::vector<double> Dh;            // [a][j][i] = int dpsi_i/dxi_a psi_j, j < NP
  std::vector<double> Ch;            // [f][m][i] = int_0^1 l_m(s) psi_i(xhat_f(s)) ds
  // triangles: orthonormal basis of the reference element's divergence-free [P^K]^2 (the
  // reference curls of the P^{K+1} modes, orthonormalised), [r][c][i], r < nDF(K)
  std::vector<double> Zh;
  // tetrahedra: rules in 3 reference coordinates ([n][3]), 4 faces; a face point r seen from
  // the neighbour through vertex permutation p (0..5) is the neighbour's point fpidx[p][r];
  // Qf[p][m][n] = <mu_m(face param q), mu_n(own face param)> for the face parameter q that
  // permutation p maps the own one to (orthogonal change of the face basis)
  std::vector<int> fpidx;            // [6][nqf]
  std::vector<double> Qf;            // [6][NF][NF]
};
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);
void triangle_rule(int degree, std::vector<double>& pts, std::vector<double>& w);
// Volume rule of the residual for degree K (nQV(K) points, exact for degree 3K-1).
void residual_volume_rule(int K, std::vector<double>& pts, std::vector<double>& w);
void dubiner(int K, double xi, double eta, double* vals, double* grads /*[2][P] or null*/);
// Jacobi polynomial P_n^{(a,b)}(x) and its derivative (three-term recurrence)
void jacobi_poly(int n, double a, double b, double x, double* val, double* der);
double legendre01_orthonormal(int m, double s);
void build_ref_tables(int K, RefTables& t);
// tetrahedra
void dubiner3(int K, double xi, double eta, double zeta, double* vals, double* grads /*[3][P] or null*/);
void tet_rule(int degree, std::vector<double>& pts, std::vector<double>& w);
void sym_face_rule(int degree, std::vector<double>& pts, std::vector<double>& w);
void build_ref_tables3(int K, RefTables& t);
bool spd_inverse(int n, double* A);

// ---- device-side views --------------------------------------------------------------
struct DevGeo {
  int T, E;
  int fgrid;            // blocks of the facet-row kernels (grid-stride loops over the rows)
  // triangles unless stated; tetrahedra: Jinv [9][T] at (3r+j)*T + t, per-face arrays
  // [4][T], code bits 0-1 neighbour's local face, 2-4 the permutation p (0..5) carrying
  // this element's face vertices to the neighbour's, bit 5 this element is the R side;
  // qL/qR offsets into a [4][NF][T] array; nz the normal's third component
  const double* Jinv;   // [4][T], Jinv[r][j] = dxi_r/dx_j at (2r+j)*T + t
  const double* detJ;   // [T]  (> 0)
  const double* isq;    // [T]  1 / sqrt(detJ)
  const int* nbr;       // [3][T] neighbour across local facet f
  const int* code;      // [3][T] bits 0-1 neighbour's local facet, bit 2 reversed parameter,
                        //        bit 3 this element is the R side of the facet
  const int* efacet;    // [3][T] facet id
  const double* nx;     // [3][T] outward normal
  const double* ny;
  const double* nz;     // tetrahedra: [4][T]
  const double* flen;   // [3][T] |F|
  const double* sig;    // [3][T] alpha k^2 / h_F
  const double* sF;     // [3][T] sqrt(|F| / detJ)
  const double* G;      // [nGpk][T] packed lower triangle of (D_T D_T^T)^{-1}
  // reduced local space of eq. (FE4) (triangles, dfdg_params.local_space), else null:
  // [nG4pk][T] packed lower triangle of (Z_T^T Z_T)^{-1}, Z_T = (J (x) I_P) Zhat / sqrt(det J)
  // the element's locally divergence-free basis (Piola image of Zhat)
  const double* G4;
  const int* qL;        // [E] f_L*NF*T + L : base of L's contribution in a [3][NF][T] array
  const int* qR;        // [E]
  const double* zdef;   // [E] normalised kernel vector of S (component m = 0)
};
struct DevTabs {
  const double* Vv; const double* Gv; const double* Wv;
  const double* Vf; const double* Gf; const double* Wf;
  const double* Vp; const double* Wp;
  const double* Dh; const double* Ch;
  const double* Zh;                    // triangles: RefTables::Zh
  const int* fpidx; const double* Qf;  // tetrahedra: face point and face basis permutations
};
struct DevBsr {
  int ns;               // blocks per row: 5 (triangles) or 7 (tetrahedra)
  // matrix-free products of the FP64 PCG (tetrahedra, dfdg_params.matrix_free): S p is formed
  // element by element as sum_T C_T W_T C_T^T p from the element data and the reference
  // tables below, through the per-element face contributions mfq [4][NF][T]; null = BSR
  double* mfq;
  const double* mfCh; const double* mfDh; const double* mfQf;
  int mfK;
  const int* cols;      // [5][E]
  const double* vals;   // [5][NF][NF][E]
  const double* dinv;   // [E][NF]       point Jacobi
  const double* binv;   // [E][NF][NF]   facet-block Jacobi
  const float* vals32;  // [5][NF][NF][E] (MIXED)
  const float* dinv32;  // [E][NF]
  const float* binv32;  // [E][NF][NF]
  // FP16 copy of S / scale16 for the finest V-cycle level, or null: [nPairs(NF, ns)][E] words;
  // word j of row F holds values 2j (low half) and 2j+1 (high half) of the row's
  // [5][NF][NF] sequence (the last high half is zero when 5 NF^2 is odd)
  const uint32_t* vals16;
  float scale16;
  // S D^{-1} z for the kernel vector z of S (zdef on mode 0), [E][NF] in FP64 and in FP32
  // (multigrid contexts, else null): the fused update and first smoothing step removes the
  // kernel component of S p from the residual and needs S D^{-1} of it
  const double* tdef;
  const float* tdef32;
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
