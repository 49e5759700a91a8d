// Smoothed-aggregation algebraic multigrid hierarchy for the facet matrix S (host set-up).
#pragma once
#include <string>
#include <vector>

namespace dfdg {

struct Csr {
  int n = 0, m = 0;              // rows, columns
  std::vector<int> ptr, col;     // ptr[n+1]
  std::vector<double> val;
  long nnz() const { return (long)col.size(); }
};

// One level below the finest: its operator A (scalar CSR), the prolongator P from it to
// the finer level (rows: finer unknowns) and R = P^T.  Level 0 is S itself (BSR on the
// device, given as CSR here).
struct AmgLevel {
  Csr A;            // operator of this level
  std::vector<double> dinv;
  double lmax = 0;  // spectral radius estimate of D^{-1} A (Chebyshev upper bound)
  Csr P;            // prolongator from the next coarser level to this one (empty on the coarsest)
  Csr R;            // restriction = P^T
  Csr AP, RA;       // A P and R A = (A P)^T, kept on levels >= 1 that have a coarser level
};

struct AmgHierarchy {
  std::vector<AmgLevel> lv;          // lv[0] = fine operator S
  std::vector<double> coarse_inv;    // dense pseudo-inverse (n_c x n_c) of the coarsest operator
  int n_coarse = 0;
};

// Builds the hierarchy for the BSR facet matrix (cols [NS][E], vals [NS][NF][NF][E]) with the
// near-null vector z (the constant multiplier, scalar length E*NF); singular: z spans the
// kernel of S (the coarsest level is then inverted as a pseudo-inverse that leaves out the
// coarse image of z), else S is definite and so is every level.  fine_smooth: damped-Jacobi
// steps applied to the finest level's tentative prolongator (1 or more; one below it).
// theta: strength threshold;
// coarsening stops at max_coarse rows, or earlier (at most 4096 rows) when aggregation
// no longer halves the level.
int build_amg(int E, int NF, int NS, const std::vector<int>& cols, const std::vector<double>& vals,
              const std::vector<double>& z, bool singular, double theta, int max_coarse, int fine_smooth,
              AmgHierarchy& H, std::string& err);

}  // namespace dfdg
