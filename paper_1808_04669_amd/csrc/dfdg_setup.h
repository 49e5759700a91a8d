// Host-side set-up structures (CPU only).
#pragma once
#include "dfdg_internal.h"

namespace dfdg {

// Periodic triangle mesh with matched facets.  Facet F is numbered at the first
// element (in element order) that touches it: that element is its L side, the facet
// parameter and normal are L's; R is the other side, frev[F] = 1 when R traverses the
// facet in the opposite direction (always, for consistently oriented meshes).
struct MeshHost {
  int dim = 2;
  int T = 0, E = 0;
  std::vector<double> xyz;  // [T][3][2] triangles, [T][4][3] tetrahedra
  double period[3] = {1, 1, 1};
  std::vector<int> efacet;  // [T][3] or [T][4]
  std::vector<int> fL, fLloc, fR, fRloc;
  std::vector<uint8_t> fopen;  // [E] or empty: 1 = outflow boundary facet (open), else closed
  std::vector<uint8_t> frev;  // triangles: R traverses the facet in the opposite direction;
                              // tetrahedra: permutation id p (L's face vertex i is R's
                              // face vertex kFacePerm[p][i])
};
// The six permutations of a face's three vertices (id = index in this list).
extern const int kFacePerm[6][3];
int face_perm_id(const int p[3]);
int face_perm_inverse(int id);

// Everything uploaded to the device at bind time (layouts as in DevGeo / DevBsr).
struct HostSetup {
  int T = 0, E = 0, K = 0;
  RefTables tabs;
  int dim = 2;
  std::vector<double> Jinv, detJ, isq, nx, ny, nz, flen, sig, sF, G, zdef, vals, dinv, binv;
  // sqrt|F| on mode 0, normalised: the kernel vector of S on meshes without an outflow
  // boundary (then zdef = nearnull), the multigrid's near-null vector on every mesh
  std::vector<double> nearnull;
  bool singular = true;  // S has the constant multiplier as its kernel (no outflow facet)
  // reduced local space (eq. (FE4)): set before build_setup; G4 as DevGeo::G4
  bool fe4 = false;
  std::vector<double> G4;
  std::vector<int> nbr, code, efacet, qL, qR, cols;
};

int build_mesh(int T, const double* xyz, const double* period, MeshHost& m, std::string& err);

// Element condensation of eq. (FE3) with the orthonormal basis (M_T = I), for all elements on
// the host's cores: build(t, D, C) fills element t's divergence matrix D [NP][NU] and face rows
// C [nfac*NF][NU] (each face's rows in its L side's basis); the packed (D D^T)^{-1} goes to
// h.G and S_T = C W_T C^T = C C^T - (C D^T)(D D^T)^{-1}(D C^T) (W_T = I - D^T (D D^T)^{-1} D
// is never formed) into the face rows of h.vals / h.cols: slot 0 the face itself, slots
// 1..nfac-1 the other faces of its L element, nfac..2nfac-2 those of its R element (in local
// order f+1, f+2, ...).  isR(t, f): element t is the R side of its local face f.
//
// With h.fe4 the condensation takes the route of eq. (FE4) instead: build_Z(t, Z) fills the
// element's locally divergence-free basis Z [NU][ND], the packed (Z^T Z)^{-1} goes to h.G4
// and S_T = (C Z)(Z^T Z)^{-1}(C Z)^T (the same operator: Z (Z^T Z)^{-1} Z^T = W_T).
struct CondenseElement {
  virtual void build(int t, double* D, double* C) const = 0;
  virtual bool isR(int t, int f) const = 0;
  virtual bool build_Z(int /*t*/, double* /*Z*/) const { return false; }
  virtual ~CondenseElement() = default;
};
int condense_elements(HostSetup& h, int nfac, int NP, int NU, int NF, const CondenseElement& el, std::string& err);
int build_setup(const MeshHost& m, int K, double alpha, HostSetup& h, std::string& err);
int build_mesh3(int T, const double* xyz, const double* period, MeshHost& m, std::string& err);
int build_setup3(const MeshHost& m, int K, double alpha, HostSetup& h, std::string& err);

}  // namespace dfdg
