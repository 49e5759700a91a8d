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
  std::vector<int> nbr, code, efacet, qL, qR, cols;
};

int build_mesh(int T, const double* xyz, const double* period, MeshHost& m, std::string& err);
int build_setup(const MeshHost& m, int K, double alpha, HostSetup& h, std::string& err);
int build_mesh3(int T, const double* xyz, const double* period, MeshHost& m, std::string& err);
int build_setup3(const MeshHost& m, int K, double alpha, HostSetup& h, std::string& err);

}  // namespace dfdg
