// Host-side set-up structures (CPU only).
#pragma once
#include "dfdg_internal.h"

namespace dfdg {

// Periodic triangle mesh with matched facets.  Facet F is numbered at the first
// element (in element order) that touches it: that element is its L side, the facet
// parameter and normal are L's; R is the other side, frev[F] = 1 when R traverses the
// facet in the opposite direction (always, for consistently oriented meshes).
struct MeshHost {
  int T = 0, E = 0;
  std::vector<double> xyz;  // [T][3][2]
  double period[2] = {1, 1};
  std::vector<int> efacet;  // [T][3]
  std::vector<int> fL, fLloc, fR, fRloc;
  std::vector<uint8_t> frev;
};

// Everything uploaded to the device at bind time (layouts as in DevGeo / DevBsr).
struct HostSetup {
  int T = 0, E = 0, K = 0;
  RefTables tabs;
  std::vector<double> Jinv, detJ, isq, nx, ny, flen, sig, sF, G, zdef, vals, dinv, binv;
  std::vector<int> nbr, code, efacet, qL, qR, cols;
};

int build_mesh(int T, const double* xyz, const double* period, MeshHost& m, std::string& err);
int build_setup(const MeshHost& m, int K, double alpha, HostSetup& h, std::string& err);

}  // namespace dfdg
