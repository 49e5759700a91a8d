// HIP kernels of the hot path for gfx950 (CDNA4, 64-wide wavefronts).
//
// Element-centred kernels run one thread per element and read the SoA velocity layout
// [2][P][T] (consecutive lanes, consecutive elements: coalesced).  Facet-centred kernels
// run one thread per facet row of the BSR facet matrix S (n_f x n_f blocks, 5 per row),
// whose values are stored SoA [slot][a][b][E] so that every load instruction of a wave is
// one contiguous 512-byte segment.  Facet vectors are [E][n_f].
//
// Reductions (PCG dot products) are deterministic and use neither atomics nor fences: each
// block reduces its lanes with wavefront shuffles and LDS and writes one partial; the next
// kernel's blocks each sum all partials in the same fixed order.  (A per-block device-scope
// release fence would write back the XCD's whole L2 on every block.)
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <mutex>

#include "dfdg_device.h"
#include "dfdg_internal.h"
#include "dfdg_kernels.h"

namespace dfdg {

// ---------------------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------------------

// ---------------------------------------------------------------------------------------
// element helpers
// ---------------------------------------------------------------------------------------

// Apply W_T = I - D_T^T (D_T D_T^T)^{-1} D_T (the divergence-free projector of the
// element, eq. (FE3) with the orthonormal basis) in place to y[2][P].
template <int K, typename R>
__device__ inline void apply_W(R (&y)[2][nP(K)], const R (&Ji)[2][2], const double* __restrict__ G, int T, int t,
                               const double* __restrict__ Dh) {
  constexpr int P = nP(K), NP = nPp(K);
  R d[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    R s = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      R a0 = 0, a1 = 0;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        a0 += (R)Dh[(0 * NP + j) * P + i] * y[c][i];
        a1 += (R)Dh[(1 * NP + j) * P + i] * y[c][i];
      }
      s += Ji[0][c] * a0 + Ji[1][c] * a1;
    }
    d[j] = s;
  }
  R e[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) e[j] = 0;
#pragma unroll
  for (int j = 0, p = 0; j < NP; ++j)
#pragma unroll
    for (int l = 0; l <= j; ++l, ++p) {
      const R gv = (R)G[(size_t)p * T + t];
      e[j] += gv * d[l];
      if (l != j) e[l] += gv * d[j];
    }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      R s = 0;
#pragma unroll
      for (int j = 0; j < NP; ++j)
        s += (Ji[0][c] * (R)Dh[(0 * NP + j) * P + i] + Ji[1][c] * (R)Dh[(1 * NP + j) * P + i]) * e[j];
      y[c][i] -= s;
    }
  }
}

// The same projector computed on the reduced local space of eq. (FE4):
// W_T = Z_T (Z_T^T Z_T)^{-1} Z_T^T with the element's locally divergence-free basis
// Z_T = (J (x) I_P) Zhat / sqrt(det J) (the Piola image of the reference basis Zhat, so only
// J and the packed Gram inverse G4 are per element), J = det J adj(Jinv).
template <int K>
__device__ inline void apply_W4(double (&y)[2][nP(K)], const double (&Ji)[2][2], double det, double isq,
                                const double* __restrict__ G4, int T, int t, const double* Zh) {
  constexpr int P = nP(K), ND = nDF(K);
  const auto Z = cst(Zh);
  const double J[2][2] = {{det * Ji[1][1], -det * Ji[0][1]}, {-det * Ji[1][0], det * Ji[0][0]}};
  double x[2][P];  // J^T y: the reference components
#pragma unroll
  for (int i = 0; i < P; ++i) {
    x[0][i] = J[0][0] * y[0][i] + J[1][0] * y[1][i];
    x[1][i] = J[0][1] * y[0][i] + J[1][1] * y[1][i];
  }
  double h[ND];
#pragma unroll
  for (int r = 0; r < ND; ++r) {
    double s = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) s += Z[(r * 2 + 0) * P + i] * x[0][i] + Z[(r * 2 + 1) * P + i] * x[1][i];
    h[r] = isq * s;
  }
  double e[ND];
#pragma unroll
  for (int r = 0; r < ND; ++r) e[r] = 0;
#pragma unroll
  for (int j = 0, p = 0; j < ND; ++j)
#pragma unroll
    for (int l = 0; l <= j; ++l, ++p) {
      const double gv = G4[(size_t)p * T + t];
      e[j] += gv * h[l];
      if (l != j) e[l] += gv * h[j];
    }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double z0 = 0, z1 = 0;
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      z0 += Z[(r * 2 + 0) * P + i] * e[r];
      z1 += Z[(r * 2 + 1) * P + i] * e[r];
    }
    y[0][i] = isq * (J[0][0] * z0 + J[0][1] * z1);
    y[1][i] = isq * (J[1][0] * z0 + J[1][1] * z1);
  }
}

template <typename R>
__device__ inline void load_Jinv(const DevGeo& g, int t, R (&Ji)[2][2]) {
  Ji[0][0] = (R)g.Jinv[t];
  Ji[0][1] = (R)g.Jinv[(size_t)g.T + t];
  Ji[1][0] = (R)g.Jinv[2 * (size_t)g.T + t];
  Ji[1][1] = (R)g.Jinv[3 * (size_t)g.T + t];
}

// Stage the reference tables of the residual into LDS.
template <int K>
struct ResTabs {
  static constexpr int P = nP(K), NQV = nQV(K), NQF = nQF(K);
  double Vv[NQV][P], Gv[NQV][2][P], Wv[NQV];
  double Vf[3][NQF][P], Gf[3][NQF][2][P], Wf[NQF];
};
template <int K>
__device__ inline void stage_tabs(ResTabs<K>& s, const DevTabs& tb) {
  constexpr int P = nP(K), NQV = nQV(K), NQF = nQF(K);
  double* d;
  d = &s.Vv[0][0];
  for (int i = threadIdx.x; i < NQV * P; i += blockDim.x) d[i] = tb.Vv[i];
  d = &s.Gv[0][0][0];
  for (int i = threadIdx.x; i < NQV * 2 * P; i += blockDim.x) d[i] = tb.Gv[i];
  for (int i = threadIdx.x; i < NQV; i += blockDim.x) s.Wv[i] = tb.Wv[i];
  d = &s.Vf[0][0][0];
  for (int i = threadIdx.x; i < 3 * NQF * P; i += blockDim.x) d[i] = tb.Vf[i];
  d = &s.Gf[0][0][0][0];
  for (int i = threadIdx.x; i < 3 * NQF * 2 * P; i += blockDim.x) d[i] = tb.Gf[i];
  for (int i = threadIdx.x; i < NQF; i += blockDim.x) s.Wf[i] = tb.Wf[i];
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// a3: DG residual L(u)(v) = -C_h(u;u,v) - B_h(u,v) on the broken basis
// ---------------------------------------------------------------------------------------
// Each element integrates its volume term and its three facet terms, reading the
// neighbour's coefficients; a facet's flux is thus evaluated by both neighbours with the
// same operations in mirrored order (no atomics, bitwise symmetric).  With n the own
// outward normal, un = {u}.n, u_up the outflow-side value (un >= 0: own side),
// du = u_own - u_nbr, the facet contributes to the own test function v
//     -(un u_up - nu {grad u} n + nu sigma du) . v  +  (nu/2) (du (x) n) : grad v
// (upwind convection, consistency, penalty, symmetry terms of eqs. (adv), (viscous)).
// VISC = false is the instantiation for nu = 0 (the Euler equations): the viscous terms
// vanish identically and the gradients of u, the neighbour's inverse Jacobian and the
// penalty are neither read nor evaluated.
template <int K, typename R, bool VISC>
__global__ __launch_bounds__(kEBlk) void k_residual(DevGeo g, DevTabs tb, const double* __restrict__ U,
                                                    R* __restrict__ Lout, double nu_d) {
  constexpr int P = nP(K), NQV = nQV(K), NQF = nQF(K);
  __shared__ ResTabs<K> s;
  stage_tabs<K>(s, tb);
  const int T = g.T;
  const int t = xcd_block() * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const R nu = (R)nu_d;
  R u[2][P], acc[2][P];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < P; ++i) {
      u[c][i] = (R)U[(size_t)(c * P + i) * T + t];
      acc[c][i] = 0;
    }
  R Ji[2][2];
  load_Jinv(g, t, Ji);
  const R isq = (R)g.isq[t];

  // volume: int (u (x) u - nu grad u) : grad v.  With a = sum_i u_i psihat_i (so that
  // u = a / sqrt(det) at the point) and gr its reference gradient, the integrand times
  // the Jacobian det is  [isq a (x) a - nu gr Jinv] Jinv^T : grad_ref v  (isq = 1/sqrt(det)).
  for (int q = 0; q < NQV; ++q) {
    R uq[2], gr[2][2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      R a = 0, b0 = 0, b1 = 0;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        a += u[c][i] * (R)s.Vv[q][i];
        if constexpr (VISC) {
          b0 += u[c][i] * (R)s.Gv[q][0][i];
          b1 += u[c][i] * (R)s.Gv[q][1][i];
        }
      }
      uq[c] = a;
      gr[c][0] = b0;
      gr[c][1] = b1;
    }
    R Gt[2][2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      R fl[2];
      const R ua = isq * uq[c];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        fl[j] = ua * uq[j];
        if constexpr (VISC) fl[j] -= nu * (gr[c][0] * Ji[0][j] + gr[c][1] * Ji[1][j]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a) Gt[c][a] = fl[0] * Ji[a][0] + fl[1] * Ji[a][1];
    }
    // the weight folded into the flux: two fused multiply-adds per test function
    const R w = (R)s.Wv[q];
    R wG[2][2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int d = 0; d < 2; ++d) wG[c][d] = w * Gt[c][d];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < P; ++i)
        acc[c][i] = fma(wG[c][1], (R)s.Gv[q][1][i], fma(wG[c][0], (R)s.Gv[q][0][i], acc[c][i]));
  }

  // facets
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const size_t idx = (size_t)f * T + t;
    const int nb = g.nbr[idx];
    const int code = g.code[idx];
    // a boundary facet (nbr = -1) closed by a wall or an inflow: no term (u.n = 0 on a
    // wall; on an inflow the term acts on v.n only, which the stage increments keep 0);
    // the viscous facet terms run over interior facets only (free-slip natural)
    if (nb < 0 && !((code >> 4) & 1)) continue;
    if (nb < 0) {  // outflow: -int max(u.n, 0) (u . v), own trace (backflow sees zero)
      const R n0 = (R)g.nx[idx], n1 = (R)g.ny[idx];
      const R li = (R)g.flen[idx] * isq;
      for (int r = 0; r < NQF; ++r) {
        R uo[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          R a = 0;
#pragma unroll
          for (int i = 0; i < P; ++i) a += u[c][i] * (R)s.Vf[f][r][i];
          uo[c] = a * isq;
        }
        const R un = uo[0] * n0 + uo[1] * n1;
        if (un > (R)0) {
          const R w = (R)s.Wf[r] * li;
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const R wq = -(w * un * uo[c]);
#pragma unroll
            for (int i = 0; i < P; ++i) acc[c][i] = fma(wq, (R)s.Vf[f][r][i], acc[c][i]);
          }
        }
      }
      continue;
    }
    const int fn = code & 3;
    const bool rev = (code >> 2) & 1;
    const R n0 = (R)g.nx[idx], n1 = (R)g.ny[idx];
    const R len = (R)g.flen[idx];
    R v[2][P];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < P; ++i) v[c][i] = (R)U[(size_t)(c * P + i) * T + nb];
    const R isqn = (R)g.isq[nb];
    const R li = len * isq;
    R Jn[2][2] = {}, nJ[2] = {}, sig = 0;
    if constexpr (VISC) {
      sig = (R)g.sig[idx];
      load_Jinv(g, nb, Jn);
#pragma unroll
      for (int a = 0; a < 2; ++a) nJ[a] = n0 * Ji[a][0] + n1 * Ji[a][1];
    }
    for (int r = 0; r < NQF; ++r) {
      const int rn = rev ? NQF - 1 - r : r;
      R uo[2], un[2], go[2][2] = {}, gn[2][2] = {};
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        R a = 0, b0 = 0, b1 = 0, an = 0, bn0 = 0, bn1 = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
          a += u[c][i] * (R)s.Vf[f][r][i];
          an += v[c][i] * (R)s.Vf[fn][rn][i];
          if constexpr (VISC) {
            b0 += u[c][i] * (R)s.Gf[f][r][0][i];
            b1 += u[c][i] * (R)s.Gf[f][r][1][i];
            bn0 += v[c][i] * (R)s.Gf[fn][rn][0][i];
            bn1 += v[c][i] * (R)s.Gf[fn][rn][1][i];
          }
        }
        uo[c] = a * isq;
        un[c] = an * isqn;
        if constexpr (VISC) {
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            go[c][j] = isq * (b0 * Ji[0][j] + b1 * Ji[1][j]);
            gn[c][j] = isqn * (bn0 * Jn[0][j] + bn1 * Jn[1][j]);
          }
        }
      }
      const R unrm = (R)0.5 * ((uo[0] + un[0]) * n0 + (uo[1] + un[1]) * n1);
      const bool own_up = unrm >= (R)0;
      R Qv[2], du[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const R up = own_up ? uo[c] : un[c];
        du[c] = uo[c] - un[c];
        Qv[c] = unrm * up;
        if constexpr (VISC) {
          const R avgn = (R)0.5 * ((go[c][0] + gn[c][0]) * n0 + (go[c][1] + gn[c][1]) * n1);
          Qv[c] = Qv[c] - nu * avgn + nu * sig * du[c];
        }
      }
      const R w = (R)s.Wf[r] * li;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const R wq = -(w * Qv[c]);
        if constexpr (VISC) {
          const R wh = w * ((R)0.5 * nu * du[c]);
          const R wh0 = wh * nJ[0], wh1 = wh * nJ[1];
#pragma unroll
          for (int i = 0; i < P; ++i)
            acc[c][i] = fma(wq, (R)s.Vf[f][r][i],
                            fma(wh1, (R)s.Gf[f][r][1][i], fma(wh0, (R)s.Gf[f][r][0][i], acc[c][i])));
        } else {
#pragma unroll
          for (int i = 0; i < P; ++i) acc[c][i] = fma(wq, (R)s.Vf[f][r][i], acc[c][i]);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < P; ++i) Lout[(size_t)(c * P + i) * T + t] = acc[c][i];
}

// ---------------------------------------------------------------------------------------
// adjoint form: Ubar = J_L(U)^T Lbar
// ---------------------------------------------------------------------------------------
// With y the broken field of coefficients Lbar, (J_L^T Lbar)_j = d/dU_j [L(u)(y)].
// Viscous part: -B_h(phi_j, y) = -B_h(y, phi_j) (symmetric), i.e. the viscous residual of
// y.  Convective part (upwind side frozen): volume  +int (phi (x) u + u (x) phi) : grad y,
// i.e. phi . (grad y u + grad y^T u); facet (own-side test function phi, n own normal,
// dy = y_own - y_nbr)  -int [ 1/2 (phi.n)(u_up.dy) + un (phi.dy) [own side upwind] ].
template <int K>
__global__ __launch_bounds__(kEBlk) void k_residual_vjp(DevGeo g, DevTabs tb, const double* __restrict__ U,
                                                        const double* __restrict__ Y, double* __restrict__ Ubar,
                                                        double nu) {
  constexpr int P = nP(K), NQV = nQV(K), NQF = nQF(K);
  __shared__ ResTabs<K> s;
  stage_tabs<K>(s, tb);
  const int T = g.T;
  const int t = xcd_block() * blockDim.x + threadIdx.x;
  if (t >= T) return;
  double u[2][P], y[2][P], acc[2][P];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < P; ++i) {
      u[c][i] = U[(size_t)(c * P + i) * T + t];
      y[c][i] = Y[(size_t)(c * P + i) * T + t];
      acc[c][i] = 0;
    }
  double Ji[2][2];
  load_Jinv(g, t, Ji);
  const double det = g.detJ[t];
  const double isq = g.isq[t];
  const double sq = det * isq;
  for (int q = 0; q < NQV; ++q) {
    double uq[2], gy[2][2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double a = 0, b0 = 0, b1 = 0;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        a += u[c][i] * s.Vv[q][i];
        b0 += y[c][i] * s.Gv[q][0][i];
        b1 += y[c][i] * s.Gv[q][1][i];
      }
      uq[c] = a * isq;
#pragma unroll
      for (int j = 0; j < 2; ++j) gy[c][j] = isq * (b0 * Ji[0][j] + b1 * Ji[1][j]);
    }
    double av[2], Gt[2][2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      av[c] = gy[c][0] * uq[0] + gy[c][1] * uq[1] + gy[0][c] * uq[0] + gy[1][c] * uq[1];
#pragma unroll
      for (int a = 0; a < 2; ++a) Gt[c][a] = -nu * (gy[c][0] * Ji[a][0] + gy[c][1] * Ji[a][1]);
    }
    const double w = s.Wv[q] * sq;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < P; ++i)
        acc[c][i] += w * (av[c] * s.Vv[q][i] + Gt[c][0] * s.Gv[q][0][i] + Gt[c][1] * s.Gv[q][1][i]);
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const size_t idx = (size_t)f * T + t;
    const int nb = g.nbr[idx];
    const int code = g.code[idx];
    // closed boundary facets contribute nothing to the residual, nor to its transpose
    if (nb < 0 && !((code >> 4) & 1)) continue;
    if (nb < 0) {  // outflow: d/du of -int max(u.n, 0) (u . y) = -int H(u.n) [(phi.n)(u.y) + u.n (phi.y)]
      const double n0 = g.nx[idx], n1 = g.ny[idx];
      const double li = g.flen[idx] * isq;
      for (int r = 0; r < NQF; ++r) {
        double uo[2], yo[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          double a = 0, ya = 0;
#pragma unroll
          for (int i = 0; i < P; ++i) {
            a += u[c][i] * s.Vf[f][r][i];
            ya += y[c][i] * s.Vf[f][r][i];
          }
          uo[c] = a * isq;
          yo[c] = ya * isq;
        }
        const double un = uo[0] * n0 + uo[1] * n1;
        if (un > 0.0) {
          const double w = s.Wf[r] * li, uy = uo[0] * yo[0] + uo[1] * yo[1];
          const double Av[2] = {-(n0 * uy + un * yo[0]), -(n1 * uy + un * yo[1])};
#pragma unroll
          for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < P; ++i) acc[c][i] += w * Av[c] * s.Vf[f][r][i];
        }
      }
      continue;
    }
    const int fn = code & 3;
    const bool rev = (code >> 2) & 1;
    const double n0 = g.nx[idx], n1 = g.ny[idx], len = g.flen[idx], sig = g.sig[idx];
    double v[2][P], yn[2][P];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < P; ++i) {
        v[c][i] = U[(size_t)(c * P + i) * T + nb];
        yn[c][i] = Y[(size_t)(c * P + i) * T + nb];
      }
    double Jn[2][2];
    load_Jinv(g, nb, Jn);
    const double isqn = g.isq[nb];
    double nJ[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) nJ[a] = n0 * Ji[a][0] + n1 * Ji[a][1];
    for (int r = 0; r < NQF; ++r) {
      const int rn = rev ? NQF - 1 - r : r;
      double uo[2], un[2], yo[2], ynb[2], go[2][2], gn[2][2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double a = 0, an = 0, ya = 0, yan = 0, b0 = 0, b1 = 0, bn0 = 0, bn1 = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
          a += u[c][i] * s.Vf[f][r][i];
          an += v[c][i] * s.Vf[fn][rn][i];
          ya += y[c][i] * s.Vf[f][r][i];
          yan += yn[c][i] * s.Vf[fn][rn][i];
          b0 += y[c][i] * s.Gf[f][r][0][i];
          b1 += y[c][i] * s.Gf[f][r][1][i];
          bn0 += yn[c][i] * s.Gf[fn][rn][0][i];
          bn1 += yn[c][i] * s.Gf[fn][rn][1][i];
        }
        uo[c] = a * isq;
        un[c] = an * isqn;
        yo[c] = ya * isq;
        ynb[c] = yan * isqn;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          go[c][j] = isq * (b0 * Ji[0][j] + b1 * Ji[1][j]);
          gn[c][j] = isqn * (bn0 * Jn[0][j] + bn1 * Jn[1][j]);
        }
      }
      const double unrm = 0.5 * ((uo[0] + un[0]) * n0 + (uo[1] + un[1]) * n1);
      const bool own_up = unrm >= 0.0;
      double dy[2], upv[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        dy[c] = yo[c] - ynb[c];
        upv[c] = own_up ? uo[c] : un[c];
      }
      const double updy = upv[0] * dy[0] + upv[1] * dy[1];
      const double nn[2] = {n0, n1};
      double Av[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double avgn = 0.5 * ((go[c][0] + gn[c][0]) * n0 + (go[c][1] + gn[c][1]) * n1);
        const double conv = -(0.5 * nn[c] * updy + (own_up ? unrm * dy[c] : 0.0));
        Av[c] = conv + nu * avgn - nu * sig * dy[c];  // minus the viscous flux Q(y)
      }
      const double w = s.Wf[r] * len * isq;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double h = 0.5 * nu * dy[c];
#pragma unroll
        for (int i = 0; i < P; ++i)
          acc[c][i] += w * (Av[c] * s.Vf[f][r][i] + h * (nJ[0] * s.Gf[f][r][0][i] + nJ[1] * s.Gf[f][r][1][i]));
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < P; ++i) Ubar[(size_t)(c * P + i) * T + t] = acc[c][i];
}

// ---------------------------------------------------------------------------------------
// a4: condensation right-hand side, element part: q_{T,f} = C_{T,f} W_T F_T
// ---------------------------------------------------------------------------------------
// C_{T,f}: (C y)_m = sgn_m sqrt(|F|/detJ) sum_c n_c sum_i Chat_f[m][i] y[c][i], with
// sgn_m = (-1)^m when the element traverses the facet against the facet's parameter.
template <int K, typename FT, bool FE4>
__global__ __launch_bounds__(kEBlk) void k_cond_rhs(DevGeo g, DevTabs tb, const FT* __restrict__ F,
                                                    double* __restrict__ q) {
  constexpr int P = nP(K), NF = nF(K);
  const int T = g.T;
  const int t = xcd_block() * blockDim.x + threadIdx.x;
  if (t >= T) return;
  double y[2][P];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < P; ++i) y[c][i] = (double)F[(size_t)(c * P + i) * T + t];
  double Ji[2][2];
  load_Jinv(g, t, Ji);
  if constexpr (FE4) apply_W4<K>(y, Ji, g.detJ[t], g.isq[t], g.G4, T, t, tb.Zh);
  else apply_W<K, double>(y, Ji, g.G, T, t, tb.Dh);
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const size_t idx = (size_t)f * T + t;
    const int code = g.code[idx];
    const bool flip = ((code >> 3) & 1) && ((code >> 2) & 1);
    const double sc = g.sF[idx], n0 = g.nx[idx], n1 = g.ny[idx];
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      double a0 = 0, a1 = 0;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const double ch = tb.Ch[(f * NF + m) * P + i];
        a0 += ch * y[0][i];
        a1 += ch * y[1][i];
      }
      double val = sc * (n0 * a0 + n1 * a1);
      if (flip && (m & 1)) val = -val;
      q[(size_t)(f * NF + m) * T + t] = val;
    }
  }
}

// ---------------------------------------------------------------------------------------
// a6: recovery u_T = W_T (F_T - C_T^T lambda_T) with the RK3 combination epilogue
// ---------------------------------------------------------------------------------------
template <int K, typename FT, bool FE4>
// out may alias Un or Us: each thread reads its own entries before writing them.
__global__ __launch_bounds__(kEBlk) void k_recover(DevGeo g, DevTabs tb, const FT* __restrict__ F,
                                                   const double* __restrict__ lam, double* out, int mode, double ca,
                                                   const double* Un, double cb, const double* Us, double dt) {
  constexpr int P = nP(K), NF = nF(K);
  const int T = g.T;
  const int t = xcd_block() * blockDim.x + threadIdx.x;
  if (t >= T) return;
  double y[2][P];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < P; ++i) y[c][i] = (double)F[(size_t)(c * P + i) * T + t];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const size_t idx = (size_t)f * T + t;
    const int code = g.code[idx];
    const bool flip = ((code >> 3) & 1) && ((code >> 2) & 1);
    const double sc = g.sF[idx], n0 = g.nx[idx], n1 = g.ny[idx];
    const int Fi = g.efacet[idx];
    double lm[NF];
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      const double l = lam[(size_t)Fi * NF + m];
      lm[m] = (flip && (m & 1)) ? -l : l;
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      double s = 0;
#pragma unroll
      for (int m = 0; m < NF; ++m) s += lm[m] * tb.Ch[(f * NF + m) * P + i];
      y[0][i] -= sc * n0 * s;
      y[1][i] -= sc * n1 * s;
    }
  }
  double Ji[2][2];
  load_Jinv(g, t, Ji);
  if constexpr (FE4) apply_W4<K>(y, Ji, g.detJ[t], g.isq[t], g.G4, T, t, tb.Zh);
  else apply_W<K, double>(y, Ji, g.G, T, t, tb.Dh);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const size_t o = (size_t)(c * P + i) * T + t;
      if (mode == 0) out[o] = y[c][i];
      else out[o] = ca * Un[o] + cb * (Us[o] + dt * y[c][i]);
    }
}

// ---------------------------------------------------------------------------------------
// a5: facet PCG
// ---------------------------------------------------------------------------------------

// Facet kernels run a grid-stride loop over facet rows on a grid of at most kMaxFacetGrid
// blocks, so that the partial buffers (and the redundant reductions) stay small.
__host__ __device__ inline int facet_grid(int E) {
  const int g = (E + kBlk - 1) / kBlk;
  return g < kMaxFacetGrid ? g : kMaxFacetGrid;
}

// g_F = q_{L,f_L} + q_{R,f_R}; partials (g,g), (zdef,g) and (q_L,q_L) + (q_R,q_R), the size
// of the element contributions that the sum cancels.
template <int NF>
__global__ __launch_bounds__(kBlk) void k_gather_g(DevGeo g, const double* __restrict__ q, double* __restrict__ gv,
                                                   double* __restrict__ part) {
  const int T = g.T;
  double v[3] = {0, 0, 0};
  for (int F = blockIdx.x * blockDim.x + threadIdx.x; F < g.E; F += gridDim.x * blockDim.x) {
    const int a = g.qL[F], b = g.qR[F];  // b = -1: boundary facet, one side
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      const double qa = q[a + (size_t)m * T], qb = b >= 0 ? q[b + (size_t)m * T] : 0.0;
      const double x = qa + qb;
      gv[(size_t)F * NF + m] = x;
      v[0] += x * x;
      if (m == 0) v[1] += g.zdef[F] * x;
      v[2] += qa * qa + qb * qb;
    }
  }
  block_write_partial<3>(v, part);
}

// (zdef, x_{.,0}) partials, one per block.
template <int NF>
__global__ __launch_bounds__(kBlk) void k_zdot(DevGeo g, const double* __restrict__ x, double* __restrict__ part) {
  double v[1] = {0};
  for (int F = blockIdx.x * blockDim.x + threadIdx.x; F < g.E; F += gridDim.x * blockDim.x)
    v[0] += g.zdef[F] * x[(size_t)F * NF];
  block_write_partial<1>(v, part);
}

// x_{F,0} -= (zdef, x) zdef_F: removes the component of x along the kernel of S.
template <int NF>
__global__ __launch_bounds__(kBlk) void k_zdeflate(DevGeo g, double* __restrict__ x, const double* __restrict__ part,
                                                   int n) {
  double t[1];
  block_sum_partials<1>(part, n, t);
  for (int F = blockIdx.x * blockDim.x + threadIdx.x; F < g.E; F += gridDim.x * blockDim.x)
    x[(size_t)F * NF] -= t[0] * g.zdef[F];
}

// One block: the deflated (g,g) and the PCG stopping threshold.  A right-hand side at the
// rounding level of the contributions it is summed from (||g|| <= 1e-13 ||q||, e.g. data
// that is already divergence-free with a continuous normal component) counts as zero: the
// multiplier is zero up to that rounding.
__global__ __launch_bounds__(kBlk) void k_finalize_gather(const double* __restrict__ part, int n, PcgScalars* sc,
                                                          double rtol, int maxit) {
  double t[3];
  block_sum_partials<3>(part, n, t);
  if (threadIdx.x == 0) {
    const double gg = t[0] - t[1] * t[1];  // ||g - (z.g) z||^2 with ||z|| = 1
    sc->gg = gg;
    sc->zg = t[1];
    sc->tol2 = rtol * rtol * gg;
    sc->maxit = maxit;
    sc->zero_rhs = !(gg > 1e-26 * t[2]);
    sc->iters = 0;
    sc->it = 1;
    sc->rr = 0;
    sc->done = !isfinite(gg) ? PCG_NONFINITE : (sc->zero_rhs ? PCG_CONVERGED : PCG_RUNNING);
  }
}

template <int NF, bool BJ, typename V, typename M>
__device__ inline void precond(const DevBsr& A, int F, const V (&r)[NF], V (&z)[NF]) {
  if (BJ) {
    const M* B = (sizeof(V) == 8) ? (const M*)A.binv : (const M*)A.binv32;
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      V s = 0;
#pragma unroll
      for (int b = 0; b < NF; ++b) s += (V)B[((size_t)F * NF + a) * NF + b] * r[b];
      z[a] = s;
    }
  } else {
    const M* d = (sizeof(V) == 8) ? (const M*)A.dinv : (const M*)A.dinv32;
#pragma unroll
    for (int a = 0; a < NF; ++a) z[a] = (V)d[(size_t)F * NF + a] * r[a];
  }
}

// y = S x for row F (x given by a functor returning the NF-vector of a column facet); NS
// blocks per row.
template <int NF, int NS, typename V, typename M, typename Getter>
__device__ inline void spmv_row(const DevBsr& A, int E, int F, Getter get, V (&y)[NF]) {
  const M* vals = (sizeof(M) == 8) ? (const M*)A.vals : (const M*)A.vals32;
#pragma unroll
  for (int a = 0; a < NF; ++a) y[a] = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = A.cols[(size_t)s * E + F];
    V xc[NF];
    get(c, xc);
#pragma unroll
    for (int a = 0; a < NF; ++a)
#pragma unroll
      for (int b = 0; b < NF; ++b) y[a] += (V)vals[(((size_t)s * NF + a) * NF + b) * E + F] * xc[b];
  }
}

// The FP16 copy of row F of S (two values per word, see DevBsr::vals16): all the row's
// words are loaded at once, and value j of the row's [5][NF][NF] sequence is half j & 1
// of word j / 2.
template <int NF, int NS>
struct HalfRow {
  uint32_t w[nPairs(NF, NS)];
  __device__ inline void load(const DevBsr& A, int E, int F) {
    const uint32_t* __restrict__ p = A.vals16;
#pragma unroll
    for (int j = 0; j < nPairs(NF, NS); ++j) w[j] = p[(size_t)j * E + F];
  }
  __device__ inline float at(int j) const {
    const uint32_t v = w[j >> 1];
    return (float)__builtin_bit_cast(_Float16, (uint16_t)((j & 1) ? (v >> 16) : (v & 0xffffu)));
  }
};

// Facet rows of tetrahedral meshes (six modes, seven slots: 252 values) are shared by two
// threads, each computing three of the row's six outputs: half the registers per thread,
// twice the threads in flight, and the pair's column gathers fall on the same addresses.
// Rows of triangle meshes (at most 80 values) keep one thread each.  Thread unit u works
// on row u / kSplit and its outputs [NA (u % kSplit), NA (u % kSplit + 1)), NA = NF / kSplit.
template <int NF, int NS>
constexpr int kSplit = facet_split(NF, NS);

__device__ inline float half_at(const uint32_t* w, int j) {
  const uint32_t v = w[j >> 1];
  return (float)__builtin_bit_cast(_Float16, (uint16_t)((j & 1) ? (v >> 16) : (v & 0xffffu)));
}

// Outputs [a0, a0 + NA) of row F of S x in the multigrid's arithmetic V (get(c, x_c) gives
// the column facet's vector): S is read from its FP16 copy (scaled by scale16) when V is
// float and there is one, else from the FP32 (V float) or FP64 copy.  For split rows the
// thread's part of slot s is the NA NF values from (s NF + a0) NF on: whole words of the
// FP16 copy, since NF is even.
template <int NF, int NS, int NA, typename V, typename Getter>
__device__ inline void spmv_part_mg(const DevBsr& A, int E, int F, int a0, Getter get, V (&y)[NA]) {
#pragma unroll
  for (int a = 0; a < NA; ++a) y[a] = 0;
  if constexpr (sizeof(V) == 4) {
    if (A.vals16) {
      if constexpr (NA < NF) {
        static_assert(NF % 2 == 0, "split rows need whole FP16 words per part");
        constexpr int kW = NA * NF / 2;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const uint32_t* __restrict__ p = A.vals16 + (size_t)((s * NF * NF + a0 * NF) / 2) * E + F;
          uint32_t w[kW];
#pragma unroll
          for (int j = 0; j < kW; ++j) w[j] = p[(size_t)j * E];
          const int c = A.cols[(size_t)s * E + F];
          V xc[NF];
          get(c, xc);
#pragma unroll
          for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int b = 0; b < NF; ++b) y[a] += (V)half_at(w, a * NF + b) * xc[b];
        }
      } else {
        HalfRow<NF, NS> m;
        m.load(A, E, F);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int c = A.cols[(size_t)s * E + F];
          V xc[NF];
          get(c, xc);
#pragma unroll
          for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int b = 0; b < NF; ++b) y[a] += (V)m.at((s * NF + a) * NF + b) * xc[b];
        }
      }
#pragma unroll
      for (int a = 0; a < NA; ++a) y[a] *= A.scale16;
      return;
    }
  }
  const V* vals = (sizeof(V) == 8) ? (const V*)A.vals : (const V*)A.vals32;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = A.cols[(size_t)s * E + F];
    V xc[NF];
    get(c, xc);
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NF; ++b) y[a] += vals[(((size_t)s * NF + a0 + a) * NF + b) * E + F] * xc[b];
  }
}

// Two products of one row part at once, y1 = S u and y2 = S w (get(c, u_c, w_c) gives the
// column facet's two vectors), with the multigrid's copy of S as in spmv_part_mg.
template <int NF, int NS, int NA, typename V, typename Getter>
__device__ inline void spmv_part_mg2(const DevBsr& A, int E, int F, int a0, Getter get, V (&y1)[NA],
                                     V (&y2)[NA]) {
#pragma unroll
  for (int a = 0; a < NA; ++a) y1[a] = y2[a] = 0;
  // value(s, a, b) gives entry (a0 + a, b) of block s of the row
  auto rowloop = [&](auto value) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int c = A.cols[(size_t)s * E + F];
      V uc[NF], wc[NF];
      get(c, uc, wc);
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NF; ++b) {
          const V m = value(s, a, b);
          y1[a] += m * uc[b];
          y2[a] += m * wc[b];
        }
    }
  };
  if constexpr (sizeof(V) == 4) {
    if (A.vals16) {
      if constexpr (NA < NF) {
        static_assert(NF % 2 == 0, "split rows need whole FP16 words per part");
        constexpr int kW = NA * NF / 2;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const uint32_t* __restrict__ p = A.vals16 + (size_t)((s * NF * NF + a0 * NF) / 2) * E + F;
          uint32_t w[kW];
#pragma unroll
          for (int j = 0; j < kW; ++j) w[j] = p[(size_t)j * E];
          const int c = A.cols[(size_t)s * E + F];
          V uc[NF], wc[NF];
          get(c, uc, wc);
#pragma unroll
          for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int b = 0; b < NF; ++b) {
              const V m = (V)half_at(w, a * NF + b);
              y1[a] += m * uc[b];
              y2[a] += m * wc[b];
            }
        }
      } else {
        HalfRow<NF, NS> m;
        m.load(A, E, F);
        rowloop([&](int s, int a, int b) { return (V)m.at((s * NF + a) * NF + b); });
      }
      const V sc16 = (V)A.scale16;
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        y1[a] *= sc16;
        y2[a] *= sc16;
      }
      return;
    }
  }
  const V* vals = (sizeof(V) == 8) ? (const V*)A.vals : (const V*)A.vals32;
  rowloop([&](int s, int a, int b) { return vals[(((size_t)s * NF + a0 + a) * NF + b) * E + F]; });
}

// r = g - zg zdef - S x (x already orthogonal to the kernel vector z), p_old = 0; the
// (z, r) partial into zr (the rounding of S x leaves a kernel component in r, which
// k_pcg_init_defl removes).
template <int NF, int NS>
__global__ __launch_bounds__(kBlk) void k_pcg_init(DevGeo g, DevBsr A, const double* __restrict__ gv,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ z, double* __restrict__ p_old,
                                                   const PcgScalars* sc, double* __restrict__ zr) {
  const int E = g.E;
  const int done = sc->done;
  if (done != PCG_RUNNING && !sc->zero_rhs) return;
  const double zg = sc->zg;
  double v[1] = {0};
  for (int F = xcd_block() * blockDim.x + threadIdx.x; F < E; F += gridDim.x * blockDim.x) {
    if (sc->zero_rhs) {
#pragma unroll
      for (int m = 0; m < NF; ++m) {
        const size_t o = (size_t)F * NF + m;
        x[o] = 0; r[o] = 0; z[o] = 0; p_old[o] = 0;
      }
      continue;
    }
    double Sx[NF];
    spmv_row<NF, NS, double, double>(A, E, F, [&](int c, double (&xc)[NF]) {
#pragma unroll
      for (int b = 0; b < NF; ++b) xc[b] = x[(size_t)c * NF + b];
    }, Sx);
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      const size_t o = (size_t)F * NF + m;
      double gm = gv[o];
      if (m == 0) gm -= zg * g.zdef[F];
      r[o] = gm - Sx[m];
      p_old[o] = 0;
    }
    v[0] += g.zdef[F] * r[(size_t)F * NF];
  }
  block_write_partial<1>(v, zr);
}

// r -= (z, r) z, z = M^{-1} r (point or facet-block Jacobi; the multigrid cycle overwrites
// z and the (r,z) partial afterwards); partials (r,z), (r,r) into rz0.
template <int NF, bool BJ>
__global__ __launch_bounds__(kBlk) void k_pcg_init_defl(DevGeo g, DevBsr A, double* __restrict__ r,
                                                        double* __restrict__ z, const PcgScalars* sc,
                                                        const double* __restrict__ zr, double* __restrict__ rz0) {
  const int E = g.E, G = gridDim.x;
  if (sc->done != PCG_RUNNING && !sc->zero_rhs) return;
  double c0[1];
  block_sum_partials<1>(zr, G, c0);
  double v[2] = {0, 0};
  if (!sc->zero_rhs)
    for (int F = xcd_block() * blockDim.x + threadIdx.x; F < E; F += G * blockDim.x) {
      double rr[NF], zz[NF];
#pragma unroll
      for (int m = 0; m < NF; ++m) rr[m] = r[(size_t)F * NF + m];
      rr[0] -= c0[0] * g.zdef[F];
      precond<NF, BJ, double, double>(A, F, rr, zz);
#pragma unroll
      for (int m = 0; m < NF; ++m) {
        const size_t o = (size_t)F * NF + m;
        r[o] = rr[m];
        z[o] = zz[m];
        v[0] += rr[m] * zz[m];
        v[1] += rr[m] * rr[m];
      }
    }
  block_write_partial<2>(v, rz0);
}

// Iteration it >= 1 (it read from the scalars, so that the same launch sequence can be
// replayed from a graph).  From the partials of the previous update (rz_{it-1}, rr_{it-1})
// and of the one before (rz_{it-2}): stopping test, beta; then p_new = z + beta p_old,
// Sp = S p_new and partials (p_new, Sp) and (z, Sp), z the normalised kernel vector of S
// (zdef on mode 0): in exact arithmetic S p is orthogonal to z, in floating point its
// rounding is not, and the update removes that component from the residual.
template <int NF, int NS, typename V, typename M>
__global__ __launch_bounds__(kBlk) void k_pcg_spmv(DevGeo g, DevBsr A, const V* __restrict__ z,
                                                   const V* __restrict__ p_old, V* __restrict__ p_new,
                                                   V* __restrict__ Sp, PcgScalars* sc,
                                                   const double* __restrict__ rz_prev,
                                                   const double* __restrict__ rz_prev2, double* __restrict__ pq) {
  if (sc->done != PCG_RUNNING) return;
  const int it = sc->it;  // advanced only by the update kernel
  const int E = g.E;
  const int G = gridDim.x;
  // beta is not needed before the end: S p_new = S z + beta S p_old.  The partials are
  // loaded first and summed after this thread's first row, whose loads overlap them.
  PartLoad<2> q1, q2;
  partials_load<2>(rz_prev, G, true, q1);
  partials_load<2>(rz_prev2, G, it >= 2, q2);
  const M* vals = (sizeof(M) == 8) ? (const M*)A.vals : (const M*)A.vals32;
  constexpr int SPL = kSplit<NF, NS>, NA = NF / SPL;
  // outputs [a0, a0 + NA) of row F
  auto row = [&](int u, V (&sz)[NA], V (&sp)[NA]) {
    const int F = u / SPL, a0 = (u % SPL) * NA;
#pragma unroll
    for (int a = 0; a < NA; ++a) sz[a] = sp[a] = 0;
#pragma unroll
    for (int s5 = 0; s5 < NS; ++s5) {
      const int c = A.cols[(size_t)s5 * E + F];
      V zc[NF], pc[NF];
#pragma unroll
      for (int bb = 0; bb < NF; ++bb) {
        zc[bb] = z[(size_t)c * NF + bb];
        pc[bb] = p_old[(size_t)c * NF + bb];
      }
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int bb = 0; bb < NF; ++bb) {
          const V m = (V)vals[(((size_t)s5 * NF + a0 + a) * NF + bb) * E + F];
          sz[a] += m * zc[bb];
          sp[a] += m * pc[bb];
        }
    }
  };
  const int u0 = xcd_block() * blockDim.x + threadIdx.x;
  V sz[NA], sp[NA];
  if (u0 < E * SPL) row(u0, sz, sp);
  double t1[2];
  partials_sum<2>(q1, G, t1);
  double beta = 0;
  if (it >= 2) {
    double t2[2];
    partials_sum<2>(q2, G, t2);
    beta = t1[0] / t2[0];
  }
  int status = PCG_RUNNING;
  if (!isfinite(t1[0]) || !isfinite(t1[1]) || !isfinite(beta)) status = PCG_NONFINITE;
  else if (t1[1] <= sc->tol2) status = PCG_CONVERGED;
  else if (it - 1 >= sc->maxit) status = PCG_MAXIT;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->iters = it - 1;
    sc->rr = t1[1];
    sc->rz = t1[0];
    if (it == 1) sc->rr0 = t1[1];
    if (status != PCG_RUNNING) sc->done = status;
  }
  if (status != PCG_RUNNING) return;
  const V b = (V)beta;
  double v[2] = {0, 0};
  for (int u = u0; u < E * SPL; u += G * blockDim.x) {
    if (u != u0) row(u, sz, sp);
    const int F = u / SPL, a0 = (u % SPL) * NA;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const size_t o = (size_t)F * NF + a0 + a;
      const V pn = z[o] + b * p_old[o];
      const V y = sz[a] + b * sp[a];
      p_new[o] = pn;
      Sp[o] = y;
      v[0] += (double)pn * (double)y;
      if (a0 + a == 0) v[1] += g.zdef[F] * (double)y;
    }
  }
  block_write_partial<2>(v, pq);
}

// x += alpha p, r -= alpha (Sp - (z, Sp) z), z = M^{-1} r with alpha = rz_{it-1} / (p, Sp);
// partials (r,z), (r,r) of iteration it.  Removing the kernel component of S p keeps the
// recursive residual in the range of S: left in, the rounding of S p accumulates there, the
// system the PCG sees becomes inconsistent at that level, and once the residual reaches it
// the iteration diverges and (p, S p) changes sign.
// PC: 0 point Jacobi, 1 facet-block Jacobi, 2 none (z comes from the multigrid V-cycle,
// which then overwrites the (r,z) partial).
template <int NF, int PC, typename V, typename M>
__global__ __launch_bounds__(kBlk) void k_pcg_update(DevGeo g, DevBsr A, const V* __restrict__ p,
                                                     const V* __restrict__ Sp, V* __restrict__ x, V* __restrict__ r,
                                                     V* __restrict__ z, PcgScalars* sc,
                                                     const double* __restrict__ rz_prev,
                                                     const double* __restrict__ pq, double* __restrict__ rz_out) {
  if (sc->done != PCG_RUNNING) return;
  const int E = g.E;
  const int G = gridDim.x;
  double t1[2], t2[2];
  block_sum_partials<2>(rz_prev, G, t1);
  block_sum_partials<2>(pq, G, t2);
  int status = PCG_RUNNING;
  if (!isfinite(t2[0])) status = PCG_NONFINITE;
  else if (!(t2[0] > 0)) status = PCG_BREAKDOWN;
  if (status != PCG_RUNNING) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->done = status;
    return;
  }
  const V alpha = (V)(t1[0] / t2[0]);
  const double dz = t2[1];  // (z, S p), z normalised
  double v[2] = {0, 0};
  if constexpr (PC != 1) {
    // point Jacobi or no preconditioner: entrywise over the E n_f entries, two per thread
    // and access (16- or 8-byte loads, coalesced across the wave)
    static_assert(sizeof(M) == sizeof(V), "point Jacobi reads D^{-1} in the vector type");
    using V2 = typename std::conditional<sizeof(V) == 8, double2, float2>::type;
    const V* dv = (sizeof(V) == 8) ? (const V*)A.dinv : (const V*)A.dinv32;
    const long n = (long)E * NF, n2 = n / 2;
    const long t0 = (long)xcd_block() * blockDim.x + threadIdx.x, st = (long)G * blockDim.x;
    auto entry = [&](V& xe, V& re, V pe, V se, V de, V& ze) {
      xe += alpha * pe;
      re = re - alpha * se;
      v[1] += (double)re * (double)re;
      if (PC == 0) {
        ze = de * re;
        v[0] += (double)re * (double)ze;
      }
    };
    // S p less its kernel component, at entry i (mode i % NF of facet i / NF)
    auto sdef = [&](long i, V sp) { return (i % NF == 0) ? (V)((double)sp - dz * g.zdef[i / NF]) : sp; };
    for (long q = t0; q < n2; q += st) {
      const V2 pv = ((const V2*)p)[q], sv = ((const V2*)Sp)[q];
      V2 xv = ((V2*)x)[q], rv = ((V2*)r)[q], zv;
      V2 dd = {};
      if (PC == 0) dd = ((const V2*)dv)[q];
      entry(xv.x, rv.x, pv.x, sdef(2 * q, sv.x), dd.x, zv.x);
      entry(xv.y, rv.y, pv.y, sdef(2 * q + 1, sv.y), dd.y, zv.y);
      ((V2*)x)[q] = xv;
      ((V2*)r)[q] = rv;
      if (PC == 0) ((V2*)z)[q] = zv;
    }
    if ((n & 1) && t0 == (n2 % st)) {  // the odd last entry, by the thread whose turn it is
      const long i = n - 1;
      V xe = x[i], re = r[i], ze = 0;
      entry(xe, re, p[i], sdef(i, Sp[i]), PC == 0 ? dv[i] : (V)0, ze);
      x[i] = xe;
      r[i] = re;
      if (PC == 0) z[i] = ze;
    }
    block_write_partial<2>(v, rz_out);
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->it = sc->it + 1;
    return;
  }
  for (int F = xcd_block() * blockDim.x + threadIdx.x; F < E; F += G * blockDim.x) {
    V rr[NF], zz[NF];
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      const size_t o = (size_t)F * NF + a;
      x[o] += alpha * p[o];
      const V spd = a == 0 ? (V)((double)Sp[o] - dz * g.zdef[F]) : Sp[o];
      rr[a] = r[o] - alpha * spd;
      r[o] = rr[a];
    }
    if (PC == 2) {
#pragma unroll
      for (int a = 0; a < NF; ++a) v[1] += (double)rr[a] * (double)rr[a];
    } else {
      precond<NF, PC == 1, V, M>(A, F, rr, zz);
#pragma unroll
      for (int a = 0; a < NF; ++a) {
        z[(size_t)F * NF + a] = zz[a];
        v[0] += (double)rr[a] * (double)zz[a];
        v[1] += (double)rr[a] * (double)rr[a];
      }
    }
  }
  block_write_partial<2>(v, rz_out);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->it = sc->it + 1;  // no other block reads it here
}

// Inner FP32 PCG start for S d = r64 (d = 0): r = (float) r64; partials (r,z), (r,r).
template <int NF, bool BJ>
__global__ __launch_bounds__(kBlk) void k_pcg32_init(DevGeo g, DevBsr A, const double* __restrict__ r64,
                                                     float* __restrict__ x, float* __restrict__ r,
                                                     float* __restrict__ z, float* __restrict__ p_old,
                                                     double* __restrict__ rz0) {
  const int E = g.E;
  double v[2] = {0, 0};
  for (int F = xcd_block() * blockDim.x + threadIdx.x; F < E; F += gridDim.x * blockDim.x) {
    float rr[NF], zz[NF];
#pragma unroll
    for (int m = 0; m < NF; ++m) rr[m] = (float)r64[(size_t)F * NF + m];
    precond<NF, BJ, float, float>(A, F, rr, zz);
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      const size_t o = (size_t)F * NF + m;
      x[o] = 0; r[o] = rr[m]; z[o] = zz[m]; p_old[o] = 0;
      v[0] += (double)rr[m] * zz[m];
      v[1] += (double)rr[m] * rr[m];
    }
  }
  block_write_partial<2>(v, rz0);
}

// FP64 refinement residual r64 = g - zg zdef - S lam; partials (r64, r64).
template <int NF>
__global__ __launch_bounds__(kBlk) void k_ir_residual(DevGeo g, DevBsr A, const double* __restrict__ gv,
                                                      const double* __restrict__ lam, double* __restrict__ r64,
                                                      const PcgScalars* sc, double* __restrict__ part) {
  const int E = g.E;
  const double zg = sc->zg;
  double v[1] = {0};
  for (int F = xcd_block() * blockDim.x + threadIdx.x; F < E; F += gridDim.x * blockDim.x) {
    double Sx[NF];
    spmv_row<NF, kSlots, double, double>(A, E, F, [&](int c, double (&xc)[NF]) {
#pragma unroll
      for (int b = 0; b < NF; ++b) xc[b] = lam[(size_t)c * NF + b];
    }, Sx);
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      double gm = gv[(size_t)F * NF + m];
      if (m == 0) gm -= zg * g.zdef[F];
      const double rm = gm - Sx[m];
      r64[(size_t)F * NF + m] = rm;
      v[0] += rm * rm;
    }
  }
  block_write_partial<1>(v, part);
}

// One block: (r64, r64) into the outer scalars; set up the inner FP32 solve's stopping test
// (sc64->tol2 holds the outer threshold, ir_rtol^2 (g, g)).
__global__ __launch_bounds__(kBlk) void k_finalize_ir(const double* __restrict__ part, int n, PcgScalars* sc64,
                                                      PcgScalars* sc32, double inner_rtol, int maxit) {
  double t[1];
  block_sum_partials<1>(part, n, t);
  if (threadIdx.x == 0) {
    sc64->rr = t[0];
    sc32->gg = t[0];
    // relative to the refinement residual, but never below half the outer target
    sc32->tol2 = fmax(inner_rtol * inner_rtol * t[0], 0.25 * sc64->tol2);
    sc32->maxit = maxit;
    sc32->iters = 0;
    sc32->it = 1;
    sc32->zero_rhs = 0;
    sc32->done = isfinite(t[0]) ? PCG_RUNNING : PCG_NONFINITE;
  }
}

// ---------------------------------------------------------------------------------------
// a5: multigrid V-cycle preconditioner for the facet PCG (smoothed aggregation)
// ---------------------------------------------------------------------------------------
// Finest level: Chebyshev(2) smoothing with the point-Jacobi scaling D^{-1}, residual,
// restriction R = P^T, coarse correction, prolongation, Chebyshev(2) post-smoothing (the
// coarser levels use degree 1, see k_mgc_restrict).
// With th, de the centre and half-width of the smoothing interval, c1 = rho1 rho0 and
// c2 = 2 rho1 / de (rho0 = de/th, rho1 = 1/(2 th/de - rho0)):
//   pre  (x0 = 0):  x1 = D^{-1} b / th,  x2 = (1 + c1) x1 + c2 D^{-1} (b - A x1)
//   post (from x3): d = D^{-1}(b - A x3) / th, x4 = x3 + d,
//                   z  = x4 + c1 d + c2 D^{-1} (b - A x4)
// The finest level uses the BSR facet matrix (grid-stride over facet rows, like the PCG
// kernels, so that the last post-smoothing kernel can emit the (r, z) partials).

template <int NF, typename V>
__device__ inline const V* bsr_vals(const DevBsr& A) { return (sizeof(V) == 8) ? (const V*)A.vals : (const V*)A.vals32; }
template <int NF, typename V>
__device__ inline const V* bsr_dinv(const DevBsr& A) { return (sizeof(V) == 8) ? (const V*)A.dinv : (const V*)A.dinv32; }

// V: arithmetic and storage type of the cycle; VB: type of the PCG vectors b (in) and z
// (out), so that an FP32 cycle can precondition an FP64 PCG.  Every kernel of the cycle
// returns at once when the PCG has already stopped (iterations replayed past the end).
template <int NF, int NS, typename V, typename VB>
__global__ __launch_bounds__(kBlk) void k_mg0_pre(DevGeo g, DevBsr A, const VB* __restrict__ b, V* __restrict__ x2,
                                                  CheB cb, const PcgScalars* sc) {
  const bool live = sc->done == PCG_RUNNING;  // tested before the stores only
  const V* dinv = bsr_dinv<NF, V>(A);
  const V ith = (V)(1.0 / cb.th), c1 = (V)cb.c1, c2 = (V)cb.c2;
  const int E = g.E;
  constexpr int SPL = kSplit<NF, NS>, NA = NF / SPL;
  for (int u = xcd_block() * blockDim.x + threadIdx.x; u < E * SPL; u += gridDim.x * blockDim.x) {
    const int F = u / SPL, a0 = (u % SPL) * NA;
    V y[NA];
    spmv_part_mg<NF, NS, NA, V>(A, E, F, a0, [&](int c, V (&xc)[NF]) {
#pragma unroll
      for (int q = 0; q < NF; ++q) xc[q] = dinv[(size_t)c * NF + q] * (V)b[(size_t)c * NF + q] * ith;
    }, y);
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const size_t o = (size_t)F * NF + a0 + a;
      const V bo = (V)b[o];
      const V x1 = dinv[o] * bo * ith;
      if (live) x2[o] = (1 + c1) * x1 + c2 * dinv[o] * (bo - y[a]);
    }
  }
}

template <int NF, int NS, typename V, typename VB>
__global__ __launch_bounds__(kBlk) void k_mg0_resid(DevGeo g, DevBsr A, const VB* __restrict__ b,
                                                    const V* __restrict__ x, V* __restrict__ r, const PcgScalars* sc) {
  const bool live = sc->done == PCG_RUNNING;  // tested before the stores only
  const int E = g.E;
  constexpr int SPL = kSplit<NF, NS>, NA = NF / SPL;
  for (int u = xcd_block() * blockDim.x + threadIdx.x; u < E * SPL; u += gridDim.x * blockDim.x) {
    const int F = u / SPL, a0 = (u % SPL) * NA;
    V y[NA];
    spmv_part_mg<NF, NS, NA, V>(A, E, F, a0, [&](int c, V (&xc)[NF]) {
#pragma unroll
      for (int q = 0; q < NF; ++q) xc[q] = x[(size_t)c * NF + q];
    }, y);
#pragma unroll
    for (int a = 0; a < NA; ++a)
      if (live) r[(size_t)F * NF + a0 + a] = (V)b[(size_t)F * NF + a0 + a] - y[a];
  }
}

template <int NF, int NS, typename V, typename VB>
__global__ __launch_bounds__(kBlk) void k_mg0_post1(DevGeo g, DevBsr A, const VB* __restrict__ b,
                                                    const V* __restrict__ x3, V* __restrict__ x4, V* __restrict__ d,
                                                    CheB cb, const PcgScalars* sc) {
  const bool live = sc->done == PCG_RUNNING;  // tested before the stores only
  const V* dinv = bsr_dinv<NF, V>(A);
  const V ith = (V)(1.0 / cb.th);
  const int E = g.E;
  constexpr int SPL = kSplit<NF, NS>, NA = NF / SPL;
  for (int u = xcd_block() * blockDim.x + threadIdx.x; u < E * SPL; u += gridDim.x * blockDim.x) {
    const int F = u / SPL, a0 = (u % SPL) * NA;
    V y[NA];
    spmv_part_mg<NF, NS, NA, V>(A, E, F, a0, [&](int c, V (&xc)[NF]) {
#pragma unroll
      for (int q = 0; q < NF; ++q) xc[q] = x3[(size_t)c * NF + q];
    }, y);
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const size_t o = (size_t)F * NF + a0 + a;
      const V dd = dinv[o] * ((V)b[o] - y[a]) * ith;
      if (live) {
        d[o] = dd;
        x4[o] = x3[o] + dd;
      }
    }
  }
}

// Last post-smoothing step; z is the preconditioned PCG residual b.  Writes the (b, z)
// partial of this block into rz[2*block] (the (r,r) slot rz[2*block+1] is left alone),
// and block 0 applies the iteration's stopping test to the (r,r) partials.
template <int NF, int NS, typename V, typename VB>
__global__ __launch_bounds__(kBlk) void k_mg0_post2(DevGeo g, DevBsr A, const VB* __restrict__ b,
                                                    const V* __restrict__ x4, const V* __restrict__ d,
                                                    VB* __restrict__ z, CheB cb, double* __restrict__ rz,
                                                    PcgScalars* sc) {
  const bool live = sc->done == PCG_RUNNING;  // tested before the stores only
  // The stopping test of this iteration on the (r, r) partials of its update (the odd
  // slots of rz), so that a converged run needs no further launch to find out; block 0
  // alone sums them.
  const bool b0 = blockIdx.x == 0;
  PartLoad<2> qr;
  partials_load<2>(rz, gridDim.x, b0, qr);
  const V* dinv = bsr_dinv<NF, V>(A);
  const V c1 = (V)cb.c1, c2 = (V)cb.c2;
  const int E = g.E;
  constexpr int SPL = kSplit<NF, NS>, NA = NF / SPL;
  double v[1] = {0};
  for (int u = xcd_block() * blockDim.x + threadIdx.x; u < E * SPL; u += gridDim.x * blockDim.x) {
    const int F = u / SPL, a0 = (u % SPL) * NA;
    V y[NA];
    spmv_part_mg<NF, NS, NA, V>(A, E, F, a0, [&](int c, V (&xc)[NF]) {
#pragma unroll
      for (int q = 0; q < NF; ++q) xc[q] = x4[(size_t)c * NF + q];
    }, y);
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const size_t o = (size_t)F * NF + a0 + a;
      const V zz = x4[o] + c1 * d[o] + c2 * dinv[o] * ((V)b[o] - y[a]);
      if (live) z[o] = (VB)zz;
      v[0] += (double)b[o] * (double)(VB)zz;
    }
  }
  double rr[2] = {0, 0};
  if (b0) partials_sum<2>(qr, gridDim.x, rr);  // rr[1] = (r, r); the branch is uniform over the block
  __shared__ double sh[kBlk / 64];
  const double s = wave_sum(v[0]);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (live && threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    rz[2 * blockIdx.x] = t;
    if (b0) {
      const int it = sc->it;  // already advanced by this iteration's update
      sc->iters = it - 1;
      sc->rr = rr[1];
      if (it == 1) sc->rr0 = rr[1];
      if (isfinite(rr[1]) && rr[1] <= sc->tol2) sc->done = PCG_CONVERGED;
    }
  }
}

// Coarse levels: padded rows (DevCsr), LPR lanes (a power of two <= 64, chosen on the
// host from the mean row length) share a row: lane j of the group takes entries j, j+LPR,
// ..., and the group reduces with shuffles in a fixed order.
template <typename V>
__device__ inline const V* csr_vals(const DevCsr& A) { return (sizeof(V) == 8) ? (const V*)A.val : (const V*)A.val32; }

// Sum over the n entries base, base + LPR, ... of a padded row, in batches of U whose loads
// are all issued before the first product (the short rows of the coarse levels are bound
// by dependent memory round trips, not bandwidth).  The last batch repeats its final entry
// and multiplies the repeats by zero; the valid products are added in entry order.
template <int LPR, int U, typename V, typename LD, typename X>
__device__ inline V ell_batched(size_t base, int n, LD ld, X x) {
  V s = 0;
  for (int j0 = 0; j0 < n; j0 += U) {
    int c[U];
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) ld(base + (size_t)min(j0 + u, n - 1) * LPR, c[u], v[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const V xv = x(c[u]);
      s += v[u] * ((j0 + u < n) ? xv : (V)0);
    }
  }
  return s;
}

// Entries sub, sub + LPR, ... below w: how many (w is a multiple of the matrix's own lpr,
// which can differ from the LPR of a kernel that walks several matrices).
template <int LPR>
__device__ inline int lane_entries(int w, int sub) { return w > sub ? (w - sub + LPR - 1) / LPR : 0; }

// ell_batched with a batch as long as the longest lane's share of a row of width w (up to
// 4; 8 beyond), so that short rows issue no repeated loads.  The choice depends on w only,
// the same for every lane of the launch.
template <int LPR, typename V, typename LD, typename X>
__device__ inline V ell_sum(int w, int sub, size_t base, LD ld, X x) {
  const int n = lane_entries<LPR>(w, sub), nmax = (w + LPR - 1) / LPR;
  if (nmax <= 1) return ell_batched<LPR, 1, V>(base, n, ld, x);
  if (nmax == 2) return ell_batched<LPR, 2, V>(base, n, ld, x);
  if (nmax == 3) return ell_batched<LPR, 3, V>(base, n, ld, x);
  if (nmax == 4) return ell_batched<LPR, 4, V>(base, n, ld, x);
  return ell_batched<LPR, 8, V>(base, n, ld, x);
}

// This lane's part of row i of M x (i < M.n).
template <int LPR, typename V, typename X>
__device__ inline V ell_part(const DevCsr& M, int i, int sub, X x) {
  const V* __restrict__ vals = csr_vals<V>(M);
  const int* __restrict__ col = M.col;
  return ell_sum<LPR, V>(M.w, sub, (size_t)i * M.w + sub, [&](size_t k, int& c, V& v) {
    c = col[k];
    v = vals[k];
  }, x);
}
template <int LPR, typename V>
__device__ inline V group_sum(V s) {
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, LPR);
  return s;
}
template <int LPR, typename V, typename X>
__device__ inline V csr_row_group(const DevCsr& A, const V* __restrict__ vals, int i, int sub, X x) {
  (void)vals;
  return group_sum<LPR, V>(i < A.n ? ell_part<LPR, V>(A, i, sub, x) : (V)0);
}

// Coarse levels (below the finest) smooth with one Chebyshev(1) step, i.e. damped Jacobi
// with weight 1/th, before and after the coarse correction: x1 = D^{-1} b / th, and after
// the correction x3 = x1 + P e, z = x3 + D^{-1} (b - A x3) / th.  Two kernels per level:
//   restriction of the smoothed residual, b_c = R (b - A x1) = R b - (R A) x1, with R A
//   precomputed and x1 formed on the fly (neither x1 nor the residual is stored);
//   prolongation fused with the post-smoothing step, A x3 = A x1 + (A P) e.
template <int LPR, typename V>
__global__ __launch_bounds__(kBlk) void k_mgc_restrict(DevCsr R, DevCsr RA, const V* __restrict__ b,
                                                       const V* __restrict__ dinv, CheB cb, V* __restrict__ bc,
                                                       const PcgScalars* sc) {
  const bool live = sc->done == PCG_RUNNING;  // tested before the store only
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = g / LPR, sub = g % LPR;
  const V ith = (V)(1.0 / cb.th);
  V s = 0;
  if (i < R.n)
    s = ell_part<LPR, V>(R, i, sub, [&](int c) { return b[c]; }) -
        ell_part<LPR, V>(RA, i, sub, [&](int c) { return dinv[c] * b[c] * ith; });
  s = group_sum<LPR, V>(s);
  if (live && i < R.n && sub == 0) bc[i] = s;
}

template <int LPR, typename V>
__global__ __launch_bounds__(kBlk) void k_mgc_post(DevCsr A, DevCsr AP, DevCsr P, const V* __restrict__ dinv,
                                                   const V* __restrict__ b, const V* __restrict__ e,
                                                   V* __restrict__ z, CheB cb, const PcgScalars* sc) {
  const bool live = sc->done == PCG_RUNNING;  // tested before the store only
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = g / LPR, sub = g % LPR;
  const V ith = (V)(1.0 / cb.th);
  V pe = 0, ax = 0;
  if (i < A.n) {
    pe = ell_part<LPR, V>(P, i, sub, [&](int c) { return e[c]; });
    ax = ell_part<LPR, V>(A, i, sub, [&](int c) { return dinv[c] * b[c] * ith; }) +
         ell_part<LPR, V>(AP, i, sub, [&](int c) { return e[c]; });
  }
  pe = group_sum<LPR, V>(pe);
  ax = group_sum<LPR, V>(ax);
  if (live && i < A.n && sub == 0) {
    const V x1 = dinv[i] * b[i] * ith;
    z[i] = (x1 + pe) + dinv[i] * (b[i] - ax) * ith;
  }
}

// y = M x (restriction with M = R), or y = y0 + M x (prolongation-add, add != 0).
template <int LPR, typename V>
__global__ __launch_bounds__(kBlk) void k_csr_apply(DevCsr M, const V* __restrict__ x, const V* __restrict__ y0,
                                                    V* __restrict__ y, int add, const PcgScalars* sc) {
  const bool live = sc->done == PCG_RUNNING;  // tested before the stores only
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = g / LPR, sub = g % LPR;
  V s = 0;
  if (sizeof(V) == 4 && LPR == 1 && M.pk) {  // packed rows: one 16-byte load per 4 entries
    if (i < M.n) {
      const int ng = M.w >> 2;  // 1 to 4 groups of 4 entries
      for (int gi = 0; gi < ng; ++gi) {
        const uint4 w = *reinterpret_cast<const uint4*>(M.pk + ((size_t)i * ng + gi) * 4);
        const _Float16 h0 = __builtin_bit_cast(_Float16, (uint16_t)(w.z & 0xffffu));
        const _Float16 h1 = __builtin_bit_cast(_Float16, (uint16_t)(w.z >> 16));
        const _Float16 h2 = __builtin_bit_cast(_Float16, (uint16_t)(w.w & 0xffffu));
        const _Float16 h3 = __builtin_bit_cast(_Float16, (uint16_t)(w.w >> 16));
        s += (V)h0 * x[w.x & 0xffffu] + (V)h1 * x[w.x >> 16] + (V)h2 * x[w.y & 0xffffu] + (V)h3 * x[w.y >> 16];
      }
      s *= (V)M.pscale;
    }
  } else if (LPR == 1 && M.w == 4) {  // rows of 4 entries, 16-byte aligned: vector loads
    if (i < M.n) {
      const int4 c = *reinterpret_cast<const int4*>(M.col + (size_t)i * 4);
      const V* v = csr_vals<V>(M) + (size_t)i * 4;
      s = v[0] * x[c.x] + v[1] * x[c.y] + v[2] * x[c.z] + v[3] * x[c.w];
    }
  } else if (sizeof(V) == 4 && M.val16) {
    const _Float16* __restrict__ v16 = reinterpret_cast<const _Float16*>(M.val16);
    const int* __restrict__ col = M.col;
    if (i < M.n)
      s = ell_sum<LPR, V>(M.w, sub, (size_t)i * M.w + sub, [&](size_t k, int& c, V& v) {
        c = col[k];
        v = (V)v16[k];
      }, [&](int c) { return x[c]; });
    s = group_sum<LPR, V>(s) * (V)M.pscale;
  } else {
    s = csr_row_group<LPR, V>(M, csr_vals<V>(M), i, sub, [&](int c) { return x[c]; });
  }
  if (live && i < M.n && sub == 0) y[i] = add ? y0[i] + s : s;
}

// ---- PCG update fused with the first smoothing step of the cycle ----------------------
// PCG update fused with the first pre-smoothing step of the cycle.  The residual is
// double-buffered: r_new = r_old - alpha (Sp - (z, Sp) z) for the own rows (the kernel
// component of S p removed, as in k_pcg_update), and the neighbours' new residual, needed
// by S x1, is formed on the fly from r_old, Sp and the precomputed S D^{-1} z.  Also
// x += alpha p, the (r,r) partial, and the iteration counter.
template <int NF, int NS, typename V, typename VB>
__global__ __launch_bounds__(kBlk) void k_pcg_upd_mg0_pre(DevGeo g, DevBsr A, const VB* __restrict__ p,
                                                          const VB* __restrict__ Sp, VB* __restrict__ x,
                                                          const VB* __restrict__ r_old, VB* __restrict__ r_new,
                                                          V* __restrict__ x2, CheB cb, PcgScalars* sc,
                                                          const double* __restrict__ rz_prev,
                                                          const double* __restrict__ pq, double* __restrict__ rz_out) {
  if (sc->done != PCG_RUNNING) return;
  const int E = g.E;
  const int G = gridDim.x;
  // alpha is not needed before the end: with u = D^{-1} r_old / th and w = D^{-1} S p / th,
  // S x1 = S u - alpha S w.  The partials are loaded first and summed after this thread's
  // first row, whose loads overlap them.
  PartLoad<2> q1, q2;
  partials_load<2>(rz_prev, G, true, q1);
  partials_load<2>(pq, G, true, q2);
  const V* dinv = bsr_dinv<NF, V>(A);
  const V ith = (V)(1.0 / cb.th), c1 = (V)cb.c1, c2 = (V)cb.c2;
  constexpr int SPL = kSplit<NF, NS>, NA = NF / SPL;
  auto row = [&](int u, V (&su)[NA], V (&sw)[NA]) {
    spmv_part_mg2<NF, NS, NA, V>(A, E, u / SPL, (u % SPL) * NA, [&](int c, V (&uc)[NF], V (&wc)[NF]) {
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        const size_t o = (size_t)c * NF + q;
        const V d = dinv[o] * ith;
        uc[q] = d * (V)r_old[o];
        wc[q] = d * (V)Sp[o];
      }
    }, su, sw);
  };
  const int u0 = xcd_block() * blockDim.x + threadIdx.x;
  V su[NA], sw[NA];
  if (u0 < E * SPL) row(u0, su, sw);
  double t1[2], t2[2];
  partials_sum<2>(q1, G, t1);
  partials_sum<2>(q2, G, t2);
  int status = PCG_RUNNING;
  if (!isfinite(t2[0])) status = PCG_NONFINITE;
  else if (!(t2[0] > 0)) status = PCG_BREAKDOWN;
  if (status != PCG_RUNNING) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->done = status;
    return;
  }
  const VB alpha = (VB)(t1[0] / t2[0]);
  const V alv = (V)alpha;
  // the kernel component of S p leaves the residual: r_new = r_old - alpha (Sp - dz z), and
  // S x1 gains alpha dz (S D^{-1} z) / th
  const double dz = t2[1];
  const V* __restrict__ tdef = (sizeof(V) == 8) ? (const V*)A.tdef : (const V*)A.tdef32;
  const V azt = (V)((double)alpha * dz) * ith;
  double v[2] = {0, 0};
  for (int u = u0; u < E * SPL; u += G * blockDim.x) {
    if (u != u0) row(u, su, sw);
    const int F = u / SPL, a0 = (u % SPL) * NA;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const size_t o = (size_t)F * NF + a0 + a;
      x[o] += alpha * p[o];
      const VB spd = (a0 + a == 0) ? (VB)((double)Sp[o] - dz * g.zdef[F]) : Sp[o];
      const VB rn = r_old[o] - alpha * spd;
      r_new[o] = rn;
      v[1] += (double)rn * (double)rn;
      const V bo = (V)rn;
      const V x1 = dinv[o] * bo * ith;
      x2[o] = (1 + c1) * x1 + c2 * dinv[o] * (bo - (su[a] - alv * sw[a] + azt * tdef[o]));
    }
  }
  block_write_partial<2>(v, rz_out);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->it = sc->it + 1;
}

// (b, z) partials into rz[2*block] (grid-stride over n).
template <typename V>
__global__ __launch_bounds__(kBlk) void k_partial_dot(long n, const V* __restrict__ b, const V* __restrict__ z,
                                                      double* __restrict__ rz, const PcgScalars* sc) {
  if (sc->done != PCG_RUNNING) return;
  double v = 0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    v += (double)b[i] * (double)z[i];
  __shared__ double sh[kBlk / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    rz[2 * blockIdx.x] = t;
  }
}

// Coarsest level: x = Ainv b with the dense (regularised) inverse; a wavefront per row.
template <typename V>
__global__ __launch_bounds__(kBlk) void k_dense_mv(int n, const double* __restrict__ Ainv, const float* __restrict__ Ainv32,
                                                   const V* __restrict__ b, V* __restrict__ x, const PcgScalars* sc) {
  const bool live = sc->done == PCG_RUNNING;  // tested before the store only
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = g >> 6, lane = g & 63;
  const V* M = (sizeof(V) == 8) ? (const V*)Ainv : (const V*)Ainv32;
  V s = 0;
  if (i < n)  // entries lane, lane + 64, ...; the column index is the entry's own
    s = ell_batched<64, 8, V>((size_t)lane, lane_entries<64>(n, lane), [&](size_t k, int& c, V& v) {
      c = (int)k;
      v = M[(size_t)i * n + k];
    }, [&](int c) { return b[c]; });
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (live && i < n && lane == 0) x[i] = s;
}

__global__ void k_add_f32(long n, const float* __restrict__ x, double* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += (double)x[i];
}

// ---------------------------------------------------------------------------------------
// a2: load vector of data given at the projection points; evaluation; diagnostics
// ---------------------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(kEBlk) void k_load_vector(DevGeo g, DevTabs tb, int nqp, const double* __restrict__ fq,
                                                       double* __restrict__ F) {
  constexpr int P = nP(K);
  const int T = g.T;
  const int t = xcd_block() * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double sq = sqrt(g.detJ[t]);
  double acc[2][P];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < P; ++i) acc[c][i] = 0;
  for (int q = 0; q < nqp; ++q) {
    const double w = tb.Wp[q] * sq;
    const double f0 = fq[(size_t)q * T + t] * w, f1 = fq[(size_t)(nqp + q) * T + t] * w;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const double v = tb.Vp[q * P + i];
      acc[0][i] += f0 * v;
      acc[1][i] += f1 * v;
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < P; ++i) F[(size_t)(c * P + i) * T + t] = acc[c][i];
}

template <int K>
__global__ __launch_bounds__(kEBlk) void k_eval(DevGeo g, int npts, const double* __restrict__ tab,
                                                const double* __restrict__ U, double* __restrict__ out) {
  constexpr int P = nP(K);
  const int T = g.T;
  const int t = xcd_block() * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double isq = g.isq[t];
  double u[2][P];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < P; ++i) u[c][i] = U[(size_t)(c * P + i) * T + t];
  for (int p = 0; p < npts; ++p)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double s = 0;
#pragma unroll
      for (int i = 0; i < P; ++i) s += u[c][i] * tab[p * P + i];
      out[(size_t)(c * npts + p) * T + t] = s * isq;
    }
}

// Per block: sum 0.5 U^2, sum curl^2 (volume rule), max |div u| (volume points),
// max |[[u.n]]| (facet points, facets this element owns as L side).
template <int K>
__global__ __launch_bounds__(kEBlk) void k_diag(DevGeo g, DevTabs tb, const double* __restrict__ U,
                                                double* __restrict__ partials) {
  constexpr int P = nP(K), NQV = nQV(K), NQF = nQF(K);
  const int T = g.T;
  const int t = xcd_block() * blockDim.x + threadIdx.x;
  double en = 0, ens = 0, dmax = 0, jmax = 0;
  if (t < T) {
    double u[2][P];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < P; ++i) {
        u[c][i] = U[(size_t)(c * P + i) * T + t];
        en += 0.5 * u[c][i] * u[c][i];
      }
    double Ji[2][2];
    load_Jinv(g, t, Ji);
    const double det = g.detJ[t], isq = g.isq[t];
    for (int q = 0; q < NQV; ++q) {
      double gr[2][2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double b0 = 0, b1 = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
          b0 += u[c][i] * tb.Gv[(q * 2 + 0) * P + i];
          b1 += u[c][i] * tb.Gv[(q * 2 + 1) * P + i];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) gr[c][j] = isq * (b0 * Ji[0][j] + b1 * Ji[1][j]);
      }
      const double curl = gr[1][0] - gr[0][1];
      ens += tb.Wv[q] * det * curl * curl;
      dmax = fmax(dmax, fabs(gr[0][0] + gr[1][1]));
    }
    for (int f = 0; f < 3; ++f) {
      const size_t idx = (size_t)f * T + t;
      const int code = g.code[idx];
      if ((code >> 3) & 1) continue;  // the L side measures the facet
      if ((code >> 4) & 1) continue;  // outflow boundary: u.n is free there
      const int nb = g.nbr[idx], fn = code & 3;
      const bool rev = (code >> 2) & 1;
      const bool wall = nb < 0;  // the jump across a wall is u.n itself
      const int nbs = wall ? t : nb;
      const double n0 = g.nx[idx], n1 = g.ny[idx], isqn = g.isq[nbs];
      for (int r = 0; r < NQF; ++r) {
        const int rn = rev ? NQF - 1 - r : r;
        double jo = 0, jn = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
          const double vo = tb.Vf[(f * NQF + r) * P + i], vn = tb.Vf[(fn * NQF + rn) * P + i];
          jo += (u[0][i] * n0 + u[1][i] * n1) * vo;
          if (!wall) jn += (U[(size_t)i * T + nbs] * n0 + U[(size_t)(P + i) * T + nbs] * n1) * vn;
        }
        jmax = fmax(jmax, fabs(jo * isq - jn * isqn));
      }
    }
  }
  __shared__ double sh[4][kEBlk / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  en = wave_sum(en);
  ens = wave_sum(ens);
  dmax = wave_max(dmax);
  jmax = wave_max(jmax);
  if (lane == 0) { sh[0][wid] = en; sh[1][wid] = ens; sh[2][wid] = dmax; sh[3][wid] = jmax; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, c = 0, d = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      a += sh[0][w]; b += sh[1][w]; c = fmax(c, sh[2][w]); d = fmax(d, sh[3][w]);
    }
    partials[4 * blockIdx.x + 0] = a;
    partials[4 * blockIdx.x + 1] = b;
    partials[4 * blockIdx.x + 2] = c;
    partials[4 * blockIdx.x + 3] = d;
  }
}

__global__ __launch_bounds__(kBlk) void k_diag_finish(int nblk, const double* __restrict__ partials,
                                                      double* __restrict__ res) {
  double a = 0, b = 0, c = 0, d = 0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    a += partials[4 * i]; b += partials[4 * i + 1];
    c = fmax(c, partials[4 * i + 2]); d = fmax(d, partials[4 * i + 3]);
  }
  __shared__ double sh[4][kBlk / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  a = wave_sum(a); b = wave_sum(b); c = wave_max(c); d = wave_max(d);
  if (lane == 0) { sh[0][wid] = a; sh[1][wid] = b; sh[2][wid] = c; sh[3][wid] = d; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      sh[0][0] += sh[0][w]; sh[1][0] += sh[1][w];
      sh[2][0] = fmax(sh[2][0], sh[2][w]); sh[3][0] = fmax(sh[3][0], sh[3][w]);
    }
    res[0] = sh[0][0]; res[1] = sh[1][0]; res[2] = sh[2][0]; res[3] = sh[3][0];
  }
}

__global__ void k_axpby(long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];  // b = 0: y may be uninitialised
}
__global__ void k_fill(long n, double v, double* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}
// Polynomial extrapolation in time from h0 (newest), h1, h2 (oldest), equal spacing.
// Lagrange extrapolation to the next equally spaced time from the last order+1 values
// (h.p[0] newest): coefficients (-1)^j C(order+1, j+1).
// Extrapolation of order o in time from q[0..o] (newest first), equal time steps:
// sum_j (-1)^j C(o+1, j+1) q[j].
template <typename Q>
__device__ inline double extrapolate_at(int order, Q q) {
  double v = 0, c = order + 1;  // C(order+1, 1)
  for (int j = 0; j <= order; ++j) {
    v += ((j & 1) ? -c : c) * q(j);
    c = c * (order - j) / (j + 2);  // C(order+1, j+2)
  }
  return v;
}

// ---- start values by projection onto earlier solutions (energy norm of S) ---------------
// The stage solves of a time integration share S; their solutions lie close to the span of
// the last few.  With a basis X_i of that span, S-orthogonal (X_i . S X_j = 0 for i != j,
// n_i = X_i . S X_i), the element of the span closest to the solution of S x = g in the
// S-norm is sum_i (X_i . g / n_i) X_i: it needs g, not the solution.  The basis is kept as
// X = B T with stored vectors B_j, their images S B_j and a unit upper triangular T (the
// second Gram-Schmidt pass of each new vector is a column of T, not a pass over the
// vectors); a vector whose n_i failed the test of k_pj_small has n_i = +inf and drops out.

// Thread i < M of the block gets the block total of acc[i] (others 0).  The kernels below
// are instantiated for each basis size NB (0..kProjMax), so that the loads of all basis
// vectors at an entry are issued together.
template <int M>
__device__ inline double pj_block_rows(const double (&acc)[M]) {
  __shared__ double sh[kBlk / 64][kProjPart];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const double v = wave_sum(acc[i]);
    if (lane == 0) sh[wv][i] = v;
  }
  __syncthreads();
  double t = 0;
  if ((int)threadIdx.x < M)
#pragma unroll
    for (int w = 0; w < kBlk / 64; ++w) t += sh[w][threadIdx.x];
  return t;
}

// part[block][i] = this block's share of Y_i . w, i < NB.
template <int NB>
__global__ __launch_bounds__(kBlk) void k_pj_dots(long n, PjVecs Y, const double* __restrict__ w,
                                                  double* __restrict__ part) {
  double acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = 0;
  for (long e = (long)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const double we = w[e];
#pragma unroll
    for (int i = 0; i < NB; ++i) acc[i] += Y.p[i][e] * we;
  }
  const double t = pj_block_rows<NB>(acc);
  if ((int)threadIdx.x < NB) part[(size_t)blockIdx.x * kProjPart + threadIdx.x] = t;
}

// x = x0 = sum_i w[i] B_i, i < NB.
template <int NB>
__global__ __launch_bounds__(kBlk) void k_pj_combine(long n, PjVecs B, const double* __restrict__ w,
                                                     double* __restrict__ x, double* __restrict__ x0) {
  __shared__ double c[kProjMax];
  if ((int)threadIdx.x < NB) c[threadIdx.x] = w[threadIdx.x];
  __syncthreads();
  for (long e = (long)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    double bv[NB], v = 0;
#pragma unroll
    for (int i = 0; i < NB; ++i) bv[i] = B.p[i][e];
#pragma unroll
    for (int i = 0; i < NB; ++i) v += c[i] * bv[i];
    x[e] = v;
    x0[e] = v;
  }
}

// New stored vector v = a - a0 (a0 given) or a - sum_i w[i] B_i, Sv = Sa - sum_i w[i] S B_i
// (i < NB); ca, cSa (optional) receive copies of a and Sa.  Partials: S B_i . v (i < NB)
// and v . Sv (slot NB).
template <int NB>
__global__ __launch_bounds__(kBlk) void k_pj_update(long n, PjVecs B, PjVecs SB, const double* __restrict__ w,
                                                    const double* __restrict__ a, const double* __restrict__ a0,
                                                    const double* __restrict__ Sa, double* __restrict__ v,
                                                    double* __restrict__ Sv, double* __restrict__ ca,
                                                    double* __restrict__ cSa, double* __restrict__ part) {
  __shared__ double c[kProjMax];
  if ((int)threadIdx.x < NB) c[threadIdx.x] = w[threadIdx.x];
  __syncthreads();
  double acc[NB + 1];
#pragma unroll
  for (int i = 0; i <= NB; ++i) acc[i] = 0;
  for (long e = (long)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    double sb[NB + 1], bv[NB + 1];
#pragma unroll
    for (int i = 0; i < NB; ++i) sb[i] = SB.p[i][e];
    const double ae = a[e], sae = Sa[e];
    double ve = ae, sve = sae;
    if (a0) {
      ve -= a0[e];
    } else {
#pragma unroll
      for (int i = 0; i < NB; ++i) bv[i] = B.p[i][e];
#pragma unroll
      for (int i = 0; i < NB; ++i) ve -= c[i] * bv[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) sve -= c[i] * sb[i];
    v[e] = ve;
    Sv[e] = sve;
    if (ca) {
      ca[e] = ae;
      cSa[e] = sae;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) acc[i] += sb[i] * ve;
    acc[NB] += ve * sve;
  }
  const double t = pj_block_rows<NB + 1>(acc);
  if ((int)threadIdx.x <= NB) part[(size_t)blockIdx.x * kProjPart + threadIdx.x] = t;
}

// One block, the small dense part (T column-major, T[j + kProjMax i] = T_ji, norms nrm).
// mode 0 (start value): d = the summed partials B_j . g (j < nb); y = T^T d, c = y / n,
//   w = T c: the start value is sum_j w_j B_j.
// mode 1 (append vector nb): q = the summed partials S B_j . v (j < nb), vv = v . S v;
//   e = T^T q / n, column nb of T = -T e (diagonal 1), and n_nb = vv - sum_i e_i^2 n_i,
//   kept when finite and above 1e-20 n_0 (positive for nb = 0), else +inf.
constexpr int kSmallBlk = 1024;
__global__ __launch_bounds__(kSmallBlk) void k_pj_small(int G, int nb, int mode, const double* __restrict__ part,
                                                   double* __restrict__ T, double* __restrict__ nrm,
                                                   double* __restrict__ w) {
  __shared__ double tot[kProjPart], y[kProjMax], Ts[kProjMax * kProjMax], ns[kProjMax];
  const int m = mode == 0 ? nb : nb + 1;
  // T and the norms into LDS: the serial part below then reads no device memory
  for (int k = threadIdx.x; k < kProjMax * nb; k += blockDim.x)
    if (k % kProjMax < k / kProjMax) Ts[k] = T[k];  // T_ji, j < i: the part written and read
  for (int k = threadIdx.x; k < nb; k += blockDim.x) ns[k] = nrm[k];
  // column sums of the G x m partials (G <= kProjGrid): thread t sums column t % kProjPart
  // over the rows congruent to t / kProjPart modulo kRowGroups, all its loads issued at once
  // (clamped rows, masked sums), then the groups
  constexpr int kRowGroups = kSmallBlk / kProjPart, kRows = kProjGrid / kRowGroups;
  __shared__ double grp[kRowGroups][kProjPart];
  {
    const int col = threadIdx.x % kProjPart, r0 = threadIdx.x / kProjPart;
    double v[kRows], t = 0;
    if (col < m) {  // columns in use only (the others were never written)
#pragma unroll
      for (int u = 0; u < kRows; ++u) v[u] = part[(size_t)min(r0 + u * kRowGroups, G - 1) * kProjPart + col];
#pragma unroll
      for (int u = 0; u < kRows; ++u) t += r0 + u * kRowGroups < G ? v[u] : 0.0;
    }
    grp[r0][col] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < m) {
    double t = 0;
#pragma unroll
    for (int r = 0; r < kRowGroups; ++r) t += grp[r][threadIdx.x];
    tot[threadIdx.x] = t;
  }
  __syncthreads();
  // y_i = (T^T tot)_i / n_i (zero for dropped vectors): a thread per i
  const int t0 = threadIdx.x;
  if (t0 < nb) {
    double t = tot[t0];
    for (int j = 0; j < t0; ++j) t += Ts[j + kProjMax * t0] * tot[j];
    y[t0] = isfinite(ns[t0]) ? t / ns[t0] : 0.0;
  }
  __syncthreads();
  // (T y)_j: a thread per j; mode 0 returns it as w, mode 1 stores -(T y) as column nb of T
  if (t0 < nb) {
    double t = y[t0];
    for (int i = t0 + 1; i < nb; ++i) t += Ts[t0 + kProjMax * i] * y[i];
    if (mode == 0) w[t0] = t;
    else T[t0 + kProjMax * nb] = -t;
  }
  if (mode == 1 && t0 == 0) {
    double nn = tot[nb];
    for (int i = 0; i < nb; ++i)
      if (isfinite(ns[i])) nn -= y[i] * y[i] * ns[i];
    T[nb + kProjMax * nb] = 1.0;
    const double ref = nb > 0 && isfinite(ns[0]) ? 1e-20 * ns[0] : 0.0;
    nrm[nb] = (isfinite(nn) && nn > ref) ? nn : INFINITY;
  }
}

int pj_grid(long n) { return (int)std::min<long>(kProjGrid, (long)nblk(n, kBlk)); }

// Calls f(std::integral_constant<int, NB>) for NB = nb in [NB, kProjMax].
template <int NB, typename F>
static hipError_t pj_dispatch(int nb, F f) {
  if constexpr (NB > kProjMax) {
    return hipErrorInvalidValue;
  } else {
    if (nb == NB) return f(std::integral_constant<int, NB>{});
    return pj_dispatch<NB + 1>(nb, f);
  }
}

hipError_t launch_pj_dots(long n, int nb, const PjVecs& Y, const double* w, double* part, hipStream_t s) {
  return pj_dispatch<1>(nb, [&](auto c) {
    constexpr int NB = decltype(c)::value;
    hipLaunchKernelGGL((k_pj_dots<NB>), dim3(pj_grid(n)), dim3(kBlk), 0, s, n, Y, w, part);
    return hipGetLastError();
  });
}
hipError_t launch_pj_combine(long n, int nb, const PjVecs& B, const double* w, double* x, double* x0,
                             hipStream_t s) {
  return pj_dispatch<1>(nb, [&](auto c) {
    constexpr int NB = decltype(c)::value;
    hipLaunchKernelGGL((k_pj_combine<NB>), dim3(pj_grid(n)), dim3(kBlk), 0, s, n, B, w, x, x0);
    return hipGetLastError();
  });
}
hipError_t launch_pj_update(long n, int nb, const PjVecs& B, const PjVecs& SB, const double* w, const double* a,
                            const double* a0, const double* Sa, double* v, double* Sv, double* ca, double* cSa,
                            double* part, hipStream_t s) {
  if ((ca == nullptr) != (cSa == nullptr)) return hipErrorInvalidValue;
  return pj_dispatch<0>(nb, [&](auto c) {
    constexpr int NB = decltype(c)::value;
    if constexpr (NB >= kProjMax) {
      return hipErrorInvalidValue;  // the new vector takes slot NB
    } else {
      hipLaunchKernelGGL((k_pj_update<NB>), dim3(pj_grid(n)), dim3(kBlk), 0, s, n, B, SB, w, a, a0, Sa, v, Sv, ca,
                         cSa, part);
      return hipGetLastError();
    }
  });
}
hipError_t launch_pj_small(long n, int nb, int mode, const double* part, double* T, double* nrm, double* w,
                           hipStream_t s) {
  if (nb < 0 || nb > kProjMax || (mode == 1 && nb >= kProjMax) || (mode == 0 && nb < 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pj_small, dim3(1), dim3(kSmallBlk), 0, s, pj_grid(n), nb, mode, part, T, nrm, w);
  return hipGetLastError();
}


__global__ void k_extrapolate(long n, int order, HistPtrs h, double* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = extrapolate_at(order, [&](int j) { return h.p[j][i]; });
}

// One-step backtest of the orders 1..omax: squared error of the prediction of p[0] from
// p[1..o+1], one partial per block and order (grid-stride).
__global__ __launch_bounds__(kBlk) void k_extrap_backtest(long n, int omax, HistPtrs h, double* __restrict__ part) {
  double e[4] = {0, 0, 0, 0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double target = h.p[0][i];
#pragma unroll
    for (int o = 1; o <= 4; ++o)
      if (o <= omax) {
        const double d = extrapolate_at(o, [&](int j) { return h.p[j + 1][i]; }) - target;
        e[o - 1] += d * d;
      }
  }
  block_write_partial<4>(e, part);
}

// Extrapolation with the order of least backtest error (every block sums the partials in
// the same order, so all take the same decision; ties keep the lower order).
__global__ __launch_bounds__(kBlk) void k_extrapolate_pick(long n, int omax, HistPtrs h, const double* __restrict__ part,
                                                           int nparts, double* __restrict__ out) {
  double e[4];
  block_sum_partials<4>(part, nparts, e);
  int best = 1;
  for (int o = 2; o <= omax; ++o)
    if (e[o - 1] < e[best - 1]) best = o;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = extrapolate_at(best, [&](int j) { return h.p[j][i]; });
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------

// Events attached to the dispatch packet of the next single-kernel launch of the SpMV or
// the residual (kernel-only start and end times, for the measurement entry point).
static thread_local hipEvent_t t_ev0 = nullptr, t_ev1 = nullptr;
void set_dispatch_events(hipEvent_t start, hipEvent_t stop) {
  t_ev0 = start;
  t_ev1 = stop;
}
void get_dispatch_events(hipEvent_t* start, hipEvent_t* stop) {
  *start = t_ev0;
  *stop = t_ev1;
}
#define DFDG_LAUNCH_TIMED(KER, GRID, BLK, SH, S, ...)                                   \
  do {                                                                                  \
    if (t_ev0) hipExtLaunchKernelGGL(KER, GRID, BLK, SH, S, t_ev0, t_ev1, 0, __VA_ARGS__); \
    else hipLaunchKernelGGL(KER, GRID, BLK, SH, S, __VA_ARGS__);                        \
  } while (0)

#define DFDG_DISPATCH_K(K, ...)                                   \
  switch (K) {                                                    \
    case 1: { constexpr int KK = 1; __VA_ARGS__; } break;         \
    case 2: { constexpr int KK = 2; __VA_ARGS__; } break;         \
    case 3: { constexpr int KK = 3; __VA_ARGS__; } break;         \
    default: return hipErrorInvalidValue;                         \
  }

hipError_t launch_residual(int K, bool fp32, const DevGeo& g, const DevTabs& tb, const double* U, void* L,
                           double nu, hipStream_t s) {
  DFDG_DISPATCH_K(K, {
    const dim3 grid(nblk(g.T, kEBlk)), blk(kEBlk);
    if (nu != 0.0) {
      if (fp32) DFDG_LAUNCH_TIMED((k_residual<KK, float, true>), grid, blk, 0, s, g, tb, U, (float*)L, nu);
      else DFDG_LAUNCH_TIMED((k_residual<KK, double, true>), grid, blk, 0, s, g, tb, U, (double*)L, nu);
    } else {
      if (fp32) DFDG_LAUNCH_TIMED((k_residual<KK, float, false>), grid, blk, 0, s, g, tb, U, (float*)L, nu);
      else DFDG_LAUNCH_TIMED((k_residual<KK, double, false>), grid, blk, 0, s, g, tb, U, (double*)L, nu);
    }
  });
  return hipGetLastError();
}

hipError_t launch_residual_vjp(int K, const DevGeo& g, const DevTabs& tb, const double* U, const double* Lbar,
                               double* Ubar, double nu, hipStream_t s) {
  DFDG_DISPATCH_K(K, hipLaunchKernelGGL((k_residual_vjp<KK>), dim3(nblk(g.T, kEBlk)), dim3(kEBlk), 0, s, g, tb, U, Lbar,
                                        Ubar, nu));
  return hipGetLastError();
}

hipError_t launch_cond_rhs(int K, bool fp32in, const DevGeo& g, const DevTabs& tb, const void* F, double* q,
                           hipStream_t s) {
  // the reduced local space (g.G4 set) is one more template instance
  const dim3 gr(nblk(g.T, kEBlk)), bl(kEBlk);
  DFDG_DISPATCH_K(K, {
    if (g.G4) {
      if (fp32in) DFDG_LAUNCH_TIMED((k_cond_rhs<KK, float, true>), gr, bl, 0, s, g, tb, (const float*)F, q);
      else DFDG_LAUNCH_TIMED((k_cond_rhs<KK, double, true>), gr, bl, 0, s, g, tb, (const double*)F, q);
    } else {
      if (fp32in) DFDG_LAUNCH_TIMED((k_cond_rhs<KK, float, false>), gr, bl, 0, s, g, tb, (const float*)F, q);
      else DFDG_LAUNCH_TIMED((k_cond_rhs<KK, double, false>), gr, bl, 0, s, g, tb, (const double*)F, q);
    }
  });
  return hipGetLastError();
}

hipError_t launch_recover(int K, bool fp32in, const DevGeo& g, const DevTabs& tb, const void* F, const double* lam,
                          double* out, int mode, double a, const double* Un, double b, const double* Us, double dt,
                          hipStream_t s) {
  const dim3 gr(nblk(g.T, kEBlk)), bl(kEBlk);
  DFDG_DISPATCH_K(K, {
    if (g.G4) {
      if (fp32in)
        DFDG_LAUNCH_TIMED((k_recover<KK, float, true>), gr, bl, 0, s, g, tb, (const float*)F, lam, out, mode, a, Un, b,
                           Us, dt);
      else
        DFDG_LAUNCH_TIMED((k_recover<KK, double, true>), gr, bl, 0, s, g, tb, (const double*)F, lam, out, mode, a, Un,
                           b, Us, dt);
    } else {
      if (fp32in)
        DFDG_LAUNCH_TIMED((k_recover<KK, float, false>), gr, bl, 0, s, g, tb, (const float*)F, lam, out, mode, a, Un,
                           b, Us, dt);
      else
        DFDG_LAUNCH_TIMED((k_recover<KK, double, false>), gr, bl, 0, s, g, tb, (const double*)F, lam, out, mode, a, Un,
                           b, Us, dt);
    }
  });
  return hipGetLastError();
}

#define DFDG_DISPATCH_NF_VOID(NF, ...)                            \
  switch (NF) {                                                   \
    case 2: { constexpr int NN = 2; __VA_ARGS__; } break;         \
    case 3: { constexpr int NN = 3; __VA_ARGS__; } break;         \
    default: { constexpr int NN = 4; __VA_ARGS__; } break;        \
  }

#define DFDG_DISPATCH_NF(NF, ...)                                 \
  switch (NF) {                                                   \
    case 2: { constexpr int NN = 2; __VA_ARGS__; } break;         \
    case 3: { constexpr int NN = 3; __VA_ARGS__; } break;         \
    case 4: { constexpr int NN = 4; __VA_ARGS__; } break;         \
    case 6: { constexpr int NN = 6; __VA_ARGS__; } break;         \
    default: return hipErrorInvalidValue;                         \
  }

// (n_f, blocks per row) in a function returning void: triangles (2|3|4, 5), tetrahedra (3|6, 7)
#define DFDG_DISPATCH_NFS_VOID(NF, NS, ...)                                            \
  if ((NS) == kSlots3) {                                                               \
    if ((NF) == 3) { constexpr int NN = 3, SS = kSlots3; __VA_ARGS__; }                \
    else { constexpr int NN = 6, SS = kSlots3; __VA_ARGS__; }                          \
  } else {                                                                             \
    switch (NF) {                                                                      \
      case 2: { constexpr int NN = 2, SS = kSlots; __VA_ARGS__; } break;               \
      case 3: { constexpr int NN = 3, SS = kSlots; __VA_ARGS__; } break;               \
      default: { constexpr int NN = 4, SS = kSlots; __VA_ARGS__; } break;              \
    }                                                                                  \
  }

// (n_f, blocks per row): triangles (2|3|4, 5), tetrahedra (3|6, 7)
#define DFDG_DISPATCH_NFS(NF, NS, ...)                                                 \
  if ((NS) == kSlots3) {                                                               \
    switch (NF) {                                                                      \
      case 3: { constexpr int NN = 3, SS = kSlots3; __VA_ARGS__; } break;              \
      case 6: { constexpr int NN = 6, SS = kSlots3; __VA_ARGS__; } break;              \
      default: return hipErrorInvalidValue;                                            \
    }                                                                                  \
  } else {                                                                             \
    switch (NF) {                                                                      \
      case 2: { constexpr int NN = 2, SS = kSlots; __VA_ARGS__; } break;               \
      case 3: { constexpr int NN = 3, SS = kSlots; __VA_ARGS__; } break;               \
      case 4: { constexpr int NN = 4, SS = kSlots; __VA_ARGS__; } break;               \
      default: return hipErrorInvalidValue;                                            \
    }                                                                                  \
  }

hipError_t launch_gather_g(int NF, const DevGeo& g, const double* q, double* gv, const PcgBufs& pb, double rtol,
                           int maxit, hipStream_t s) {
  const int G = g.fgrid;
  DFDG_DISPATCH_NF(NF, hipLaunchKernelGGL((k_gather_g<NN>), dim3(G), dim3(kBlk), 0, s, g, q, gv, pb.gg));
  hipLaunchKernelGGL(k_finalize_gather, dim3(1), dim3(kBlk), 0, s, (const double*)pb.gg, G, pb.sc, rtol, maxit);
  return hipGetLastError();
}

hipError_t launch_deflate(int NF, const DevGeo& g, double* x, double* part, hipStream_t s) {
  const int G = g.fgrid;
  DFDG_DISPATCH_NF(NF, {
    hipLaunchKernelGGL((k_zdot<NN>), dim3(G), dim3(kBlk), 0, s, g, (const double*)x, part);
    hipLaunchKernelGGL((k_zdeflate<NN>), dim3(G), dim3(kBlk), 0, s, g, x, (const double*)part, G);
  });
  return hipGetLastError();
}

hipError_t launch_pcg_init(int NF, bool bj, const DevGeo& g, const DevBsr& A, const double* gv, double* x, double* r,
                           double* z, double* p_old, const PcgBufs& pb, hipStream_t s, bool deflate_start) {
  const int G = g.fgrid;
  // the start without its kernel component (a start far along it would leave a kernel
  // component of its rounding in r that no iteration removes; a combination of earlier,
  // deflated solutions has none to remove), then r and its deflation; the right-hand
  // side's partials in pb.gg are consumed by now and hold (z, .) partials
  if (deflate_start) {
    hipError_t e = launch_deflate(NF, g, x, pb.gg, s);
    if (e != hipSuccess) return e;
  }
  DFDG_DISPATCH_NFS(NF, A.ns, hipLaunchKernelGGL((k_pcg_init<NN, SS>), dim3(G), dim3(kBlk), 0, s, g, A, gv, x, r, z,
                                                 p_old, (const PcgScalars*)pb.sc, pb.gg));
  DFDG_DISPATCH_NF(NF, {
    if (bj) hipLaunchKernelGGL((k_pcg_init_defl<NN, true>), dim3(G), dim3(kBlk), 0, s, g, A, r, z, (const PcgScalars*)pb.sc, (const double*)pb.gg, pb.rz[0]);
    else hipLaunchKernelGGL((k_pcg_init_defl<NN, false>), dim3(G), dim3(kBlk), 0, s, g, A, r, z, (const PcgScalars*)pb.sc, (const double*)pb.gg, pb.rz[0]);
  });
  return hipGetLastError();
}

template <typename V>
static hipError_t spmv_any(int NF, const DevGeo& g, const DevBsr& A, const V* z, const V* p_old, V* p_new, V* Sp,
                           const PcgBufs& pb, int it, hipStream_t s) {
  const int G = g.fgrid;
  const double* prev = pb.rz[(it - 1) & 1];
  const double* prev2 = pb.rz[it & 1];
  if constexpr (sizeof(V) == 8) {
    if (A.mfq) return launch_mf_spmv3(NF, g, A, (const double*)z, (const double*)p_old, (double*)p_new, (double*)Sp, pb,
                                      it, s);
  }
  if (sizeof(V) == 4 && A.ns != kSlots) return hipErrorInvalidValue;  // FP32 copies: triangles only
  DFDG_DISPATCH_NFS(NF, A.ns, DFDG_LAUNCH_TIMED((k_pcg_spmv<NN, SS, V, V>), dim3(G), dim3(kBlk), 0, s, g, A, z, p_old,
                                                p_new, Sp, pb.sc, prev, prev2, pb.pq));
  return hipGetLastError();
}

template <typename V>
static hipError_t update_any(int NF, int pc, const DevGeo& g, const DevBsr& A, const V* p, const V* Sp, V* x, V* r,
                             V* z, const PcgBufs& pb, int it, hipStream_t s) {
  const int G = g.fgrid;
  // the entrywise form (point Jacobi, multigrid) reads and writes entry pairs
  const uintptr_t al = 2 * sizeof(V) - 1;
  if (pc != 1 && (((uintptr_t)p | (uintptr_t)Sp | (uintptr_t)x | (uintptr_t)r | (uintptr_t)z |
                   (uintptr_t)(sizeof(V) == 8 ? (const void*)A.dinv : (const void*)A.dinv32)) & al))
    return hipErrorInvalidValue;
  const double* prev = pb.rz[(it - 1) & 1];
  double* out = pb.rz[it & 1];
  DFDG_DISPATCH_NF(NF, {
    if (pc == 1) hipLaunchKernelGGL((k_pcg_update<NN, 1, V, V>), dim3(G), dim3(kBlk), 0, s, g, A, p, Sp, x, r, z, pb.sc, prev, (const double*)pb.pq, out);
    else if (pc == 2) hipLaunchKernelGGL((k_pcg_update<NN, 2, V, V>), dim3(G), dim3(kBlk), 0, s, g, A, p, Sp, x, r, z, pb.sc, prev, (const double*)pb.pq, out);
    else hipLaunchKernelGGL((k_pcg_update<NN, 0, V, V>), dim3(G), dim3(kBlk), 0, s, g, A, p, Sp, x, r, z, pb.sc, prev, (const double*)pb.pq, out);
  });
  return hipGetLastError();
}

hipError_t launch_pcg_spmv(int NF, const DevGeo& g, const DevBsr& A, const double* z, const double* p_old,
                           double* p_new, double* Sp, const PcgBufs& pb, int it, hipStream_t s) {
  return spmv_any<double>(NF, g, A, z, p_old, p_new, Sp, pb, it, s);
}
hipError_t launch_pcg_update(int NF, int pc, const DevGeo& g, const DevBsr& A, const double* p, const double* Sp,
                             double* x, double* r, double* z, const PcgBufs& pb, int it, hipStream_t s) {
  return update_any<double>(NF, pc, g, A, p, Sp, x, r, z, pb, it, s);
}
hipError_t launch_pcg32_spmv(int NF, const DevGeo& g, const DevBsr& A, const float* z, const float* p_old,
                             float* p_new, float* Sp, const PcgBufs& pb, int it, hipStream_t s) {
  return spmv_any<float>(NF, g, A, z, p_old, p_new, Sp, pb, it, s);
}
hipError_t launch_pcg32_update(int NF, int pc, const DevGeo& g, const DevBsr& A, const float* p, const float* Sp,
                               float* x, float* r, float* z, const PcgBufs& pb, int it, hipStream_t s) {
  return update_any<float>(NF, pc, g, A, p, Sp, x, r, z, pb, it, s);
}

hipError_t launch_pcg32_init(int NF, bool bj, const DevGeo& g, const DevBsr& A, const double* r64, float* x, float* r,
                             float* z, float* p_old, const PcgBufs& pb, hipStream_t s) {
  const int G = g.fgrid;
  DFDG_DISPATCH_NF(NF, {
    if (bj) hipLaunchKernelGGL((k_pcg32_init<NN, true>), dim3(G), dim3(kBlk), 0, s, g, A, r64, x, r, z, p_old, pb.rz[0]);
    else hipLaunchKernelGGL((k_pcg32_init<NN, false>), dim3(G), dim3(kBlk), 0, s, g, A, r64, x, r, z, p_old, pb.rz[0]);
  });
  return hipGetLastError();
}

hipError_t launch_ir_residual(int NF, const DevGeo& g, const DevBsr& A, const double* gv, double* lam,
                              const float* x32, int add, double* r64, const PcgBufs& pb64, PcgScalars* sc32,
                              double inner_rtol, int inner_maxit, hipStream_t s) {
  const int G = g.fgrid;
  if (add) {
    const long n = (long)g.E * NF;
    hipLaunchKernelGGL(k_add_f32, dim3(nblk(n, kBlk)), dim3(kBlk), 0, s, n, x32, lam);
  }
  DFDG_DISPATCH_NF(NF, hipLaunchKernelGGL((k_ir_residual<NN>), dim3(G), dim3(kBlk), 0, s, g, A, gv, lam, r64,
                                          (const PcgScalars*)pb64.sc, pb64.gg));
  hipLaunchKernelGGL(k_finalize_ir, dim3(1), dim3(kBlk), 0, s, (const double*)pb64.gg, G, pb64.sc, sc32, inner_rtol,
                     inner_maxit);
  return hipGetLastError();
}

int facet_grid_size(int E, int cap) {
  const int g = facet_grid(E);
  return (cap > 0 && cap < g) ? cap : g;
}

// ---- multigrid launchers -------------------------------------------------------------
#define DFDG_DISPATCH_LPR(L, ...)                                  \
  switch (L) {                                                     \
    case 1: { constexpr int LP = 1; __VA_ARGS__; } break;          \
    case 2: { constexpr int LP = 2; __VA_ARGS__; } break;          \
    case 4: { constexpr int LP = 4; __VA_ARGS__; } break;          \
    case 8: { constexpr int LP = 8; __VA_ARGS__; } break;          \
    case 16: { constexpr int LP = 16; __VA_ARGS__; } break;        \
    case 32: { constexpr int LP = 32; __VA_ARGS__; } break;        \
    default: { constexpr int LP = 64; __VA_ARGS__; } break;        \
  }

template <typename V>
static void csr_apply(const DevCsr& M, const V* x, const V* y0, V* y, int add, const PcgScalars* sc, hipStream_t s) {
  DFDG_DISPATCH_LPR(M.lpr, hipLaunchKernelGGL((k_csr_apply<LP, V>), dim3(nblk((long)M.n * LP, kBlk)), dim3(kBlk), 0, s,
                                              M, x, y0, y, add, sc));
}

// Everything of a cycle after the first pre-smoothing step (x2 = pre(b) already in v0.x).
template <typename V, typename VB>
static void vcycle_body(int NF, const DevGeo& g, const DevBsr& A, const MgDev& mg, const VB* b, VB* z, double* rz,
                        PcgScalars* sc, hipStream_t s) {
  const int G = g.fgrid;
  const int L = mg.nlev;
  const MgVec<V>& v0 = mg_vec<V>(mg, 0);
  DFDG_DISPATCH_NFS_VOID(NF, A.ns, hipLaunchKernelGGL((k_mg0_resid<NN, SS, V, VB>), dim3(G), dim3(kBlk), 0, s, g, A,
                                                       b, (const V*)v0.x, v0.r, sc));
  csr_apply<V>(mg.R[0], (const V*)v0.r, (const V*)nullptr, mg_vec<V>(mg, 1).b, 0, sc, s);
  for (int l = 1; l < L - 1; ++l) {
    const MgVec<V>& v = mg_vec<V>(mg, l);
    const DevCsr& R = mg.R[l];
    const DevCsr& RA = mg.RA[l];
    DFDG_DISPATCH_LPR(std::max(R.lpr, RA.lpr),
                      hipLaunchKernelGGL((k_mgc_restrict<LP, V>), dim3(nblk((long)R.n * LP, kBlk)), dim3(kBlk), 0, s, R,
                                         RA, (const V*)v.b, mg_dinv<V>(mg, l), mg.cheb[l], mg_vec<V>(mg, l + 1).b, sc));
  }
  {
    const MgVec<V>& vc = mg_vec<V>(mg, L - 1);
    hipLaunchKernelGGL((k_dense_mv<V>), dim3(nblk((long)mg.n_coarse * 64, kBlk)), dim3(kBlk), 0, s, mg.n_coarse,
                       mg.coarse_inv, mg.coarse_inv32, (const V*)vc.b, vc.z, sc);
  }
  for (int l = L - 2; l >= 1; --l) {
    const MgVec<V>& v = mg_vec<V>(mg, l);
    const DevCsr& Al = mg.A[l];
    const DevCsr& AP = mg.AP[l];
    const DevCsr& P = mg.P[l];
    DFDG_DISPATCH_LPR(std::max(Al.lpr, std::max(AP.lpr, P.lpr)),
                      hipLaunchKernelGGL((k_mgc_post<LP, V>), dim3(nblk((long)Al.n * LP, kBlk)), dim3(kBlk), 0, s, Al,
                                         AP, P, mg_dinv<V>(mg, l), (const V*)v.b, (const V*)mg_vec<V>(mg, l + 1).z, v.z,
                                         mg.cheb[l], sc));
  }
  csr_apply<V>(mg.P[0], (const V*)mg_vec<V>(mg, 1).z, (const V*)v0.x, v0.x, 1, sc, s);
  DFDG_DISPATCH_NFS_VOID(NF, A.ns, {
    hipLaunchKernelGGL((k_mg0_post1<NN, SS, V, VB>), dim3(G), dim3(kBlk), 0, s, g, A, b, (const V*)v0.x, v0.y, v0.d,
                       mg.cheb[0], sc);
    hipLaunchKernelGGL((k_mg0_post2<NN, SS, V, VB>), dim3(G), dim3(kBlk), 0, s, g, A, b, (const V*)v0.y,
                       (const V*)v0.d, z, mg.cheb[0], rz, sc);
  });
}

template <typename V, typename VB>
hipError_t launch_vcycle(int NF, const DevGeo& g, const DevBsr& A, const MgDev& mg, const VB* b, VB* z, double* rz,
                         PcgScalars* sc, hipStream_t s) {
  const int G = g.fgrid;
  const int L = mg.nlev;
  const MgVec<V>& v0 = mg_vec<V>(mg, 0);
  if (L == 1) {  // the facet matrix itself is the coarsest level: exact (regularised) solve in VB
    hipLaunchKernelGGL((k_dense_mv<VB>), dim3(nblk((long)mg.n_coarse * 64, kBlk)), dim3(kBlk), 0, s, mg.n_coarse,
                       mg.coarse_inv, mg.coarse_inv32, b, z, sc);
    hipLaunchKernelGGL((k_partial_dot<VB>), dim3(G), dim3(kBlk), 0, s, (long)g.E * NF, b, (const VB*)z, rz, sc);
    return hipGetLastError();
  }
  DFDG_DISPATCH_NFS(NF, A.ns, hipLaunchKernelGGL((k_mg0_pre<NN, SS, V, VB>), dim3(G), dim3(kBlk), 0, s, g, A, b,
                                                 v0.x, mg.cheb[0], sc));
  vcycle_body<V, VB>(NF, g, A, mg, b, z, rz, sc, s);
  return hipGetLastError();
}

// One PCG iteration with the multigrid preconditioner, residual double-buffered:
// spmv (p, S p), fused update + pre-smoothing, rest of the cycle (z, (r,z) partial).
template <typename V, typename VB>
hipError_t launch_pcg_iteration_mg(int NF, const DevGeo& g, const DevBsr& A, const MgDev& mg, const PcgBufs& pb,
                                   int it, const VB* z_in, const VB* p_old, VB* p_new, VB* Sp, VB* x,
                                   const VB* r_old, VB* r_new, VB* z, hipStream_t s) {
  const int G = g.fgrid;
  hipError_t e = spmv_any<VB>(NF, g, A, z_in, p_old, p_new, Sp, pb, it, s);
  if (e != hipSuccess) return e;
  const double* prev = pb.rz[(it - 1) & 1];
  double* out = pb.rz[it & 1];
  DFDG_DISPATCH_NFS(NF, A.ns, hipLaunchKernelGGL((k_pcg_upd_mg0_pre<NN, SS, V, VB>), dim3(G), dim3(kBlk), 0, s, g, A,
                                          (const VB*)p_new, (const VB*)Sp, x, r_old, r_new, mg_vec<V>(mg, 0).x,
                                          mg.cheb[0], pb.sc, prev, (const double*)pb.pq, out));
  vcycle_body<V, VB>(NF, g, A, mg, (const VB*)r_new, z, out, pb.sc, s);
  return hipGetLastError();
}
template hipError_t launch_pcg_iteration_mg<float, double>(int, const DevGeo&, const DevBsr&, const MgDev&,
                                                           const PcgBufs&, int, const double*, const double*, double*,
                                                           double*, double*, const double*, double*, double*,
                                                           hipStream_t);
template hipError_t launch_pcg_iteration_mg<double, double>(int, const DevGeo&, const DevBsr&, const MgDev&,
                                                            const PcgBufs&, int, const double*, const double*, double*,
                                                            double*, double*, const double*, double*, double*,
                                                            hipStream_t);
template hipError_t launch_pcg_iteration_mg<float, float>(int, const DevGeo&, const DevBsr&, const MgDev&,
                                                          const PcgBufs&, int, const float*, const float*, float*,
                                                          float*, float*, const float*, float*, float*, hipStream_t);

template hipError_t launch_vcycle<double, double>(int, const DevGeo&, const DevBsr&, const MgDev&, const double*,
                                                  double*, double*, PcgScalars*, hipStream_t);
template hipError_t launch_vcycle<float, double>(int, const DevGeo&, const DevBsr&, const MgDev&, const double*,
                                                 double*, double*, PcgScalars*, hipStream_t);
template hipError_t launch_vcycle<float, float>(int, const DevGeo&, const DevBsr&, const MgDev&, const float*, float*,
                                                double*, PcgScalars*, hipStream_t);


hipError_t launch_load_vector(int K, int nqp, const DevGeo& g, const DevTabs& tb, const double* fq, double* F,
                              hipStream_t s) {
  DFDG_DISPATCH_K(K, hipLaunchKernelGGL((k_load_vector<KK>), dim3(nblk(g.T, kEBlk)), dim3(kEBlk), 0, s, g, tb, nqp, fq, F));
  return hipGetLastError();
}

hipError_t launch_eval(int K, int npts, const DevGeo& g, const double* tab, const double* U, double* out,
                       hipStream_t s) {
  DFDG_DISPATCH_K(K, hipLaunchKernelGGL((k_eval<KK>), dim3(nblk(g.T, kEBlk)), dim3(kEBlk), 0, s, g, npts, tab, U, out));
  return hipGetLastError();
}

hipError_t launch_diag_finish(int nb, const double* partials, double* res, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(kBlk), 0, s, nb, partials, res);
  return hipGetLastError();
}

hipError_t launch_diagnostics(int K, const DevGeo& g, const DevTabs& tb, const double* U, double* partials,
                              double* res, hipStream_t s) {
  const unsigned nb = nblk(g.T, kEBlk);
  DFDG_DISPATCH_K(K, hipLaunchKernelGGL((k_diag<KK>), dim3(nb), dim3(kEBlk), 0, s, g, tb, U, partials));
  hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(kBlk), 0, s, (int)nb, partials, res);
  return hipGetLastError();
}

hipError_t launch_axpby(long n, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(nblk(n, kBlk)), dim3(kBlk), 0, s, n, a, x, b, y);
  return hipGetLastError();
}
__global__ void k_to_half(long n, const double* __restrict__ x, double scale, _Float16* __restrict__ out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = (_Float16)(float)(x[i] * scale);
}

__global__ void k_pack_half_pairs(int nv, int E, const double* __restrict__ vals, double scale,
                                  uint32_t* __restrict__ out, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long j = i / E, F = i % E;
    const _Float16 lo = (_Float16)(float)(vals[2 * j * E + F] * scale);
    const _Float16 hi = (2 * j + 1 < nv) ? (_Float16)(float)(vals[(2 * j + 1) * E + F] * scale) : (_Float16)0.0f;
    out[i] = (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
  }
}

// Packed rows of w = 4 ng entries (ng = 1..4): group g of row i is one 16-byte word (4 16-bit column ids,
// then the 4 values in FP16, scaled), entries 4g .. 4g+3 of the padded row.
__global__ void k_pack_rows(int n, int w, const int* __restrict__ col, const double* __restrict__ val,
                            double inv_scale, uint32_t* __restrict__ pk) {
  const long u = (long)blockIdx.x * blockDim.x + threadIdx.x;  // one group per thread
  const int ng = w >> 2;
  if (u >= (long)n * ng) return;
  const long e = 4 * u;  // the group's first entry in the padded row-major layout
  uint32_t q[4];
#pragma unroll
  for (int k = 0; k < 2; ++k)
    q[k] = (uint32_t)(col[e + 2 * k] & 0xffff) | ((uint32_t)(col[e + 2 * k + 1] & 0xffff) << 16);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const uint16_t lo = __builtin_bit_cast(uint16_t, (_Float16)(float)(val[e + 2 * k] * inv_scale));
    const uint16_t hi = __builtin_bit_cast(uint16_t, (_Float16)(float)(val[e + 2 * k + 1] * inv_scale));
    q[2 + k] = (uint32_t)lo | ((uint32_t)hi << 16);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) pk[4 * u + k] = q[k];
}

hipError_t launch_pack_rows(int n, int w, const int* col, const double* val, double inv_scale, uint32_t* pk,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (w % 4 != 0 || w < 4 || w > 16) return hipErrorInvalidValue;
  const long groups = (long)n * (w / 4);
  hipLaunchKernelGGL(k_pack_rows, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, s, n, w, col, val, inv_scale,
                     pk);
  return hipGetLastError();
}

hipError_t launch_to_half(long n, const double* x, double scale, uint16_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long nb = std::min<long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_to_half, dim3((unsigned)nb), dim3(256), 0, s, n, x, scale, reinterpret_cast<_Float16*>(out));
  return hipGetLastError();
}

hipError_t launch_pack_half_pairs(int NF, int ns, int E, const double* vals, double scale, uint32_t* out,
                                  hipStream_t s) {
  const long n = (long)nPairs(NF, ns) * E;
  const long nb = std::min<long>(nblk(n, 256), 65536);
  hipLaunchKernelGGL(k_pack_half_pairs, dim3((unsigned)nb), dim3(256), 0, s, ns * NF * NF, E, vals, scale, out, n);
  return hipGetLastError();
}
hipError_t launch_fill(long n, double v, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(nblk(n, kBlk)), dim3(kBlk), 0, s, n, v, y);
  return hipGetLastError();
}
hipError_t launch_extrapolate(long n, int order, const HistPtrs& h, double* out, hipStream_t s) {
  if (order < 0 || order >= kHistDepth) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_extrapolate, dim3(nblk(n, kBlk)), dim3(kBlk), 0, s, n, order, h, out);
  return hipGetLastError();
}
hipError_t launch_extrapolate_adaptive(long n, int omax, const HistPtrs& h, double* part, double* out,
                                       hipStream_t s) {
  if (omax < 1 || omax > 4 || omax > kHistDepth - 2) return hipErrorInvalidValue;
  const int G = (int)std::min<long>(nblk(n, kBlk), kExtrapParts / 4);
  hipLaunchKernelGGL(k_extrap_backtest, dim3(G), dim3(kBlk), 0, s, n, omax, h, part);
  hipLaunchKernelGGL(k_extrapolate_pick, dim3(G), dim3(kBlk), 0, s, n, omax, h, (const double*)part, G, out);
  return hipGetLastError();
}

// ---- allocation-free diagnostics ---------------------------------------------------------
// Scratch of dfdg_diagnostics_noalloc: the per-block partials [kNoAllocDiagBlocks][4] and the
// four results, in a file-scope device array (each GPU holds its own copy until the process
// ends).  In host code the array's name is a host-side stand-in, never a device address:
// kernels and copies get the address from hipGetSymbolAddress, looked up once per device.
static __device__ __align__(256) double scratch[4 * kNoAllocDiagBlocks + 4];

hipError_t noalloc_scratch(double** out) {
  static std::mutex mu;
  static double* ptr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[dev] = static_cast<double*>(p);
  }
  *out = ptr[dev];
  return hipSuccess;
}

int diag_blocks(int T) { return (int)nblk(T, kEBlk); }

}  // namespace dfdg
