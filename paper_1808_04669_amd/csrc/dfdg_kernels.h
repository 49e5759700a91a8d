// Launchers of the HIP kernels (implemented in dfdg_kernels.hip).  All launches are
// asynchronous on `stream`; every launcher checks nothing and returns the launch status.
#pragma once
#include <hip/hip_runtime_api.h>

#include "dfdg_internal.h"

namespace dfdg {

// Residual L(U) on the broken basis (a3).  Real = double (FP64) or float (MIXED, output
// in FP32).  U is always FP64.
hipError_t launch_residual(int K, bool fp32, const DevGeo& g, const DevTabs& tb, const double* U, void* L,
                           double nu, hipStream_t s);
// Residual VJP: Ubar = J_L(U)^T Lbar.
hipError_t launch_residual_vjp(int K, const DevGeo& g, const DevTabs& tb, const double* U, const double* Lbar,
                               double* Ubar, double nu, hipStream_t s);
// q[3][NF][T] = C_T W_T F_T per element and local facet (a4, element part).  F is FP64
// or FP32 (fp32in); q is written in FP64 or FP32 (fp32out).
hipError_t launch_cond_rhs(int K, bool fp32in, const DevGeo& g, const DevTabs& tb, const void* F, double* q,
                           hipStream_t s);
// Partial-sum buffers and scalars of one PCG run.  Every reducing kernel writes one
// partial per block; the following kernel sums them (no atomics, no fences).
struct PcgBufs {
  PcgScalars* sc;
  double* gg;      // [G][2] (g,g),(z,g) partials; reused for the FP64 refinement residual
  double* rz[2];   // [G][2] (r,z),(r,r) partials of even / odd iterations
  double* pq;      // [G][2] (p,Sp), (z,Sp) partials (z the normalised kernel vector of S)
};
// G: blocks of the facet kernels, ceil(E/256) up to 1024, or at most cap (> 0)
int facet_grid_size(int E, int cap);

// Multigrid hierarchy on the device (level 0 = the BSR facet matrix itself).
constexpr int kMaxLev = 16;
struct CheB { double th, c1, c2; };  // Chebyshev smoothing constants of a level
// Coarse-level sparse matrix in padded row-major (ELL) form: row i holds its entries at
// [i*w, i*w + w); the padding repeats a column of the row with value 0.  A fixed row
// width lets a kernel load columns and values at once, without first reading a row pointer.
struct DevCsr {
  int n;
  int lpr;  // lanes per row of the kernels that walk it (power of two <= 64)
  int w;    // entries per row (the longest row rounded up to a multiple of lpr)
  const int* col;
  const double* val;
  const float* val32;
  // rows of 4, 8, 12 or 16 entries (w) in an FP32 cycle with fewer than 65536 columns: one 16-byte
  // word per 4 entries of a row, 4 16-bit column ids then 4 FP16 values of val / pscale (or
  // null)
  const uint32_t* pk;
  float pscale;
  // FP16 values / pscale in the padded layout (the finest-level restriction of an FP32
  // cycle, rounded like the packed prolongation so that R = P^T holds exactly), or null
  const uint16_t* val16;
};
template <typename V>
struct MgVec { V *b, *x, *y, *d, *r, *z; };
struct MgDev {
  int nlev = 0;
  DevCsr A[kMaxLev];   // A[0] unused (the BSR facet matrix)
  DevCsr P[kMaxLev];   // prolongation from level l+1 to level l (rows: level l)
  DevCsr R[kMaxLev];   // restriction P^T
  DevCsr AP[kMaxLev];  // A P and R A on levels >= 1 (fused transfers; unused on level 0)
  DevCsr RA[kMaxLev];
  const double* dinv[kMaxLev];
  const float* dinv32[kMaxLev];
  CheB cheb[kMaxLev];
  MgVec<double> v64[kMaxLev];
  MgVec<float> v32[kMaxLev];
  int n_coarse = 0;
  const double* coarse_inv = nullptr;
  const float* coarse_inv32 = nullptr;
};
template <typename V>
inline const MgVec<V>& mg_vec(const MgDev& m, int l) {
  if constexpr (sizeof(V) == 8) return m.v64[l]; else return m.v32[l];
}
template <typename V>
inline const V* mg_dinv(const MgDev& m, int l) {
  if constexpr (sizeof(V) == 8) return m.dinv[l]; else return m.dinv32[l];
}
// z = V-cycle(b) (one smoothed-aggregation multigrid cycle run in type V on PCG vectors
// of type VB); writes the (b, z) partial of each facet block into rz[2*block].  Every
// kernel returns at once when sc->done says the PCG has stopped.
template <typename V, typename VB>
hipError_t launch_vcycle(int NF, const DevGeo& g, const DevBsr& A, const MgDev& mg, const VB* b, VB* z, double* rz,
                         PcgScalars* sc, hipStream_t s);
// One multigrid-preconditioned PCG iteration (needs at least two levels): p_new = z_in +
// beta p_old, Sp = S p_new; x += alpha p_new, r_new = r_old - alpha Sp fused with the
// first smoothing step; the rest of the cycle writes z = cycle(r_new) and its partials.
template <typename V, typename VB>
hipError_t launch_pcg_iteration_mg(int NF, const DevGeo& g, const DevBsr& A, const MgDev& mg, const PcgBufs& pb,
                                   int it, const VB* z_in, const VB* p_old, VB* p_new, VB* Sp, VB* x,
                                   const VB* r_old, VB* r_new, VB* z, hipStream_t s);

// g[E][NF] = facet sums of q, then (one block) the deflated (g,g) and the stopping
// threshold tol2 = rtol^2 (g,g) into pb.sc (done = RUNNING, or CONVERGED for g = 0).
// Start/stop events for the dispatch packet of the next SpMV or residual launch (kernel
// execution only; nullptr restores plain launches).
void set_dispatch_events(hipEvent_t start, hipEvent_t stop);
void get_dispatch_events(hipEvent_t* start, hipEvent_t* stop);
// Sum of the per-block diagnostics partials into res[4] (one block).
hipError_t launch_diag_finish(int nb, const double* partials, double* res, hipStream_t s);

// ---- tetrahedra (dfdg_kernels3.hip): the element steps; the facet kernels above are shared
// (DevBsr::ns = 7).  FP64 only, K = 1, 2.
hipError_t launch_residual_vjp3(int K, const DevGeo& g, const DevTabs& tb, const double* U, const double* Lbar,
                                double* Ubar, double nu, hipStream_t s);
hipError_t launch_residual3(int K, const DevGeo& g, const DevTabs& tb, const double* U, double* L, double nu,
                            hipStream_t s);
hipError_t launch_cond_rhs3(int K, const DevGeo& g, const DevTabs& tb, const double* F, double* q, hipStream_t s);
hipError_t launch_recover3(int K, const DevGeo& g, const DevTabs& tb, const double* F, const double* lam, double* out,
                           int mode, double a, const double* Un, double b, const double* Us, double dt, hipStream_t s);
hipError_t launch_load_vector3(int K, int nqp, const DevGeo& g, const DevTabs& tb, const double* fq, double* F,
                               hipStream_t s);
hipError_t launch_eval3(int K, int npts, const DevGeo& g, const double* tab, const double* U, double* out,
                        hipStream_t s);
hipError_t launch_diagnostics3(int K, const DevGeo& g, const DevTabs& tb, const double* U, double* partials,
                               double* res, hipStream_t s);
// The PCG product p_new = z + beta p_old, Sp = S p_new and its (p, Sp) partials, matrix free
// (A.mfq set): an element pass and a face pass (same role and arguments as launch_pcg_spmv).
hipError_t launch_mf_spmv3(int NF, const DevGeo& g, const DevBsr& A, const double* z, const double* p_old,
                           double* p_new, double* Sp, const PcgBufs& pb, int it, hipStream_t s);
// x_{.,0} -= (zdef, x_{.,0}) zdef (part: scratch for one partial per facet block).
hipError_t launch_deflate(int NF, const DevGeo& g, double* x, double* part, hipStream_t s);
hipError_t launch_gather_g(int NF, const DevGeo& g, const double* q, double* gv, const PcgBufs& pb, double rtol,
                           int maxit, hipStream_t s);
// r = g - zg zdef - S x, z = M^{-1} r, p_old = 0; partials of iteration 0.
hipError_t launch_pcg_init(int NF, bool block_jacobi, const DevGeo& g, const DevBsr& A, const double* gv, double* x,
                           double* r, double* z, double* p_old, const PcgBufs& pb, hipStream_t s, bool deflate_start = true);
// Iteration it >= 1: stopping test on iteration it-1, beta, p_new = z + beta p_old, Sp = S p_new.
// `it` selects the parity of the partial buffers (the kernels read the iteration count
// itself from pb.sc, so a captured launch sequence can be replayed).
hipError_t launch_pcg_spmv(int NF, const DevGeo& g, const DevBsr& A, const double* z, const double* p_old,
                           double* p_new, double* Sp, const PcgBufs& pb, int it, hipStream_t s);
// x += alpha p, r -= alpha Sp, z = M^{-1} r (pc: 0 Jacobi, 1 block Jacobi, 2 none).
hipError_t launch_pcg_update(int NF, int pc, const DevGeo& g, const DevBsr& A, const double* p,
                             const double* Sp, double* x, double* r, double* z, const PcgBufs& pb, int it,
                             hipStream_t s);
// FP32 inner PCG (MIXED): the same kernels on float vectors and the FP32 copy of S.
hipError_t launch_pcg32_init(int NF, bool block_jacobi, const DevGeo& g, const DevBsr& A, const double* r64,
                             float* x, float* r, float* z, float* p_old, const PcgBufs& pb, hipStream_t s);
hipError_t launch_pcg32_spmv(int NF, const DevGeo& g, const DevBsr& A, const float* z, const float* p_old,
                             float* p_new, float* Sp, const PcgBufs& pb, int it, hipStream_t s);
hipError_t launch_pcg32_update(int NF, int pc, const DevGeo& g, const DevBsr& A, const float* p,
                               const float* Sp, float* x, float* r, float* z, const PcgBufs& pb, int it,
                               hipStream_t s);
// FP64 refinement residual r64 = g - zg zdef - S lam (lam += x32 first if add), its norm
// into pb64.sc->rr, and the inner solve's threshold (inner_rtol relative to ||r64||) into sc32.
hipError_t launch_ir_residual(int NF, const DevGeo& g, const DevBsr& A, const double* gv, double* lam,
                              const float* x32, int add, double* r64, const PcgBufs& pb64, PcgScalars* sc32,
                              double inner_rtol, int inner_maxit, hipStream_t s);
// Recovery (a6): u = W_T (F_T - C_T^T lambda_T); out = u (mode 0) or
// out = a Un + b (Us + dt u) (mode 1).  F is FP64 or FP32.
hipError_t launch_recover(int K, bool fp32in, const DevGeo& g, const DevTabs& tb, const void* F, const double* lam,
                          double* out, int mode, double a, const double* Un, double b, const double* Us, double dt,
                          hipStream_t s);
hipError_t launch_load_vector(int K, int nqp, const DevGeo& g, const DevTabs& tb, const double* fq, double* F,
                              hipStream_t s);
hipError_t launch_eval(int K, int npts, const DevGeo& g, const double* tab, const double* U, double* out,
                       hipStream_t s);
// Diagnostics: per-block partials then a one-block finish into res[4].
hipError_t launch_diagnostics(int K, const DevGeo& g, const DevTabs& tb, const double* U, double* partials,
                              double* res, hipStream_t s);
// Linear combination y = a x + b y on n doubles.
hipError_t launch_axpby(long n, double a, const double* x, double b, double* y, hipStream_t s);
// Warm-start history: up to kHistDepth earlier multipliers, p[0] the newest.
constexpr int kHistDepth = 6;
constexpr int kExtrapAdaptive = 5;  // dfdg_params.extrapolate value of the adaptive choice
struct HistPtrs { const double* p[kHistDepth]; };
// out = extrapolation of order `order` (<= 4) in time from p[0..order].
hipError_t launch_extrapolate(long n, int order, const HistPtrs& h, double* out, hipStream_t s);
// out = extrapolation from p[0..o] with the order o in 1..omax (omax <= min(4, kHistDepth - 2))
// whose prediction of p[0] from p[1..o+1] has the smallest squared error; part: scratch
// for kExtrapParts doubles.
constexpr int kExtrapParts = 4 * 1024;
hipError_t launch_extrapolate_adaptive(long n, int omax, const HistPtrs& h, double* part, double* out,
                                       hipStream_t s);
hipError_t launch_fill(long n, double v, double* y, hipStream_t s);

// Start values projected onto earlier solutions: basis X = B T of stored vectors B_j with
// images S B_j, a unit upper triangular T (column-major, kProjMax x kProjMax) and S-norms
// squared nrm[i]; block partials in part[kProjGrid][kProjPart].
constexpr int kProjMax = 24;   // basis vectors kept
constexpr int kProjKeep = 8;   // latest solutions the basis is rebuilt from when full
constexpr int kProjGrid = 512;
constexpr int kProjPart = 32;  // >= kProjMax + 1
struct PjVecs { const double* p[kProjMax]; };
// part = block partials of Y_i . w, i < nb (1..kProjMax)
hipError_t launch_pj_dots(long n, int nb, const PjVecs& Y, const double* w, double* part, hipStream_t s);
// x = x0 = sum_i w_i B_i, i < nb (1..kProjMax)
hipError_t launch_pj_combine(long n, int nb, const PjVecs& B, const double* w, double* x, double* x0,
                             hipStream_t s);
// v = a - a0 (a0 given) or a - sum_i w_i B_i, Sv = Sa - sum_i w_i S B_i (i < nb <
// kProjMax); optional copies ca, cSa of a, Sa; partials S B_i . v (i < nb) and v . Sv (nb)
hipError_t launch_pj_update(long n, int nb, const PjVecs& B, const PjVecs& SB, const double* w, const double* a,
                            const double* a0, const double* Sa, double* v, double* Sv, double* ca, double* cSa,
                            double* part, hipStream_t s);
// the dense part: mode 0 start-value coefficients w from the partials B_j . g; mode 1
// column nb of T and nrm[nb] from the partials of launch_pj_update
hipError_t launch_pj_small(long n, int nb, int mode, const double* part, double* T, double* nrm, double* w,
                           hipStream_t s);
// pk[4i..4i+3] = row i of a 4-wide padded matrix packed as above (columns < 65536).
hipError_t launch_pack_rows(int n, int w, const int* col, const double* val, double inv_scale, uint32_t* pk,
                             hipStream_t s);
// out[i] = FP16 bits of x[i] * scale (round to nearest even).
hipError_t launch_to_half(long n, const double* x, double scale, uint16_t* out, hipStream_t s);
// S (FP64, [5][NF][NF][E]) times scale in FP16, two values per word (DevBsr::vals16)
hipError_t launch_pack_half_pairs(int NF, int ns, int E, const double* vals, double scale, uint32_t* out,
                                  hipStream_t s);

// Allocation-free diagnostics: a static device scratch of kNoAllocDiagBlocks partials (one per
// element block of the diagnostics kernel, i.e. meshes of up to 2097152 elements) plus the
// results.  noalloc_scratch gives its address on the current device (looked up once per
// device); diag_blocks(T) is the number of partials a mesh of T elements needs.
constexpr int kNoAllocDiagBlocks = 16384;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(double** out);
int diag_blocks(int T);

}  // namespace dfdg
